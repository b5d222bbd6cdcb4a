// Plan creation (tables prepared once per plan), argument checking, host
// Laguerre helpers and the thin C entry points of the hot-path calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "lg_internal.h"

// Staging area of lg_trace_synthesize_noalloc: the [nt][n] synthesis weights
// are copied here instead of into a per-call allocation.  One copy per GPU,
// held until the process ends; every call on a GPU shares it.
static __device__ __align__(256) double scratch[LG_TRACE_SCRATCH_MAX];

namespace lg {

namespace {
// device address of `scratch` on each GPU, looked up once per device (the
// host-side name of the array is not a device address)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Look up this device's copy of the staging array (device `dev` current).
lg_status scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LG_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] != nullptr) return LG_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (ptr == nullptr) return fail(LG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = (double*)ptr;
    return LG_OK;
}

double* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

lg_status fail(lg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

lg_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? LG_ERR_OOM : LG_ERR_HIP;
}

namespace {

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename P>
lg_status dev_alloc(lg_plan* pl, P** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc((void**)out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    pl->bytes_allocated += bytes;
    return LG_OK;
}

// upload a host FP64 array as the plan working type
lg_status upload_working(lg_plan* pl, void** dst, const std::vector<double>& h) {
    const size_t n = h.size();
    lg_status s = dev_alloc(pl, (char**)dst, n * wsize(pl));
    if (s != LG_OK) return s;
    if (pl->prec == LG_FP64) {
        LG_HIP(hipMemcpy(*dst, h.data(), n * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(n);
        for (size_t i = 0; i < n; ++i) f[i] = (float)h[i];
        LG_HIP(hipMemcpy(*dst, f.data(), n * 4, hipMemcpyHostToDevice));
    }
    return LG_OK;
}

double midrange(const double* a, size_t n) {
    double lo = a[0], hi = a[0];
    for (size_t i = 1; i < n; ++i) {
        lo = std::min(lo, a[i]);
        hi = std::max(hi, a[i]);
    }
    return 0.5 * (lo + hi);
}

// Solve tridiag(-c, diag, -c) x = e_col (size n) by the Thomas algorithm in
// long double (preparation only).
void toeplitz_unit_solve(long double diag, long double c, int n, int col, std::vector<long double>& x) {
    std::vector<long double> cp(n), dp(n);
    for (int i = 0; i < n; ++i) {
        const long double den = diag + (i ? c * cp[i - 1] : 0.0L);
        const long double rhs = (i == col) ? 1.0L : 0.0L;
        cp[i] = -c / den;
        dp[i] = (rhs + (i ? c * dp[i - 1] : 0.0L)) / den;
    }
    x.assign(n, 0.0L);
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

// Free-surface tables: per wavenumber, the normalised Dirichlet z-system is
// T_k = tridiag(-1, theta_k, -1) of size nz-1 and the flux-free top face
// makes it T_k - e1 e1^T.  Sherman-Morrison: (T - e1 e1^T)^{-1} r =
// T^{-1} r + g (e1^T T^{-1} r) / (1 - g_0), g = T^{-1} e1.  g (all rows) and
// 1 / (1 - g_0) are prepared here in long double.
lg_status prepare_free_surface(lg_plan* pl, const PrecBlock& B) {
    const int nx = pl->g.nx, nx1 = pl->nx1, nz1 = pl->nz1;
    const long double dx = pl->g.dx, dz = pl->g.dz;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> g((size_t)nz1 * nx1), t(nx1);
    std::vector<long double> col;
    for (int kk = 0; kk < nx1; ++kk) {
        const long double s = std::sin(pi * (kk + 1) / (2.0L * nx));
        const long double mu = 4.0L / (dx * dx) * s * s;
        const long double diag = 2.0L * B.kz / (dz * dz) + (long double)B.kx * mu + (long double)B.d;
        const long double theta = diag / ((long double)B.kz / (dz * dz));
        toeplitz_unit_solve(theta, 1.0L, nz1, 0, col);
        for (int j = 0; j < nz1; ++j) g[(size_t)j * nx1 + kk] = (double)col[j];
        t[kk] = (double)(1.0L / (1.0L - col[0]));
    }
    lg_status st = upload_working(pl, &pl->sm_g, g);
    if (st != LG_OK) return st;
    st = dev_alloc(pl, &pl->sm_t, (size_t)nx1 * 8);
    if (st != LG_OK) return st;
    LG_HIP(hipMemcpy(pl->sm_t, t.data(), (size_t)nx1 * 8, hipMemcpyHostToDevice));
    return dev_alloc(pl, &pl->sm_c, (size_t)pl->S * pl->C * nx1 * 8);
}

// Elastic traction-free surface tables of block c: with the surface on the
// first unknown row the normalised z-system becomes T_k - e1 e2^T (the
// surface row reads theta s_0 - 2 s_1).  Sherman-Morrison:
// (T - e1 e2^T)^{-1} r = y + g (e2^T y) / (1 - g_1), y = T^{-1} r,
// g = T^{-1} e1; g (all rows) and 1 / (1 - g_1) in long double.
lg_status prepare_surface_rows(lg_plan* pl, const PrecBlock& B, int c) {
    const int nx = pl->g.nx, nx1 = pl->nx1, nz1 = pl->nz1;
    const long double dx = pl->g.dx, dz = pl->g.dz;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> g((size_t)nz1 * nx1), t(nx1);
    std::vector<long double> col;
    for (int kk = 0; kk < nx1; ++kk) {
        const long double s = std::sin(pi * (kk + 1) / (2.0L * nx));
        const long double mu = 4.0L / (dx * dx) * s * s;
        const long double diag = 2.0L * B.kz / (dz * dz) + (long double)B.kx * mu + (long double)B.d;
        const long double theta = diag / ((long double)B.kz / (dz * dz));
        toeplitz_unit_solve(theta, 1.0L, nz1, 0, col);
        for (int j = 0; j < nz1; ++j) g[(size_t)j * nx1 + kk] = (double)col[j];
        t[kk] = nz1 >= 2 ? (double)(1.0L / (1.0L - col[1])) : 0.0;
    }
    lg_status st = upload_working(pl, &pl->es_g[c], g);
    if (st != LG_OK) return st;
    st = dev_alloc(pl, &pl->es_t[c], (size_t)nx1 * 8);
    if (st != LG_OK) return st;
    LG_HIP(hipMemcpy(pl->es_t[c], t.data(), (size_t)nx1 * 8, hipMemcpyHostToDevice));
    return LG_OK;
}

// 2.5D axisymmetric tables (Sec. 2.3, eq. precond1).  kap: node kappa
// [Nr][Nz].  Operator faces: a1 = rbar_j kappa_face / h_r^2 between rows j
// and j+1 (rbar_j = (j+1) h_r; the last face borders the Dirichlet row),
// a2 = r_j kappa_face / h_z^2 between columns k-1 and k (zero at both ends).
// Preconditioner: per z-wavenumber k the r-system with off-diagonals
// -rbar_j kappa~/h_r^2 and diagonal (A1_j + A1_{j-1} + r_j rho~ h^2/4 +
// r_j kappa~ lambda_k), lambda_k = (4/h_z^2) sin^2(pi k / (2 Nz)); its
// Dichotomy tables (segment factors, separator responses, reduced system)
// in long double.
lg_status prepare_cylindrical(lg_plan* pl, const double* kap) {
    const int nx = pl->g.nx, nz1 = pl->nz1, nx1 = pl->nx1;   // nx1 = Nz
    const long double hr = pl->g.dz, hz = pl->g.dx;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> a1((size_t)nz1 * nx1), a2((size_t)nz1 * (nx1 + 1), 0.0);
    for (int j = 0; j < nz1; ++j) {
        const long double r = (j + 0.5L) * hr, rbar = (j + 1.0L) * hr;
        for (int k = 0; k < nx1; ++k) {
            const long double kf = 0.5L * ((long double)kap[(size_t)j * nx + k] + kap[(size_t)(j + 1) * nx + k]);
            a1[(size_t)j * nx1 + k] = (double)(rbar * kf / (hr * hr));
            if (k > 0) {
                const long double kz = 0.5L * ((long double)kap[(size_t)j * nx + k - 1] + kap[(size_t)j * nx + k]);
                a2[(size_t)j * (nx1 + 1) + k] = (double)(r * kz / (hz * hz));
            }
        }
    }
    lg_status st = upload_working(pl, &pl->cy_a1, a1);
    if (st != LG_OK) return st;
    if ((st = upload_working(pl, &pl->cy_a2, a2)) != LG_OK) return st;
    if (pl->prec == LG_MIXED) {   // FP64 operator for the true residual
        if ((st = dev_alloc(pl, &pl->cy_a1_64, a1.size() * 8)) != LG_OK) return st;
        if ((st = dev_alloc(pl, &pl->cy_a2_64, a2.size() * 8)) != LG_OK) return st;
        LG_HIP(hipMemcpy(pl->cy_a1_64, a1.data(), a1.size() * 8, hipMemcpyHostToDevice));
        LG_HIP(hipMemcpy(pl->cy_a2_64, a2.data(), a2.size() * 8, hipMemcpyHostToDevice));
    }
    std::vector<double> ctw(2 * (size_t)nx1);
    for (int k = 0; k < nx1; ++k) {
        ctw[2 * k] = (double)std::cos(pi * k / (2.0L * nx1));
        ctw[2 * k + 1] = (double)(-std::sin(pi * k / (2.0L * nx1)));
    }
    if ((st = upload_working(pl, &pl->cy_ctw, ctw)) != LG_OK) return st;
    // r-systems by the Dichotomy: P segments of Ls-1 rows, separated by the
    // rows c_s = s Ls + Ls - 1 (s < P-1); n = nz1 = P Ls - 1.
    const int Ls = pl->blk[0].Ls, P = pl->blk[0].P;
    const long double kt = pl->kappa_t, dsh = (long double)pl->rho_t * pl->lag.h * pl->lag.h / 4.0L;
    std::vector<long double> A1(nz1), lo(nz1), up(nz1);
    for (int j = 0; j < nz1; ++j) A1[j] = (j + 1.0L) * hr * kt / (hr * hr);
    for (int j = 0; j < nz1; ++j) {
        lo[j] = (j > 0) ? -A1[j - 1] : 0.0L;          // coupling of row j to row j-1
        up[j] = (j + 1 < nz1) ? -A1[j] : 0.0L;        // coupling of row j to row j+1
    }
    std::vector<double> cp((size_t)nz1 * nx1, 0.0), inv((size_t)nz1 * nx1, 0.0), U((size_t)nz1 * nx1, 0.0),
        V((size_t)nz1 * nx1, 0.0), lowr(nz1), cpl64(2 * (size_t)nz1), red((size_t)nx1 * 3 * std::max(1, P - 1), 0.0);
    for (int j = 0; j < nz1; ++j) {
        lowr[j] = (double)lo[j];
        cpl64[j] = (double)lo[j];
        cpl64[nz1 + j] = (double)up[j];
    }
    std::vector<long double> d(nz1), c(Ls), w(Ls), Us(nz1), Vs(nz1);
    for (int k = 0; k < nx1; ++k) {
        const long double sn = std::sin(pi * k / (2.0L * nx1));
        const long double lam = 4.0L / (hz * hz) * sn * sn;
        for (int j = 0; j < nz1; ++j) {
            const long double r = (j + 0.5L) * hr;
            d[j] = A1[j] + (j > 0 ? A1[j - 1] : 0.0L) + r * dsh + r * kt * lam;
        }
        for (int sg = 0; sg < P; ++sg) {
            const int a = sg * Ls, b = a + Ls - 2, L = Ls - 1;
            // local Thomas factors of the segment (no coupling to its separators)
            long double cprev = 0.0L;
            for (int i = 0; i < L; ++i) {
                const int j = a + i;
                const long double den = d[j] - (i > 0 ? lo[j] * cprev : 0.0L);
                cprev = (i + 1 < L) ? up[j] / den : 0.0L;
                c[i] = cprev;
                w[i] = 1.0L / den;
                cp[(size_t)j * nx1 + k] = (double)cprev;
                inv[(size_t)j * nx1 + k] = (double)w[i];
            }
            // responses to the separator values: U = T_s^{-1}(-lo_a e_1), V = T_s^{-1}(-up_b e_L)
            auto solve = [&](int unit, long double val, std::vector<long double>& out) {
                long double dp = 0.0L;
                std::vector<long double> t(L);
                for (int i = 0; i < L; ++i) {
                    const int j = a + i;
                    const long double g = (i == unit ? val : 0.0L) - (i > 0 ? lo[j] * dp : 0.0L);
                    dp = g * w[i];
                    t[i] = dp;
                }
                long double x = 0.0L;
                for (int i = L - 1; i >= 0; --i) {
                    x = t[i] - c[i] * x;
                    out[a + i] = x;
                }
            };
            solve(0, -lo[a], Us);
            solve(L - 1, -up[b], Vs);
            for (int i = 0; i < L; ++i) {
                U[(size_t)(a + i) * nx1 + k] = (double)Us[a + i];
                V[(size_t)(a + i) * nx1 + k] = (double)Vs[a + i];
            }
        }
        // reduced (Schur) system over the separators, with its Thomas factors
        long double cR = 0.0L;
        for (int sg = 0; sg + 1 < P; ++sg) {
            const int cs = sg * Ls + Ls - 1, b = cs - 1, a1n = cs + 1;
            const long double al = lo[cs] * Us[b];
            const long double D = d[cs] + lo[cs] * Vs[b] + up[cs] * Us[a1n];
            const long double ga = up[cs] * Vs[a1n];
            const long double den = D - (sg > 0 ? al * cR : 0.0L);
            cR = ga / den;
            double* row = &red[(size_t)k * 3 * (P - 1) + 3 * sg];
            row[0] = (double)al;
            row[1] = (double)cR;
            row[2] = (double)(1.0L / den);
        }
    }
    if ((st = upload_working(pl, &pl->cy_cp, cp)) != LG_OK) return st;
    if ((st = upload_working(pl, &pl->cy_invden, inv)) != LG_OK) return st;
    if (P > 1) {   // the correction table, (U, V) pairs (zero for one segment)
        std::vector<double> uv(2 * U.size());
        for (size_t i = 0; i < U.size(); ++i) {
            uv[2 * i] = U[i];
            uv[2 * i + 1] = V[i];
        }
        if ((st = upload_working(pl, &pl->cy_UV, uv)) != LG_OK) return st;
    }
    if ((st = upload_working(pl, &pl->cy_lowr, lowr)) != LG_OK) return st;
    if ((st = dev_alloc(pl, &pl->cy_cpl64, cpl64.size() * 8)) != LG_OK) return st;
    LG_HIP(hipMemcpy(pl->cy_cpl64, cpl64.data(), cpl64.size() * 8, hipMemcpyHostToDevice));
    if ((st = dev_alloc(pl, &pl->cy_red, red.size() * 8)) != LG_OK) return st;
    LG_HIP(hipMemcpy(pl->cy_red, red.data(), red.size() * 8, hipMemcpyHostToDevice));
    return LG_OK;
}

// Face values of the fourth-order operator along one line of n+1 nodes
// k[0], k[s], ..., k[n s]: the cubic interpolant at the face midpoints
// (one-sided at the two end faces), or the two-point mean where it falls
// under half the smaller of the face's two nodes (keeps every face > 0).
static void faces4(const double* k, int n, size_t s, double* out) {
    for (int m = 0; m < n; ++m) {
        const double a = k[(size_t)m * s], b = k[(size_t)(m + 1) * s];
        double f = 0.5 * (a + b);
        if (n >= 3) {
            if (m == 0)
                f = (5.0 * a + 15.0 * b - 5.0 * k[2 * s] + k[3 * s]) / 16.0;
            else if (m == n - 1)
                f = (5.0 * b + 15.0 * a - 5.0 * k[(size_t)(n - 2) * s] + k[(size_t)(n - 3) * s]) / 16.0;
            else
                f = (9.0 * (a + b) - k[(size_t)(m - 1) * s] - k[(size_t)(m + 2) * s]) / 16.0;
            if (f < 0.5 * std::min(a, b)) f = 0.5 * (a + b);
        }
        out[m] = f;
    }
}

// Tables of the fourth-order operator (order 4): x-faces of the interior
// rows and z-faces of the interior columns, times 1/(24 h)^2.
lg_status prepare_order4(lg_plan* pl, const double* kap) {
    const int nx = pl->g.nx, nz = pl->g.nz;
    const double sx = 1.0 / (576.0 * pl->g.dx * pl->g.dx), sz = 1.0 / (576.0 * pl->g.dz * pl->g.dz);
    std::vector<double> kx((size_t)(nz - 1) * nx), kz((size_t)nz * (nx - 1)), line(std::max(nx, nz));
    for (int j = 1; j < nz; ++j) {
        faces4(kap + (size_t)j * (nx + 1), nx, 1, line.data());
        for (int m = 0; m < nx; ++m) kx[(size_t)(j - 1) * nx + m] = line[m] * sx;
    }
    for (int i = 1; i < nx; ++i) {
        faces4(kap + i, nz, (size_t)(nx + 1), line.data());
        for (int n = 0; n < nz; ++n) kz[(size_t)n * (nx - 1) + (i - 1)] = line[n] * sz;
    }
    lg_status st = upload_working(pl, &pl->ho_kx, kx);
    if (st != LG_OK) return st;
    if ((st = upload_working(pl, &pl->ho_kz, kz)) != LG_OK) return st;
    if (pl->prec == LG_MIXED) {
        if ((st = dev_alloc(pl, &pl->ho_kx64, kx.size() * 8)) != LG_OK) return st;
        if ((st = dev_alloc(pl, &pl->ho_kz64, kz.size() * 8)) != LG_OK) return st;
        LG_HIP(hipMemcpy(pl->ho_kx64, kx.data(), kx.size() * 8, hipMemcpyHostToDevice));
        LG_HIP(hipMemcpy(pl->ho_kz64, kz.data(), kz.size() * 8, hipMemcpyHostToDevice));
    }
    return LG_OK;
}

// Prepare the Dichotomy tables of one preconditioner block (done once).
lg_status prepare_block(lg_plan* pl, PrecBlock& B, double kx, double kz, double d, int P) {
    const int nx = pl->g.nx, nz = pl->g.nz, nx1 = pl->nx1;
    const long double dx = pl->g.dx, dz = pl->g.dz;
    B.kx = kx;
    B.kz = kz;
    B.d = d;
    B.b = (double)((long double)kz / (dz * dz));
    B.P = P;
    B.Ls = nz / P;
    B.q = ilog2(P);
    B.RW = 2 + B.q + (P - 1);
    const int Ls = B.Ls, L = Ls - 1, q = B.q;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> et((size_t)Ls * nx1, 0.0), ut((size_t)Ls * nx1, 0.0);
    std::vector<double> red((size_t)nx1 * B.RW, 0.0);
    std::vector<long double> e(Ls), u(Ls + 1), w;
    for (int kk = 0; kk < nx1; ++kk) {
        const int k = kk + 1;
        const long double s = std::sin(pi * k / (2.0L * nx));
        const long double mu = 4.0L / (dx * dx) * s * s;
        const long double diag = 2.0L * kz / (dz * dz) + (long double)kx * mu + (long double)d;
        const long double theta = diag / ((long double)kz / (dz * dz));
        // Thomas factors of the (Ls-1) interior block
        long double ep = 0.0L;
        for (int i = 1; i <= L; ++i) {
            ep = 1.0L / (theta - ep);
            e[i] = ep;
            et[(size_t)i * nx1 + kk] = (double)ep;
        }
        // end response u = T^{-1} e_1 (forward sweep of e_1, then back substitution)
        long double Ar = theta, Br = 1.0L;
        if (L >= 1) {
            std::vector<long double> dd(L + 2, 0.0L);
            long double prev = 0.0L;
            for (int i = 1; i <= L; ++i) {
                prev = ((i == 1 ? 1.0L : 0.0L) + prev) * e[i];
                dd[i] = prev;
            }
            u[L] = dd[L];
            for (int i = L - 1; i >= 1; --i) u[i] = dd[i] + e[i] * u[i + 1];
            for (int i = 1; i <= L; ++i) ut[(size_t)i * nx1 + kk] = (double)u[i];
            Ar = theta - 2.0L * u[1];
            Br = u[L];
        }
        double* row = &red[(size_t)kk * B.RW];
        row[0] = (double)Ar;
        row[1] = (double)Br;
        int woff = 2 + q;
        for (int l = 0; l < q; ++l) {
            const int size = P >> l, M = size - 1, c = size / 2 - 1;
            toeplitz_unit_solve(Ar, Br, M, c, w);   // middle row (= column) of the inverse
            for (int i = 0; i <= c; ++i) row[woff + i] = (double)w[i];
            row[2 + l] = (double)(Br * w[0]);
            woff += size >> 1;
        }
    }
    lg_status st = upload_working(pl, &B.etab, et);
    if (st != LG_OK) return st;
    st = upload_working(pl, &B.utab, ut);
    if (st != LG_OK) return st;
    st = dev_alloc(pl, &B.red, red.size() * 8);
    if (st != LG_OK) return st;
    LG_HIP(hipMemcpy(B.red, red.data(), red.size() * 8, hipMemcpyHostToDevice));
    return LG_OK;
}

void free_plan(lg_plan* p) {
    if (!p) return;
    pcg_release(p);
    void* ptrs[] = {p->kap, p->lam, p->mu, p->w, p->rho64, p->kap64, p->w64, p->tw, p->src_dev, p->r, p->p, p->qv,
                    p->rhat, p->y, p->E, p->partial, p->partial_pq, p->ctl, p->xslot, p->ahist, p->giter, p->gm_V,
                    p->gm_w, p->gm_z, p->gm_x, p->gm_dots, p->blk[0].etab, p->blk[0].utab,
                    p->blk[0].red, p->blk[1].etab, p->blk[1].utab, p->blk[1].red, p->sm_g, p->sm_t,
                    p->sm_c, p->cy_a1, p->cy_a2, p->cy_ctw, p->cy_cp, p->cy_invden, p->cy_lowr, p->cy_a1_64, p->cy_a2_64,
                    p->cy_UV, p->cy_cpl64, p->cy_red, p->es_g[0], p->es_g[1], p->es_t[0], p->es_t[1],
                    p->ho_kx, p->ho_kz, p->ho_kx64, p->ho_kz64};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p->ctl_host) (void)hipHostFree(p->ctl_host);
    if (p->gm_hb) (void)hipHostFree(p->gm_hb);
    for (hipEvent_t e : p->gm_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
}

lg_status check_vec(const void* p, const char* name) {
    if (p == nullptr) return fail(LG_ERR_INVALID_ARG, std::string(name) + " is NULL");
    return LG_OK;
}

#define LG_CHECK(expr)                    \
    do {                                  \
        lg_status _s = (expr);            \
        if (_s != LG_OK) return _s;       \
    } while (0)

lg_status check_plan(const lg_plan* p) {
    if (p == nullptr) return fail(LG_ERR_INVALID_ARG, "plan is NULL");
    return LG_OK;
}

// ---------------------------------------------------------------------------
// host Laguerre functions: psi_m(x) = n_m e^{-x/2} L_m^alpha(x), carried as
// mantissa * 2^exponent (three-term recurrence in m, normalised).
// ---------------------------------------------------------------------------
void psi_all(int n, long double x, int alpha, std::vector<long double>& mant,
             std::vector<long double>& ex) {
    mant.assign(n, 0.0L);
    ex.assign(n, 0.0L);
    const long double a = alpha;
    long double e = (-0.5L * x - 0.5L * std::lgamma(a + 1.0L)) / std::log(2.0L);
    long double p2 = 0.0L, p1 = 1.0L;
    mant[0] = 1.0L;
    ex[0] = e;
    if (n == 1) return;
    long double cur = (1.0L + a - x) / std::sqrt(1.0L + a);
    mant[1] = cur;
    ex[1] = e;
    p2 = p1;
    p1 = cur;
    const long double big = std::ldexp(1.0L, 500);
    for (int m = 2; m < n; ++m) {
        const long double mm = m;
        cur = ((2.0L * mm - 1.0L + a - x) * p1 - std::sqrt((mm - 1.0L) * (mm - 1.0L + a)) * p2) /
              std::sqrt(mm * (mm + a));
        if (std::fabs(cur) > big) {
            cur /= big;
            p1 /= big;
            e += 500.0L;
        }
        mant[m] = cur;
        ex[m] = e;
        p2 = p1;
        p1 = cur;
    }
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w) {
    x.resize(n);
    w.resize(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double pk = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

long double wavelet(lg_wavelet wv, long double t, double f0, double t0, double gamma) {
    const long double pi = 3.141592653589793238462643383279502884L;
    if (wv == LG_RICKER) {
        const long double a = (pi * f0 * (t - t0)) * (pi * f0 * (t - t0));
        return (1.0L - 2.0L * a) * std::exp(-a);
    }
    const long double s = 2.0L * pi * f0 * (t - t0);
    return std::exp(-(s * s) / ((long double)gamma * gamma)) * std::sin(s);
}

}  // namespace
}  // namespace lg

using namespace lg;

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

const char* lg_status_string(lg_status s) {
    switch (s) {
        case LG_OK: return "ok";
        case LG_ERR_INVALID_ARG: return "invalid argument";
        case LG_ERR_NOT_CONVERGED: return "not converged";
        case LG_ERR_BREAKDOWN: return "breakdown";
        case LG_ERR_NONFINITE: return "non-finite value";
        case LG_ERR_HIP: return "HIP error";
        case LG_ERR_OOM: return "out of device memory";
        case LG_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* lg_last_error(void) { return g_last_error.c_str(); }

lg_status lg_plan_create(lg_plan** out, lg_kind kind, const lg_grid* grid, const lg_laguerre* lag,
                         lg_precision prec, int32_t nshots, const double* medium_host,
                         const lg_tuning* tuning, void* hip_stream) {
    if (out == nullptr) return fail(LG_ERR_INVALID_ARG, "out is NULL");
    if (grid == nullptr || lag == nullptr || medium_host == nullptr)
        return fail(LG_ERR_INVALID_ARG, "grid, lag and medium_host must not be NULL");
    if (kind != LG_ACOUSTIC && kind != LG_ELASTIC) return fail(LG_ERR_INVALID_ARG, "bad kind");
    if (prec != LG_FP64 && prec != LG_MIXED) return fail(LG_ERR_INVALID_ARG, "bad precision");
    if (grid->nx < 2 || grid->nz < 2) return fail(LG_ERR_INVALID_ARG, "nx and nz must be >= 2");
    if (!finite_pos(grid->dx) || !finite_pos(grid->dz))
        return fail(LG_ERR_INVALID_ARG, "dx and dz must be finite and > 0");
    if (lag->alpha < 2) return fail(LG_ERR_INVALID_ARG, "alpha must be >= 2");
    if (!finite_pos(lag->h)) return fail(LG_ERR_INVALID_ARG, "h must be finite and > 0");
    if (lag->n < 1) return fail(LG_ERR_INVALID_ARG, "n must be >= 1");
    if (nshots < 1) return fail(LG_ERR_INVALID_ARG, "nshots must be >= 1");
    if (!is_pow2(grid->nx) || !is_pow2(grid->nz) || grid->nx > 4096 || grid->nz > 4096)
        return fail(LG_ERR_UNSUPPORTED, "nx and nz must be powers of two <= 4096");
    if (grid->top_bc != LG_TOP_DIRICHLET && grid->top_bc != LG_TOP_FREE)
        return fail(LG_ERR_INVALID_ARG, "top_bc must be LG_TOP_DIRICHLET or LG_TOP_FREE");

    if (grid->geometry != LG_CARTESIAN && grid->geometry != LG_CYLINDRICAL)
        return fail(LG_ERR_INVALID_ARG, "geometry must be LG_CARTESIAN or LG_CYLINDRICAL");
    const bool cyl = grid->geometry == LG_CYLINDRICAL;
    if (cyl && kind != LG_ACOUSTIC)
        return fail(LG_ERR_UNSUPPORTED, "the axisymmetric geometry is implemented for acoustic plans");
    if (grid->top_bc == LG_TOP_FREE && kind == LG_ELASTIC && (cyl || (grid->order != 0 && grid->order != 2)))
        return fail(LG_ERR_UNSUPPORTED, "the elastic traction-free surface is implemented for Cartesian "
                                        "second-order plans");
    if (grid->order != 0 && grid->order != 2 && grid->order != 4)
        return fail(LG_ERR_INVALID_ARG, "order must be 0, 2 or 4");
    if (grid->reserved != 0) return fail(LG_ERR_INVALID_ARG, "lg_grid.reserved must be 0");
    const int order = grid->order == 4 ? 4 : 2;
    if (order == 4 && (kind != LG_ACOUSTIC || cyl || grid->top_bc != LG_TOP_DIRICHLET))
        return fail(LG_ERR_UNSUPPORTED, "the fourth-order operator is implemented for Cartesian acoustic plans "
                                        "with Dirichlet sides");
    int P = 0, gi = 8, osh = 8, spw = 0, fus = 1, ring = 0;
    if (tuning != nullptr) {
        P = tuning->segments;
        if (tuning->graph_iters != 0) gi = tuning->graph_iters;
        if (tuning->op_shots != 0) osh = tuning->op_shots;
        spw = tuning->seg_per_wave;
        if (tuning->op_fusion != 0) fus = tuning->op_fusion;
        ring = tuning->x_ring;
        if (tuning->reserved[0] != 0 || tuning->reserved[1] != 0)
            return fail(LG_ERR_INVALID_ARG, "lg_tuning.reserved must be 0");
    }
    // held search directions: acoustic CG (every geometry and operator order)
    const bool ring_ok = kind == LG_ACOUSTIC;
    if (ring < 0 || ring > 64) return fail(LG_ERR_INVALID_ARG, "x_ring must be in 0..64");
    if (ring > 1 && !ring_ok)
        return fail(LG_ERR_UNSUPPORTED, "x_ring > 1 is implemented for acoustic plans");
    // a batch of CG iterations between flushes (graph_iters, or 8 without a
    // graph) must leave a free slot for the next direction
    const int batch = gi > 0 ? gi : 8;
    if (ring > 1 && ring <= batch) return fail(LG_ERR_INVALID_ARG, "x_ring must exceed graph_iters (8 without a graph)");
    if (fus != 1 && fus != 2) return fail(LG_ERR_INVALID_ARG, "op_fusion must be 0, 1 or 2");
    // default form: the FP64 axisymmetric update is register-bound with A p
    // recomputed (measured faster with the stored q)
    if ((tuning == nullptr || tuning->op_fusion == 0) && cyl && prec == LG_FP64) fus = 2;
    if (gi < -1 || gi == 0 || gi > 64) return fail(LG_ERR_INVALID_ARG, "graph_iters must be -1 or 1..64");
    if (osh < 1 || osh > 64) return fail(LG_ERR_INVALID_ARG, "op_shots must be in 1..64");
    if (spw != 0 && spw != 1 && spw != 2 && spw != 4)
        return fail(LG_ERR_INVALID_ARG, "seg_per_wave must be 0, 1, 2 or 4");
    // default segment counts: segments of 16 rows (z-systems), 64 rows
    // (r-systems of axisymmetric plans; below 128 rows one segment: Thomas)
    if (P == 0) P = cyl ? (grid->nz >= 128 ? std::min(64, grid->nz / 64) : 1) : std::max(1, std::min(64, grid->nz / 16));
    if (!(cyl && P == 1) && (!is_pow2(P) || P > 64 || grid->nz % P != 0 || grid->nz / P < 2 || grid->nz / P > 64))
        return fail(LG_ERR_INVALID_ARG, "segments must be a power of two <= 64 with nz/segments in 2..64");
    // one-dimensional launches map every element of a vector to a work-item,
    // and a grid dimension holds fewer than 2^32 work-items
    {
        const size_t C = (kind == LG_ACOUSTIC) ? 1 : 2;
        const size_t nvec = (size_t)nshots * C * (size_t)(cyl ? grid->nx : grid->nx - 1) * (size_t)(grid->nz - 1);
        if (nvec >= ((size_t)1 << 32))
            return fail(LG_ERR_UNSUPPORTED, "shots x components x interior points must be below 2^32");
    }
    const int F = (kind == LG_ACOUSTIC) ? 2 : 3;
    // node arrays: (nz+1)(nx+1) Cartesian nodes, or Nr x Nz axisymmetric nodes
    const size_t nn = cyl ? (size_t)grid->nx * grid->nz : (size_t)(grid->nx + 1) * (grid->nz + 1);
    for (size_t i = 0; i < (size_t)F * nn; ++i)
        if (!std::isfinite(medium_host[i])) return fail(LG_ERR_INVALID_ARG, "medium has a non-finite value");

    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
    {
        const lg_status ss = scratch_setup(dev);
        if (ss != LG_OK) return ss;
    }

    lg_plan* p = new lg_plan();
    p->kind = kind;
    p->g = *grid;
    p->lag = *lag;
    p->prec = prec;
    p->S = nshots;
    p->C = (kind == LG_ACOUSTIC) ? 1 : 2;
    p->cyl = cyl;
    p->nx1 = cyl ? grid->nx : grid->nx - 1;
    p->nz1 = grid->nz - 1;
    p->npts = (size_t)p->nx1 * p->nz1;
    p->nvec = (size_t)p->S * p->C * p->npts;
    p->graph_iters = gi;
    p->op_shots = osh;
    p->td_spw = spw;
    p->order = order;
    p->fuse_op = (fus == 1) && order == 2;
    if (ring == 0 && ring_ok) {
        // default: 16 held directions (32 for axisymmetric plans, whose solves
        // run two to three times longer: fewer flushes inside a phase), more
        // than a batch; fewer where the slots would pass 64 GiB, none where
        // fewer would not exceed a batch
        const size_t slot = p->nvec * (prec == LG_FP64 ? 8 : 4);
        ring = std::max(cyl ? 32 : 16, batch + 1);
        while (ring > batch + 1 && (size_t)ring * slot > ((size_t)64 << 30)) ring = std::max(batch + 1, ring / 2);
        if ((size_t)ring * slot > ((size_t)64 << 30) || ring < 4) ring = 1;
    }
    p->pring = std::max(1, ring);
    p->free_top = (grid->top_bc == LG_TOP_FREE) && !cyl && kind == LG_ACOUSTIC;
    p->el_free = (grid->top_bc == LG_TOP_FREE) && kind == LG_ELASTIC;
    p->src_scale = cyl ? 1.0 / (2.0 * 3.141592653589793 * grid->dx * grid->dz) : 1.0 / (grid->dx * grid->dz);
    p->device = dev;
    p->stream = (hipStream_t)hip_stream;

    auto bail = [&](lg_status s) {
        const std::string msg = g_last_error;
        free_plan(p);
        g_last_error = msg;
        return s;
    };

    const double hh4 = lag->h * lag->h / 4.0;
    std::vector<double> w_int(p->npts), rho_int(p->npts);
    const double* rho_node = medium_host + (size_t)(F - 1) * nn;
    for (int j = 0; j < p->nz1; ++j)
        for (int i = 0; i < p->nx1; ++i) {
            if (cyl) {   // the equation multiplied by r_j: w = r rho h^2/4, history weight r rho
                const double rj = (j + 0.5) * grid->dz;
                const double r = rho_node[(size_t)j * grid->nx + i];
                rho_int[(size_t)j * p->nx1 + i] = rj * r;
                w_int[(size_t)j * p->nx1 + i] = rj * r * hh4;
                continue;
            }
            const double r = rho_node[(size_t)(j + 1) * (grid->nx + 1) + (i + 1)];
            rho_int[(size_t)j * p->nx1 + i] = r;
            w_int[(size_t)j * p->nx1 + i] = r * hh4;
        }
    lg_status st;
    if ((st = upload_working(p, &p->w, w_int)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, &p->rho64, p->npts * 8)) != LG_OK) return bail(st);
    if ((he = hipMemcpy(p->rho64, rho_int.data(), p->npts * 8, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(he, "hipMemcpy"));

    if (cyl) {
        p->kappa_t = midrange(medium_host, nn);
        p->rho_t = midrange(rho_node, nn);
        if (!(p->kappa_t > 0.0) || !(p->rho_t >= 0.0))
            return bail(fail(LG_ERR_INVALID_ARG,
                             "midrange kappa must be > 0 and midrange rho >= 0 (SPD preconditioner)"));
        p->blk[0].P = P;
        p->blk[0].Ls = grid->nz / P;
        if ((st = prepare_cylindrical(p, medium_host)) != LG_OK) return bail(st);
        if (prec == LG_MIXED) {
            if ((st = dev_alloc(p, &p->w64, p->npts * 8)) != LG_OK) return bail(st);
            if ((he = hipMemcpy(p->w64, w_int.data(), p->npts * 8, hipMemcpyHostToDevice)) != hipSuccess)
                return bail(hip_fail(he, "hipMemcpy"));
        }
    } else if (kind == LG_ACOUSTIC) {
        std::vector<double> kap(medium_host, medium_host + nn);
        if ((st = upload_working(p, &p->kap, kap)) != LG_OK) return bail(st);
        if (prec == LG_MIXED) {   // FP64 medium for the true residual of the refinement
            if ((st = dev_alloc(p, &p->kap64, nn * 8)) != LG_OK) return bail(st);
            if ((st = dev_alloc(p, &p->w64, p->npts * 8)) != LG_OK) return bail(st);
            if ((he = hipMemcpy(p->kap64, kap.data(), nn * 8, hipMemcpyHostToDevice)) != hipSuccess)
                return bail(hip_fail(he, "hipMemcpy"));
            if ((he = hipMemcpy(p->w64, w_int.data(), p->npts * 8, hipMemcpyHostToDevice)) != hipSuccess)
                return bail(hip_fail(he, "hipMemcpy"));
        }
        p->kappa_t = midrange(medium_host, nn);
        p->rho_t = midrange(rho_node, nn);
        if (!(p->kappa_t > 0.0) || !(p->rho_t >= 0.0))
            return bail(fail(LG_ERR_INVALID_ARG,
                             "midrange kappa must be > 0 and midrange rho >= 0 (SPD preconditioner)"));
        if ((st = prepare_block(p, p->blk[0], p->kappa_t, p->kappa_t, p->rho_t * hh4, P)) != LG_OK)
            return bail(st);
        if (p->free_top && (st = prepare_free_surface(p, p->blk[0])) != LG_OK) return bail(st);
        if (order == 4 && (st = prepare_order4(p, medium_host)) != LG_OK) return bail(st);
    } else {
        const double* lam = medium_host;
        const double* mu = medium_host + nn;
        std::vector<double> lv(lam, lam + nn), mv(mu, mu + nn), lp2m(nn);
        for (size_t i = 0; i < nn; ++i) lp2m[i] = lam[i] + 2.0 * mu[i];
        if ((st = upload_working(p, &p->lam, lv)) != LG_OK) return bail(st);
        if ((st = upload_working(p, &p->mu, mv)) != LG_OK) return bail(st);
        p->lp2m_t = midrange(lp2m.data(), nn);
        p->mu_t = midrange(mu, nn);
        p->rho_t = midrange(rho_node, nn);
        if (!(p->lp2m_t > 0.0) || !(p->mu_t > 0.0) || !(p->rho_t >= 0.0))
            return bail(fail(LG_ERR_INVALID_ARG, "midrange lambda+2mu, mu must be > 0, rho >= 0"));
        if ((st = prepare_block(p, p->blk[0], p->lp2m_t, p->mu_t, p->rho_t * hh4, P)) != LG_OK)
            return bail(st);
        if ((st = prepare_block(p, p->blk[1], p->mu_t, p->lp2m_t, p->rho_t * hh4, P)) != LG_OK)
            return bail(st);
        if (p->el_free) {
            for (int c = 0; c < 2; ++c)
                if ((st = prepare_surface_rows(p, p->blk[c], c)) != LG_OK) return bail(st);
            if ((st = dev_alloc(p, &p->sm_c, (size_t)p->S * p->C * p->nx1 * 8)) != LG_OK) return bail(st);
        }
    }

    // FFT twiddles for length M = 2 nx
    {
        const int M = 2 * grid->nx;
        const long double pi = 3.141592653589793238462643383279502884L;
        std::vector<double> tw(2 * (size_t)M);
        for (int j = 0; j < M; ++j) {
            tw[2 * j] = (double)std::cos(2.0L * pi * j / M);
            tw[2 * j + 1] = (double)(-std::sin(2.0L * pi * j / M));
        }
        if ((st = upload_working(p, &p->tw, tw)) != LG_OK) return bail(st);
    }

    // sources default to the centre of the second row
    p->src_host.assign(2 * (size_t)p->S, 0);
    for (int s = 0; s < p->S; ++s) {
        p->src_host[2 * s] = std::max(1, grid->nx / 2);
        p->src_host[2 * s + 1] = 1;
    }

    // Krylov workspace
    const size_t ws = wsize(p);
    const int SC = p->S * p->C;
    if ((st = dev_alloc(p, &p->r, p->nvec * 8)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, (char**)&p->p, (size_t)p->pring * p->nvec * ws)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, &p->ahist, (size_t)SC * p->pring * 8)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, (char**)&p->giter, 2 * sizeof(int))) != LG_OK) return bail(st);
    if ((he = hipMemset(p->giter, 0, 2 * sizeof(int))) != hipSuccess) return bail(hip_fail(he, "hipMemset"));
    if ((st = dev_alloc(p, (char**)&p->qv, p->nvec * ws)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, (char**)&p->rhat, p->nvec * ws)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, (char**)&p->y, p->nvec * ws)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, &p->E, (size_t)SC * P * 3 * p->nx1 * 8)) != LG_OK) return bail(st);
    {
        const size_t sb = (size_t)((p->nx1 + 63) / 64) * ((p->nz1 + 15) / 16);   // operator tiles (<= 16 rows)
        const size_t db = (size_t)dst_blocks_per_field(grid->nx, p->nz1, (int)wsize(p));
        const size_t rb = (size_t)((p->nx1 + 15) / 16);
        // the transform kernel's start from a given x writes two partial sets
        p->partial_stride = std::max(sb, std::max(2 * db, rb));
    }
    if ((st = dev_alloc(p, &p->partial, (size_t)SC * p->partial_stride * 8)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, &p->partial_pq, (size_t)SC * p->partial_stride * 8)) != LG_OK) return bail(st);
    if ((st = dev_alloc(p, &p->ctl, (size_t)SC * sizeof(ShotCtl))) != LG_OK) return bail(st);
    if ((he = hipMemset(p->ctl, 0, (size_t)SC * sizeof(ShotCtl))) != hipSuccess)
        return bail(hip_fail(he, "hipMemset"));
    if ((he = hipHostMalloc((void**)&p->ctl_host, (size_t)SC * sizeof(ShotCtl), hipHostMallocDefault)) !=
        hipSuccess)
        return bail(hip_fail(he, "hipHostMalloc"));
    if ((st = dev_alloc(p, &p->xslot, 2 * sizeof(double*))) != LG_OK) return bail(st);
    if ((he = hipDeviceSynchronize()) != hipSuccess) return bail(hip_fail(he, "hipDeviceSynchronize"));
    *out = p;
    return LG_OK;
}

lg_status lg_plan_destroy(lg_plan* plan) {
    LG_CHECK(check_plan(plan));
    (void)hipStreamSynchronize(plan->stream);
    free_plan(plan);
    return LG_OK;
}

lg_status lg_plan_set_stream(lg_plan* plan, void* hip_stream) {
    LG_CHECK(check_plan(plan));
    plan->stream = (hipStream_t)hip_stream;
    return LG_OK;
}

lg_status lg_plan_set_sources(lg_plan* plan, const int32_t* src) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(src, "src_ij_host"));
    for (int s = 0; s < plan->S; ++s) {
        const int i = src[2 * s], j = src[2 * s + 1];
        if (i < 1 || i > plan->nx1 || j < 1 || j > plan->nz1)
            return fail(LG_ERR_INVALID_ARG, "source node outside the interior");
    }
    plan->src_host.assign(src, src + 2 * (size_t)plan->S);
    return LG_OK;
}

lg_status lg_plan_layout(const lg_plan* plan, int32_t* segments, int32_t* seg_len) {
    LG_CHECK(check_plan(plan));
    if (segments) *segments = plan->blk[0].P;
    if (seg_len) *seg_len = plan->blk[0].Ls;
    return LG_OK;
}

lg_status lg_plan_x_ring(const lg_plan* plan, int32_t* x_ring) {
    LG_CHECK(check_plan(plan));
    if (x_ring == nullptr) return fail(LG_ERR_INVALID_ARG, "NULL argument");
    *x_ring = plan->pring;
    return LG_OK;
}

lg_status lg_source_coeffs(lg_wavelet wv, double f0, double t0, double gamma, const lg_laguerre* lag,
                           double* f_m_host) {
    if (lag == nullptr || f_m_host == nullptr) return fail(LG_ERR_INVALID_ARG, "NULL argument");
    if (wv != LG_RICKER && wv != LG_GAUSS_SINE) return fail(LG_ERR_INVALID_ARG, "bad wavelet");
    if (lag->alpha < 2 || !finite_pos(lag->h) || lag->n < 1)
        return fail(LG_ERR_INVALID_ARG, "bad Laguerre parameters");
    if (!finite_pos(f0) || !std::isfinite(t0) || t0 < 0.0)
        return fail(LG_ERR_INVALID_ARG, "f0 must be > 0 and t0 >= 0");
    if (wv == LG_GAUSS_SINE && !finite_pos(gamma)) return fail(LG_ERR_INVALID_ARG, "gamma must be > 0");
    const int n = lag->n;
    const long double h = lag->h;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double t_end =
        (wv == LG_RICKER) ? t0 + 8.0L / f0 : t0 + 8.0L * gamma / (2.0L * pi * f0);
    std::vector<long double> xg, wg;
    gauss_legendre(32, xg, wg);
    std::vector<long double> mant, ex, acc(n), prev(n);
    auto integrate = [&](int panels) {
        std::fill(acc.begin(), acc.end(), 0.0L);
        const long double wdt = t_end / panels;
        for (int pnl = 0; pnl < panels; ++pnl) {
            const long double mid = (pnl + 0.5L) * wdt, half = 0.5L * wdt;
            for (int g = 0; g < 32; ++g) {
                const long double t = mid + half * xg[g];
                const long double fw = wavelet(wv, t, f0, t0, gamma) * half * wg[g];
                if (fw == 0.0L) continue;
                psi_all(n, h * t, lag->alpha, mant, ex);
                for (int m = 0; m < n; ++m) acc[m] += fw * mant[m] * std::exp2(ex[m]);
            }
        }
        for (int m = 0; m < n; ++m) acc[m] *= std::sqrt(h);
    };
    int panels = 8;
    integrate(panels);
    prev = acc;
    while (panels < 4096) {
        panels *= 2;
        integrate(panels);
        long double dmax = 0.0L, amax = 0.0L;
        for (int m = 0; m < n; ++m) {
            dmax = std::max(dmax, std::fabs(acc[m] - prev[m]));
            amax = std::max(amax, std::fabs(acc[m]));
        }
        prev = acc;
        if (dmax <= 1e-14L * amax) break;
    }
    for (int m = 0; m < n; ++m) f_m_host[m] = (double)acc[m];
    return LG_OK;
}

lg_status lg_laguerre_weights(const lg_laguerre* lag, const double* t_host, int32_t nt, double* W_host) {
    if (lag == nullptr || t_host == nullptr || W_host == nullptr)
        return fail(LG_ERR_INVALID_ARG, "NULL argument");
    if (lag->alpha < 2 || !finite_pos(lag->h) || lag->n < 1 || nt < 0)
        return fail(LG_ERR_INVALID_ARG, "bad Laguerre parameters");
    const int n = lag->n;
    std::vector<long double> mant, ex;
    for (int q = 0; q < nt; ++q) {
        const double t = t_host[q];
        if (!std::isfinite(t) || t < 0.0) return fail(LG_ERR_INVALID_ARG, "times must be finite and >= 0");
    }
    for (int q = 0; q < nt; ++q) {
        const long double x = (long double)lag->h * t_host[q];
        double* row = W_host + (size_t)q * n;
        if (x <= 0.0L) {
            for (int m = 0; m < n; ++m) row[m] = 0.0;
            continue;
        }
        psi_all(n, x, lag->alpha, mant, ex);
        const long double lg2 = 0.5L * std::log2((long double)lag->h) + lag->alpha * std::log2(x);
        for (int m = 0; m < n; ++m) row[m] = (double)(mant[m] * std::exp2(ex[m] + lg2));
    }
    return LG_OK;
}

lg_status lg_laguerre_rhs(lg_plan* plan, int32_t m, const double* R_prev, double* Phat, double* Qhat,
                          const double* fsrc_host, double* rhs) {
    LG_CHECK(check_plan(plan));
    if (m < 0) return fail(LG_ERR_INVALID_ARG, "m must be >= 0");
    if (m > 0) LG_CHECK(check_vec(R_prev, "R_prev"));
    LG_CHECK(check_vec(Phat, "Phat"));
    LG_CHECK(check_vec(Qhat, "Qhat"));
    LG_CHECK(check_vec(fsrc_host, "fsrc_host"));
    LG_CHECK(check_vec(rhs, "rhs"));
    LG_HIP(hipSetDevice(plan->device));
    LG_HIP(launch_rhs(plan, m, R_prev, Phat, Qhat, fsrc_host, rhs));
    return LG_OK;
}

lg_status lg_stencil_apply(lg_plan* plan, const void* x, void* y) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(x, "x"));
    LG_CHECK(check_vec(y, "y"));
    if (x == y) return fail(LG_ERR_INVALID_ARG, "x and y must differ");
    LG_HIP(hipSetDevice(plan->device));
    if (plan->kind == LG_ELASTIC) {
        LG_HIP(launch_elastic_stencil(plan, x, y));
        return LG_OK;
    }
    LG_HIP(launch_stencil(plan, x, y, false));
    return LG_OK;
}

lg_status lg_precond_dst(lg_plan* plan, int32_t inverse, const void* in, void* out) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(in, "in"));
    LG_CHECK(check_vec(out, "out"));
    if (in == out) return fail(LG_ERR_INVALID_ARG, "in and out must differ");
    LG_HIP(hipSetDevice(plan->device));
    LG_HIP(launch_dst(plan, inverse ? 1 : 0, in, out, plan->S * plan->C));
    return LG_OK;
}

lg_status lg_precond_dichotomy_tdma(lg_plan* plan, int32_t block, const void* rhs_hat, void* sol_hat) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(rhs_hat, "rhs_hat"));
    LG_CHECK(check_vec(sol_hat, "sol_hat"));
    if (rhs_hat == sol_hat) return fail(LG_ERR_INVALID_ARG, "rhs_hat and sol_hat must differ");
    int bi;
    if (plan->kind == LG_ACOUSTIC) {
        if (block != 0) return fail(LG_ERR_INVALID_ARG, "acoustic plans have block 0 only");
        bi = 0;
    } else {
        if (block != 1 && block != 2) return fail(LG_ERR_INVALID_ARG, "elastic plans have blocks 1, 2");
        bi = block - 1;
    }
    LG_HIP(hipSetDevice(plan->device));
    const int nf = plan->S;   // acoustic: S fields; elastic: one component per shot
    if (plan->cyl) {          // non-Toeplitz r-systems, one per z-wavenumber
        LG_HIP(cyl_launch_rsys(plan, rhs_hat, sol_hat, nf, 0));
        if (plan->blk[0].P > 1) LG_HIP(cyl_launch_corr(plan, sol_hat, nf));
        return LG_OK;
    }
    LG_HIP(launch_td(plan, bi, rhs_hat, sol_hat, nf, 0));
    if (plan->blk[bi].P > 1 || plan->free_top) {
        LG_HIP(launch_rs(plan, bi, rhs_hat, sol_hat, nf, 0));
        LG_HIP(launch_correct(plan, bi, sol_hat, nf));
    }
    if (plan->el_free) LG_HIP(launch_surface_rows(plan, bi, sol_hat, nf, 1, 0));
    return LG_OK;
}

lg_status lg_laguerre_synthesize(lg_plan* plan, int32_t m, const double* R_m, const double* W_snap_host,
                                 int32_t n_snap, double* snap_accum, int32_t rec_row, double* rec_coeff) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(R_m, "R_m"));
    if (m < 0 || m >= plan->lag.n) return fail(LG_ERR_INVALID_ARG, "m out of range");
    if (n_snap < 0 || n_snap > 8) return fail(LG_ERR_INVALID_ARG, "n_snap must be in 0..8");
    if (n_snap > 0) {
        LG_CHECK(check_vec(W_snap_host, "W_snap_host"));
        LG_CHECK(check_vec(snap_accum, "snap_accum"));
    }
    if (rec_coeff != nullptr && (rec_row < 1 || rec_row > plan->nz1))
        return fail(LG_ERR_INVALID_ARG, "rec_row out of range");
    LG_HIP(hipSetDevice(plan->device));
    LG_HIP(launch_synth(plan, m, 1, &R_m, W_snap_host, n_snap, snap_accum, rec_row, rec_coeff));
    return LG_OK;
}

lg_status lg_laguerre_synthesize_batch(lg_plan* plan, int32_t m0, int32_t nb, const double* const* R_host,
                                       const double* W_snap_host, int32_t n_snap, double* snap_accum,
                                       int32_t rec_row, double* rec_coeff) {
    LG_CHECK(check_plan(plan));
    if (nb < 1 || nb > LG_SYNTH_BATCH_MAX) return fail(LG_ERR_INVALID_ARG, "nb must be in 1..8");
    LG_CHECK(check_vec(R_host, "R_host"));
    for (int b = 0; b < nb; ++b) LG_CHECK(check_vec(R_host[b], "R_host[b]"));
    if (m0 < 0 || m0 > plan->lag.n - nb) return fail(LG_ERR_INVALID_ARG, "harmonics m0 .. m0+nb-1 out of range");
    if (n_snap < 0 || n_snap > 8) return fail(LG_ERR_INVALID_ARG, "n_snap must be in 0..8");
    if (n_snap > 0) {
        LG_CHECK(check_vec(W_snap_host, "W_snap_host"));
        LG_CHECK(check_vec(snap_accum, "snap_accum"));
    }
    if (rec_coeff != nullptr && (rec_row < 1 || rec_row > plan->nz1))
        return fail(LG_ERR_INVALID_ARG, "rec_row out of range");
    LG_HIP(hipSetDevice(plan->device));
    LG_HIP(launch_synth(plan, m0, nb, R_host, W_snap_host, n_snap, snap_accum, rec_row, rec_coeff));
    return LG_OK;
}

lg_status lg_trace_synthesize(lg_plan* plan, const double* rec_coeff, const double* W_host, int32_t nt,
                              double* traces) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(rec_coeff, "rec_coeff"));
    LG_CHECK(check_vec(W_host, "W_host"));
    LG_CHECK(check_vec(traces, "traces"));
    if (nt < 1) return fail(LG_ERR_INVALID_ARG, "nt must be >= 1");
    LG_HIP(hipSetDevice(plan->device));
    double* Wd = nullptr;
    const size_t bytes = (size_t)nt * plan->lag.n * 8;
    LG_HIP(hipMalloc((void**)&Wd, bytes));
    hipError_t e = hipMemcpyAsync(Wd, W_host, bytes, hipMemcpyHostToDevice, plan->stream);
    if (e == hipSuccess) e = launch_traces(plan, rec_coeff, Wd, nt, traces);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    (void)hipFree(Wd);
    if (e != hipSuccess) return hip_fail(e, "lg_trace_synthesize");
    return LG_OK;
}

lg_status lg_trace_synthesize_noalloc(lg_plan* plan, const double* rec_coeff, const double* W_host,
                                      int32_t nt, double* traces) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(rec_coeff, "rec_coeff"));
    LG_CHECK(check_vec(W_host, "W_host"));
    LG_CHECK(check_vec(traces, "traces"));
    if (nt < 1) return fail(LG_ERR_INVALID_ARG, "nt must be >= 1");
    const size_t count = (size_t)nt * plan->lag.n;
    if (count > (size_t)LG_TRACE_SCRATCH_MAX)
        return fail(LG_ERR_UNSUPPORTED, "nt * n = " + std::to_string(count) +
                                            " exceeds the allocation-free staging limit LG_TRACE_SCRATCH_MAX = " +
                                            std::to_string((size_t)LG_TRACE_SCRATCH_MAX));
    LG_HIP(hipSetDevice(plan->device));
    double* Wd = scratch_ptr(plan->device);   // looked up when the plan was created
    if (Wd == nullptr) return fail(LG_ERR_HIP, "staging array of this device was not set up");
    hipError_t e = hipMemcpyAsync(Wd, W_host, count * 8, hipMemcpyHostToDevice, plan->stream);
    if (e == hipSuccess) e = launch_traces(plan, rec_coeff, Wd, nt, traces);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "lg_trace_synthesize_noalloc");
    return LG_OK;
}

lg_status lg_pcg_solve(lg_plan* plan, const double* b, double* x, const lg_solve_opts* opts,
                       lg_solve_info* info_host) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(b, "b"));
    LG_CHECK(check_vec(x, "x"));
    LG_CHECK(check_vec(opts, "opts"));
    if (b == x) return fail(LG_ERR_INVALID_ARG, "b and x must differ");
    if (plan->kind != LG_ACOUSTIC) return fail(LG_ERR_INVALID_ARG, "PCG needs an acoustic plan");
    if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) return fail(LG_ERR_INVALID_ARG, "tol must be >= 0");
    if (opts->max_iter < 1) return fail(LG_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (opts->x0_given != 0 && opts->x0_given != 1) return fail(LG_ERR_INVALID_ARG, "x0_given must be 0 or 1");
    if (opts->x0_given && (plan->cyl || plan->order == 4))
        return fail(LG_ERR_UNSUPPORTED, "axisymmetric and fourth-order plans start from x0 = 0");
    LG_HIP(hipSetDevice(plan->device));
    return lg::pcg_solve(plan, b, x, opts, info_host);
}

lg_status lg_gmres_solve(lg_plan* plan, const double* b, double* x, const lg_solve_opts* opts,
                         lg_solve_info* info_host) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(b, "b"));
    LG_CHECK(check_vec(x, "x"));
    LG_CHECK(check_vec(opts, "opts"));
    if (b == x) return fail(LG_ERR_INVALID_ARG, "b and x must differ");
    if (plan->kind != LG_ELASTIC) return fail(LG_ERR_INVALID_ARG, "GMRES needs an elastic plan");
    if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) return fail(LG_ERR_INVALID_ARG, "tol must be >= 0");
    if (opts->max_iter < 1) return fail(LG_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (opts->restart < 1) return fail(LG_ERR_INVALID_ARG, "restart must be >= 1");
    if (opts->x0_given != 0) return fail(LG_ERR_UNSUPPORTED, "GMRES starts from x0 = 0 (x0_given must be 0)");
    LG_HIP(hipSetDevice(plan->device));
    return lg::gmres_solve(plan, b, x, opts, info_host);
}

}  // extern "C"

extern "C" lg_status lg_precond_apply(lg_plan* plan, const void* r, void* z) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(r, "r"));
    LG_CHECK(check_vec(z, "z"));
    if (r == z) return fail(LG_ERR_INVALID_ARG, "r and z must differ");
    LG_HIP(hipSetDevice(plan->device));
    if (plan->kind == LG_ELASTIC) {
        LG_HIP(launch_elastic_precond(plan, r, z));
        return LG_OK;
    }
    const int nf = plan->S;
    LG_HIP(launch_dst(plan, 0, r, plan->rhat, nf));
    if (plan->cyl) {
        LG_HIP(cyl_launch_rsys(plan, plan->rhat, plan->y, nf, 0));
        LG_HIP(cyl_launch_dct(plan, 1, plan->y, z, nf, plan->blk[0].P > 1));
        return LG_OK;
    }
    LG_HIP(launch_td(plan, 0, plan->rhat, plan->y, nf, 0));
    if (plan->blk[0].P > 1 || plan->free_top) {
        LG_HIP(launch_rs(plan, 0, plan->rhat, plan->y, nf, 0));
        LG_HIP(launch_correct(plan, 0, plan->y, nf));
    }
    LG_HIP(launch_dst(plan, 1, plan->y, z, nf));
    return LG_OK;
}

extern "C" lg_status lg_pcg_profile(lg_plan* plan, const double* b, double* x, int32_t iters, float* ms_host) {
    LG_CHECK(check_plan(plan));
    LG_CHECK(check_vec(b, "b"));
    LG_CHECK(check_vec(x, "x"));
    LG_CHECK(check_vec(ms_host, "ms_host"));
    if (b == x) return fail(LG_ERR_INVALID_ARG, "b and x must differ");
    if (plan->kind != LG_ACOUSTIC) return fail(LG_ERR_INVALID_ARG, "profiling needs an acoustic plan");
    if (iters < 1 || iters > 1000) return fail(LG_ERR_INVALID_ARG, "iters must be in 1..1000");
    LG_HIP(hipSetDevice(plan->device));
    return lg::pcg_profile(plan, b, x, iters, ms_host);
}
