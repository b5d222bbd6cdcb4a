"""Helpers for the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import sys

import numpy as np

from paper_1005_0542_amd import api, inputs


def log(msg: str) -> None:
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def to_np(t):
    return t.detach().to("cpu").double().numpy()


def acoustic_plan(nx, nz, dx, dz, kappa, rho, alpha=9, h=200.0, n=8, precision="fp64", shots=1,
                  segments=0, graph_iters=0):
    med = np.stack([kappa, rho])
    return api.Plan("acoustic", nx, nz, dx, dz, alpha, h, n, med, precision=precision, nshots=shots,
                    segments=segments, graph_iters=graph_iters)


def heterogeneous(nx, nz, seed=1, variable_density=True):
    """Layered + perturbed velocity on an nx x nz grid (cropped square recipe)."""
    n = max(nx, nz)
    v = inputs.perturbed_layered_velocity(n, 2560.0 / n, 1500.0, 4000.0, seed)[: nz + 1, : nx + 1]
    if variable_density:
        return inputs.variable_density_coeffs(v)
    return inputs.acoustic_coeffs(v)


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))
