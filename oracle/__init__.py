"""FP64 CPU oracle for the Laguerre-harmonic Krylov solve (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously correct restatement of what the
method of Fatyanov & Terekhov (arXiv 1005.0542) computes, written in numpy /
scipy in double precision.  It exists only to check the HIP library:

* it is imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
  ``cpu_baseline`` leg of ``bench.py`` -- nothing else may use it;
* it shares no code with the HIP path (``paper_1005_0542_amd/``): no kernel,
  header, table or constant generator, and it imports nothing from there
  except the neutral seeded input generators in ``paper_1005_0542_amd.inputs``.

Modules
-------
``laguerre``   Laguerre functions, the forward transform of the source wavelet
               and the synthesis weights (Sec. 2.1, eqs. series_lag, laguerre_h).
``operator``   the 5-point second-order operator A (Sec. 2.3, eqs.
               poisson_diff_2, scheme_op_r_z, diff_approx1) in 2D Cartesian form.
``precond``    the Laplace preconditioner B (Sec. 2.4, eq. precond1) inverted by
               separation of variables: DST-I along x, Thomas along z.
``krylov``     preconditioned CG (Sec. 2.3) and restarted GMRES(k) (Sec. 2.3).
``harmonics``  the right-hand-side recurrence over harmonics (eq. laguerre_h),
               the harmonic loop and the inverse-transform synthesis.
``elastic``    the 2D Cartesian elastic operator C and block preconditioner K
               (eqs. elastic_problemQn, precond2) -- the finite-volume scheme is
               not printed in the paper, so this part is "parity unpinned"
               against the paper (it is pinned against its own brute force).

Status codes follow the C library: 0 ok, 2 not converged, 3 breakdown,
4 non-finite.
"""

OK = 0
NOT_CONVERGED = 2
BREAKDOWN = 3
NONFINITE = 4
