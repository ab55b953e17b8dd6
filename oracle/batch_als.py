"""Batch TR-ALS (Alg. 1) and TR-ALS-NE (Alg. 2), FP64.

TEST INFRASTRUCTURE (CPU oracle).  These are not on the streaming path; the
tests use them as the batch accuracy reference that STR is compared with
(Sec. 4.1) and as an alternative initialiser (Sec. 4, protocol: TR-ALS on the
first part of the stream, stopping when the change of relative error falls
below a tolerance or after a maximum number of sweeps).
"""

import numpy as np

from . import tensor_ring as tr
from .streaming import pinv


def tr_als(X, cores0, max_sweeps=100, tol=1e-8, on_mode=None):
    """Alg. 1: per mode, form G^{!=n}_[2] and solve the LS problem of
    eq. tr_als with a least-squares solver.  Returns (cores, rel_errors).
    Stops when the relative error changes by less than ``tol`` between two
    sweeps or after ``max_sweeps`` (Sec. 4 protocol).  ``on_mode(n, cores)``
    (test hook) sees the cores right after each mode update."""
    N = X.ndim
    cores = [np.array(G, dtype=np.float64, copy=True) for G in cores0]
    errs = [tr.rel_error(X, cores)]
    for _ in range(max_sweeps):
        for n in range(N):
            S = tr.subchain_unfold2(tr.subchain(cores, n))
            sol, *_ = np.linalg.lstsq(S, tr.unfold_mode(X, n).T, rcond=None)
            cores[n] = tr.core_fold2(sol.T, cores[n].shape[0], cores[n].shape[2])
            if on_mode is not None:
                on_mode(n, cores)
        errs.append(tr.rel_error(X, cores))
        if abs(errs[-2] - errs[-1]) < tol:
            break
    return cores, errs


def tr_als_ne(X, cores0, max_sweeps=100, tol=1e-8, on_mode=None):
    """Alg. 2: Gram tensors Z_n, H^{!=n} by the contracted chain, M_n by the
    subchain, and the normal-equation solve G_{n(2)} H_<2> = M_n (with the
    pseudo-inverse of the dagger rule).  Same stopping rule and hook as
    ``tr_als``."""
    N = X.ndim
    cores = [np.array(G, dtype=np.float64, copy=True) for G in cores0]
    Z = [tr.gram_tensor(G) for G in cores]
    errs = [tr.rel_error(X, cores)]
    for _ in range(max_sweeps):
        for n in range(N):
            H = tr.gram_chain([Z[k] for k in tr.chain_order(N, n)])
            S = tr.subchain_unfold2(tr.subchain(cores, n))
            M = tr.unfold_mode(X, n) @ S
            Gn2 = M @ pinv(tr.h_unfold(H))
            cores[n] = tr.core_fold2(Gn2, cores[n].shape[0], cores[n].shape[2])
            Z[n] = tr.gram_tensor(cores[n])
            if on_mode is not None:
                on_mode(n, cores)
        errs.append(tr.rel_error(X, cores))
        if abs(errs[-2] - errs[-1]) < tol:
            break
    return cores, errs
