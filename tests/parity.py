"""Entry-by-entry comparison of a GPU result with the oracle's.

dev(got, ref) is the largest per-entry deviation

    max_i |got_i - ref_i| / (|ref_i| + rms(ref)),

so a bound dev < tol requires every entry to agree to `tol` relative to its
own size, or to the array's root-mean-square size for entries much smaller
than that (an absolute floor scaled to the array).  Unlike a relative
Frobenius norm of the difference, a wrong small entry (a ragged tile, a
small core row) cannot hide under the norm of the large ones.
"""

import numpy as np


def dev(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    d = np.abs(got - ref)
    if not np.all(np.isfinite(d)):
        return float("inf")
    scale = np.abs(ref) + float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    scale = np.where(scale > 0, scale, 1e-300)
    return float(np.max(d / scale))


def assert_close(got, ref, tol, what=""):
    e = dev(got, ref)
    assert e < tol, f"{what}: per-entry deviation {e:.3e} >= {tol:.1e}"
    return e
