"""CPU oracle for streaming tensor-ring (TR) tracking, FP64, NumPy.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This package is a plain, slow and
deliberately literal implementation of what Yu & Li, "Tracking Tensor Ring
Decompositions of Streaming Tensors" (arXiv 2307.00719) compute: the tensor
primitives of Sec. 2, STR (Alg. 4), rSTR with uniform, leverage-score and
KSRFT sketches (Algs. 5, 7, 8, 9 with Algs. 3 and 6), and the TR fit loss
with its gradient.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP library in ``paper_2307_00719_amd/`` and neither side imports the
other; both receive the same inputs from ``workloads/``.

Conventions (0-based indices throughout):
  * a tensor X is an ``ndarray`` indexed X[i_1, ..., i_N]; whenever it is
    flattened, the first index runs fastest (the paper's column-major
    multi-index of Sec. 2);
  * a TR-core G_n is an ``ndarray`` of shape (R_n, I_n, R_{n+1}), with lateral
    slice G_n(i) = G_n[:, i, :] (Sec. 1);
  * every function states the passage it follows.

Parity status of each function is recorded in its docstring; every function
used by the parity tests is pinned by a CPU test in ``tests/test_oracle_*.py``
against something other than itself (brute force, closed forms, library
routines or invariants).
"""

from . import tensor_ring, rng, streaming, randomized, fitloss, batch_als  # noqa: F401
