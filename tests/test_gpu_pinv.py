"""The pseudo-inverse of the normal-equation solves on rank-deficient inputs
(the dagger of G_{n(2)} = P_n Q_n^dagger in Alg. 4 and in Algs. 7-9, and
the rank in the leverage-score lemma), GPU against the FP64 oracle.

The inputs make every rank decision exact, so both sides must take the same
one whatever their rounding:
* a zero core: every Gram chain through it is exactly zero, Q^dagger = 0;
* a TR whose declared rank R_2 is one more than the data's, the extra index
  padded with zeros (row 0 of every slice of core 2, column 0 of every slice
  of core 1): the subchain columns of that index vanish exactly, so Q_n has
  exact zero rows and columns, and the updates keep the padding at zero;
* a zero slice of the data and of a core with I_k <= R_k R_{k+1}: the row
  Gram of the leverage rank check has an exact zero row, rank I_k - 1.
Tolerances: those of the full-rank FP64 parity tests (1e-10 for the fit
error and P/Q, 1e-9 for the cores), entry by entry.  The fallback is
counted by the handle (tr_stream_get_stats).
"""

import numpy as np
import pytest

import workloads as W
from oracle import randomized as rs
from oracle import streaming as st
from parity import dev

pytestmark = pytest.mark.gpu


def padded_problem(dims, ranks, t_init, nb, t_new, seed, noise=0.05):
    """Data of TR-ranks (R_1, R_2 - 1, R_3, ..) and initial cores of ranks
    `ranks` whose extra index of R_2 is zero."""
    small = list(ranks)
    small[1] -= 1
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), small, seed, noise=noise)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    init = W.perturb(init, 0.05, np.random.default_rng(seed + 1))
    N = len(ranks)
    out = []
    for k, G in enumerate(init):
        R0, I, R1 = ranks[k], G.shape[1], ranks[(k + 1) % N]
        H = np.zeros((R0, I, R1))
        r0 = 1 if k == 1 else 0                  # row 0 of core 1's slices is padding
        c0 = 1 if k == 0 else 0                  # column 0 of core 0's slices is padding
        H[r0:, :, c0:] = G
        out.append(H)
    return out, X


def compare(g, o, X, T, N, tag, real=False):
    eo, eg = o.rel_error(X[..., :T]), g.reconstruct_error(X[..., :T])
    cores = max(dev(a, c) for a, c in zip(g.cores(), o.cores))
    pq = 0.0
    for n in range(N - 1):
        Pg, Qg = g.PQ(n)
        Po, Qo = (o.P[n].real, o.Q[n].real) if real else (o.P[n], o.Q[n])
        pq = max(pq, dev(Pg, Po), dev(Qg, Qo))
    fb = g.stats()["pinv_fallbacks"]
    print(f"[pinv {tag}] err gpu {eg:.6e} oracle {eo:.6e} cores {cores:.2e} PQ {pq:.2e} "
          f"fallbacks {fb}", flush=True)
    assert abs(eg - eo) <= 1e-10 * max(eo, 1e-300) and cores < 1e-9 and pq < 1e-10
    assert fb > 0
    return fb


@pytest.mark.parametrize("sketch", [None, "uniform", "ksrft"])
def test_zero_core_matches_oracle(trlib, sketch):
    """Core 2 of 3 is zero: the temporal Gram chain and Q_1 are zero, so the
    new temporal rows and core 1 become zero (P Q^dagger with Q^dagger = 0);
    the fit error is that of the zero tensor, 1."""
    dims, ranks, t_init, t_new, nb, m = (14, 12), (2, 3, 2), 8, 4, 2, 40
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, 6, noise=0.05)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    init[1] = np.zeros_like(init[1])
    if sketch:
        o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch=sketch, seed=2)
    else:
        o = st.STR(X[..., :t_init], [G.copy() for G in init])
    g = trlib.TRStream(X[..., :t_init], init, sketch=sketch, sketch_size=m if sketch else 0,
                       seed=2)
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
    compare(g, o, X, T, len(ranks), f"zero core {sketch}", real=sketch == "ksrft")
    g.close()


# (dims, ranks): the fused per-mode launch (d <= 64) and, with d = 72..90,
# the side kernel on the second stream; order 3 and 4
PADDED = [
    ((16, 13), (2, 3, 2)),
    ((9, 8, 7), (2, 3, 2, 2)),
    ((20, 18), (8, 9, 10)),
]


@pytest.mark.parametrize("dims,ranks", PADDED)
def test_padded_rank_str(trlib, dims, ranks):
    t_init, t_new, nb = 12, 4, 3
    init, X = padded_problem(dims, ranks, t_init, nb, t_new, 31)
    o = st.STR(X[..., :t_init], [G.copy() for G in init])
    g = trlib.TRStream(X[..., :t_init], init)
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
    T = t_init + nb * t_new
    compare(g, o, X, T, len(ranks), f"padded STR {dims} {ranks}")
    # the padding stays exactly zero on the device
    gc = g.cores()
    assert np.all(gc[1][0, :, :] == 0) and np.all(gc[0][:, :, 0] == 0)
    g.close()


@pytest.mark.parametrize("sketch", ["uniform", "leverage", "ksrft"])
def test_padded_rank_sketched(trlib, sketch):
    dims, ranks, t_init, t_new, nb, m = (20, 18), (2, 3, 2), 8, 5, 3, 60
    init, X = padded_problem(dims, ranks, t_init, nb, t_new, 41)
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch=sketch, seed=4)
    g = trlib.TRStream(X[..., :t_init], init, sketch=sketch, sketch_size=m, seed=4)
    N = len(ranks)
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
        sg = g.samples()
        assert all(np.array_equal(sg[k], o.idxs[k]) for k in range(N)), "samples differ"
    T = t_init + nb * t_new
    compare(g, o, X, T, N, f"padded {sketch}", real=sketch == "ksrft")
    g.close()


def test_leverage_rank_deficient_row_gram(trlib):
    """Mode 1 has I_1 = 7 <= R_1 R_2 = 9 and a zero data slice at i_1 = 3
    with the matching zero core slice: the row Gram of core 1 has rank 6, so
    l_3 = 0 and the other scores are 1 (diag of K K^dagger), p = l / 6, on
    both sides; the zero slice persists through the updates."""
    dims, ranks, t_init, t_new, nb, m = (16, 7, 6), (2, 3, 3, 2), 8, 4, 3, 60
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, 51, noise=0.05)
    X = np.asfortranarray(X)
    X[:, 3, :, :] = 0.0
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    init = W.perturb(init, 0.05, np.random.default_rng(52))
    init[1][:, 3, :] = 0.0
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch="leverage", seed=8)
    assert np.allclose(o.p[1][3], 0.0) and np.allclose(o.p[1].sum(), 1.0)
    g = trlib.TRStream(X[..., :t_init], init, sketch="leverage", sketch_size=m, seed=8)
    N = len(ranks)
    s0 = g.samples()
    assert all(np.array_equal(s0[k], o.idxs[k]) for k in range(N)), "initial samples differ"
    assert not np.any(s0[1] == 3)
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
        sg = g.samples()
        assert all(np.array_equal(sg[k], o.idxs[k]) for k in range(N)), "samples differ"
    compare(g, o, X, T, N, "leverage row Gram")
    g.close()
