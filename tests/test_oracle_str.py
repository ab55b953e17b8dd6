"""Pins of the STR oracle (Alg. 4) against least squares, batch
recomputation and exact-recovery fixed points."""

import numpy as np
import pytest

from oracle import batch_als, streaming as st, tensor_ring as tr
import workloads as W


def _problem(dims, ranks, T, t_init, seed, noise):
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, seed, noise=noise)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    return cores, X, init


def test_pinv_rule():
    r = np.random.default_rng(0)
    A = r.standard_normal((6, 6))
    S = A @ A.T + 6 * np.eye(6)
    assert np.allclose(st.pinv(S) @ S, np.eye(6), atol=1e-12)
    B = r.standard_normal((6, 3))
    S2 = B @ B.T                                   # rank 3
    assert np.allclose(st.pinv(S2), np.linalg.pinv(S2, rcond=6 * np.finfo(float).eps),
                       atol=1e-10)


def test_init_matches_batch_products():
    """Initialisation of Alg. 4: P_n = X_[n] G^{!=n}_[2], Q_n = Gram of the
    explicit subchain over the initial slices."""
    cores, X, init = _problem((4, 5, 3), (2, 3, 2, 3), 9, 9, 1, 0.1)
    s = st.STR(X, cores)
    for n in range(3):
        S = tr.subchain_unfold2(tr.subchain_bruteforce(cores, n))
        assert np.allclose(s.P[n], tr.unfold_mode(X, n) @ S, atol=1e-10)
        assert np.allclose(s.Q[n], S.T @ S, atol=1e-10 * np.abs(S.T @ S).max())


def test_temporal_rows_are_least_squares():
    """G_N^new solves min ||X_[N]^new - G_N(2)^new (G^{!=N}_[2])^T|| for the
    cores at the start of the step (Sec. 3.1, temporal mode)."""
    cores, X, init = _problem((5, 6), (2, 3, 4), 14, 8, 2, 0.3)
    s = st.STR(X[..., :8], [G.copy() for G in init])
    S = tr.subchain_unfold2(tr.subchain(s.cores, 2))
    s.update(X[..., 8:11])
    ref, *_ = np.linalg.lstsq(S, tr.unfold_mode(X[..., 8:11], 2).T, rcond=None)
    assert np.allclose(tr.core_unfold2(s.G_new), ref.T, atol=1e-10)


def test_nontemporal_solve_satisfies_normal_equation():
    cores, X, init = _problem((5, 6), (2, 3, 4), 14, 8, 3, 0.3)
    s = st.STR(X[..., :8], [G.copy() for G in init])
    s.update(X[..., 8:11])
    for n in range(2):
        G2 = tr.core_unfold2(s.cores[n])
        assert np.allclose(G2 @ s.Q[n], s.P[n], atol=1e-9 * np.abs(s.P[n]).max())


@pytest.mark.parametrize("dims,ranks", [((4, 5), (2, 3, 2)), ((3, 4, 5), (2, 2, 3, 2))])
def test_frozen_core_incremental_equals_batch(dims, ranks):
    """With the non-temporal cores frozen, the incremental P_n / Q_n of
    eq. partial equal X_[n] G^{!=n}_[2] and its Gram over all slices seen."""
    cores, X, init = _problem(dims, ranks, 23, 5, 4, 0.5)
    s = st.STR(X[..., :5], [G.copy() for G in init], freeze_nontemporal=True)
    for t0 in (5, 8, 11, 16):
        t1 = {5: 8, 8: 11, 11: 16, 16: 23}[t0]
        s.update(X[..., t0:t1])
    N = len(ranks)
    for n in range(N - 1):
        S = tr.subchain_unfold2(tr.subchain(s.cores, n))
        P_batch = tr.unfold_mode(X, n) @ S
        assert np.allclose(s.P[n], P_batch, rtol=0, atol=1e-11 * np.abs(P_batch).max())
        assert np.allclose(s.Q[n], S.T @ S, rtol=0, atol=1e-11 * np.abs(S.T @ S).max())


def test_batch_size_invariance_with_frozen_cores():
    cores, X, init = _problem((4, 5), (2, 3, 2), 36, 6, 5, 0.5)
    a = st.STR(X[..., :6], [G.copy() for G in init], freeze_nontemporal=True)
    for b in range(6):
        a.update(X[..., 6 + 5 * b:11 + 5 * b])
    c = st.STR(X[..., :6], [G.copy() for G in init], freeze_nontemporal=True)
    c.update(X[..., 6:36])
    assert np.allclose(a.cores[-1], c.cores[-1], atol=1e-12)
    for n in range(2):
        assert np.allclose(a.P[n], c.P[n], atol=1e-10 * np.abs(c.P[n]).max())
        assert np.allclose(a.Q[n], c.Q[n], atol=1e-10 * np.abs(c.Q[n]).max())


@pytest.mark.parametrize("dims,ranks", [((5, 6), (2, 3, 4)), ((4, 3, 5), (2, 3, 2, 2)),
                                        ((3, 4, 2, 3), (2, 2, 2, 1, 2))])
def test_exact_recovery_fixed_point(dims, ranks):
    """Noiseless TR data and the generating cores as initial cores: every
    step of Alg. 4 keeps a zero-residual decomposition."""
    cores, X, init = _problem(dims, ranks, 17, 5, 6, 0.0)
    s = st.STR(X[..., :5], init)
    for t0 in (5, 9, 13):
        s.update(X[..., t0:t0 + 4])
    assert s.rel_error(X) < 1e-12


def test_zero_batch_leaves_state():
    cores, X, init = _problem((4, 5), (2, 3, 2), 12, 6, 7, 0.2)
    s = st.STR(X[..., :6], [G.copy() for G in init])
    s.update(X[..., 6:9])
    P0 = [p.copy() for p in s.P]
    Q0 = [q.copy() for q in s.Q]
    C0 = [c.copy() for c in s.cores]
    s.update(np.zeros(X[..., 9:12].shape, order="F"))
    assert np.all(s.G_new == 0)
    for n in range(2):
        assert np.allclose(s.P[n], P0[n]) and np.allclose(s.Q[n], Q0[n])
        assert np.allclose(s.cores[n], C0[n], atol=1e-10)
    assert np.allclose(s.cores[-1][:, :9, :], C0[-1])


def test_c1_streaming_tracks():
    w = W.make("c1")
    s = st.STR(w.X_init(), w.cores_init)
    e0 = s.rel_error(w.X_init())
    for b in range(w.n_batches):
        s.update(w.batch(b))
    e = s.rel_error(w.X[..., :w.t_init + w.n_batches * w.t_new])
    assert e < e0 and e < 0.01


def test_str_close_to_batch_als_ne():
    """STR's final error is close to that of batch TR-ALS-NE run on all the
    data from the same start (Sec. 4.1 reports them as very similar; the
    paper prints no number, so this bound is ours: parity unpinned)."""
    w = W.make("c1")
    s = st.STR(w.X_init(), w.cores_init)
    for b in range(w.n_batches):
        s.update(w.batch(b))
    start = [G.copy() for G in w.cores_init]
    start[-1] = np.concatenate([start[-1], s.cores[-1][:, w.t_init:, :]], axis=1)
    _, errs = batch_als.tr_als_ne(w.X, start, max_sweeps=30, tol=1e-10)
    e_str = s.rel_error(w.X)
    assert e_str < 1.5 * errs[-1]
