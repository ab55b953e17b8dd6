"""Pins of the randomized oracle (Algs. 3, 5-9): the counter generator,
sampled subchains and fibres against explicit rows, Monte-Carlo
unbiasedness of the rescaled sketches, leverage identities, KSRFT
unitarity and exact recovery."""

import os

import numpy as np
import pytest

from oracle import randomized as rs, rng, tensor_ring as tr
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if l.startswith("0x")]
    state, out = 0, []
    for _ in vals:
        out.append(rng.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    assert out == vals
    # vectorised form agrees with the scalar reference
    xs = np.arange(50, dtype=np.uint64) * np.uint64(12345)
    assert [int(v) for v in rng.splitmix64_array(xs)] == [rng.splitmix64(int(x)) for x in xs]


def test_uniform_stream_properties():
    u = rng.uniforms(7, 3, 2, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1 / 12) < 0.002
    idx = rng.uniform_indices(7, 3, 2, 200000, 13)
    counts = np.bincount(idx, minlength=13)
    assert counts.min() > 0.9 * 200000 / 13 and counts.max() < 1.1 * 200000 / 13
    s = rng.signs(7, 3, 2, 100000)
    assert set(np.unique(s)) == {-1.0, 1.0} and abs(s.mean()) < 0.02
    # distinct (step, core, kind) give different streams
    assert not np.array_equal(rng.uniforms(7, 3, 2, 64), rng.uniforms(7, 3, 1, 64))


def test_distribution_sampler():
    p = np.array([0.0, 0.0, 1.0, 0.0])
    assert np.all(rng.distribution_indices(1, 0, 0, 500, p) == 2)
    p = np.array([0.1, 0.2, 0.3, 0.4])
    idx = rng.distribution_indices(1, 0, 0, 400000, p)
    assert np.allclose(np.bincount(idx, minlength=4) / 400000, p, atol=0.004)


def _problem(dims, ranks, T, seed, noise=0.0):
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, seed, noise=noise)
    return cores, X


def test_sampled_subchain_rows_and_fibres():
    """Alg. 3: row s of the sampled subchain is the subchain row at the
    sampled multi-index, and column s of X_S[n] is that column of X_[n]."""
    cores, X = _problem((4, 5, 3), (2, 3, 2, 2), 6, 1, noise=0.1)
    r = rs.RSTR(X, cores, m=17, sketch="uniform", seed=3)
    N = 4
    for n in range(N - 1):
        A = tr.subchain_unfold2(rs.sampled_subchain(r.GS, n))
        S = tr.subchain_unfold2(tr.subchain(cores, n))
        Xn = tr.unfold_mode(X, n)
        XS = rs.sampled_fibres(X, r.idxs, n)
        order = list(range(n + 1, N)) + list(range(n))
        dims = [X.shape[k] for k in order]
        for s in range(17):
            j = tr.lin([r.idxs[k][s] for k in order], dims)
            assert np.allclose(A[s], S[j])
            assert np.allclose(XS[:, s], Xn[:, j])


def _mc_mean(make, trials):
    acc = None
    for t in range(trials):
        P = make(t)
        acc = P if acc is None else acc + P
    return acc / trials


@pytest.mark.parametrize("sketch", ["uniform", "leverage", "ksrft"])
def test_sketched_increments_unbiased(sketch):
    """E[rescaled sketched P_n, Q_n] = exact P_n, Q_n (eq. sampDS and the
    leverage rescaling; E[Psi^T Psi] = I for KSRFT)."""
    cores, X = _problem((4, 3), (2, 2, 3), 5, 2, noise=0.3)
    S = tr.subchain_unfold2(tr.subchain(cores, 0))
    P_ex = tr.unfold_mode(X, 0) @ S
    Q_ex = S.T @ S
    trials = 600

    def mk(t):
        r = rs.RSTR(X, cores, m=8, sketch=sketch, seed=1000 + t)
        return np.concatenate([np.real(r.P[0]).ravel(), np.real(r.Q[0]).ravel()])

    mean = _mc_mean(mk, trials)
    ref = np.concatenate([P_ex.ravel(), Q_ex.ravel()])
    rel = np.linalg.norm(mean - ref) / np.linalg.norm(ref)
    assert rel < 0.08, rel


def test_leverage_identities():
    r = np.random.default_rng(3)
    tall = r.standard_normal((3, 40, 4))            # I = 40 > R^2 = 12
    p = rs.leverage_distribution(tall)
    assert np.isclose(p.sum(), 1.0)
    A = tr.core_unfold2(tall)
    lev = np.einsum("ij,jk,ik->i", A, np.linalg.inv(A.T @ A), A)
    assert np.isclose(lev.sum(), 12.0)
    assert np.allclose(p, lev / 12.0)
    wide = r.standard_normal((3, 7, 4))             # I = 7 <= R^2: uniform
    assert np.allclose(rs.leverage_distribution(wide), 1.0 / 7)


def test_ksrft_unitarity_and_mixing():
    r = np.random.default_rng(4)
    for I in (1, 3, 7, 20):
        F = rs.dft(I)
        assert np.allclose(F.conj().T @ F, np.eye(I))
    X = r.standard_normal((4, 3, 5))
    ds = [rng.signs(9, 0, j, X.shape[j]) for j in range(3)]
    Y = rs.mix_tensor(X, ds)
    for n in range(3):                                # undo every mode
        FD = rs.dft(X.shape[n]) * ds[n][None, :]
        Y = tr.ttm(Y, np.linalg.inv(FD), n)
    assert np.allclose(Y, X)
    # TR of the mixed cores is the mixed TR tensor
    cores, X = _problem((4, 3), (2, 3, 2), 5, 5)
    ds = [rng.signs(9, 1, j, X.shape[j]) for j in range(3)]
    mixed = [rs.mix_core(G, d) for G, d in zip(cores, ds)]
    XT = np.zeros(X.shape, complex)
    for idx in np.ndindex(*X.shape):
        M = np.eye(2, dtype=complex)
        for G, i in zip(mixed, idx):
            M = M @ G[:, i, :]
        XT[idx] = np.trace(M)
    assert np.allclose(XT, rs.mix_tensor(X, ds))
    # unmixing the sampled fibres of mode n gives the fibre mixed on the
    # other modes only
    XS = rs.sampled_fibres(rs.mix_tensor(X, ds), [np.array([1]), np.array([0]),
                                                  np.array([2])], 0)
    part = X.astype(complex)
    for n in (1, 2):
        part = tr.ttm(part, rs.dft(X.shape[n]) * ds[n][None, :], n)
    assert np.allclose(rs.unmix(XS, ds[0])[:, 0], part[:, 0, 2])


@pytest.mark.parametrize("sketch", ["uniform", "leverage", "ksrft"])
@pytest.mark.parametrize("dims,ranks", [((6, 7), (2, 3, 2)), ((5, 6, 4), (2, 2, 3, 2))])
def test_exact_recovery(sketch, dims, ranks):
    cores, X = _problem(dims, ranks, 14, 6)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :6, :]
    r = rs.RSTR(X[..., :6], init, m=40, sketch=sketch, seed=11)
    for t0 in (6, 8, 11):
        t1 = {6: 8, 8: 11, 11: 14}[t0]
        r.update(X[..., t0:t1])
    assert r.rel_error(X) < 1e-11


@pytest.mark.parametrize("sketch", ["uniform", "leverage", "ksrft"])
def test_rstr_tracks_noisy_stream(sketch):
    cores, X = _problem((12, 10), (2, 2, 2), 40, 7, noise=0.05)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :10, :]
    r = rs.RSTR(X[..., :10], init, m=60, sketch=sketch, seed=2)
    for b in range(6):
        r.update(X[..., 10 + 5 * b:15 + 5 * b])
    assert r.rel_error(X) < 0.2
