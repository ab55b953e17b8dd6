"""Pins of the oracle parts that the plain-definition tests do not reach:

* the in-step Gauss-Seidel order of Alg. 4 (replay invariant: every P_n, Q_n
  increment was formed with the cores current when mode n was updated), with
  planted Jacobi-order and stale-Gram variants that the replay must reject;
* the temporal step of rSTR (Algs. 7-9) against least squares set up from
  scratch (leverage scores by QR, sampled subchain rows by slice products,
  KSRFT mixing by an explicit Kronecker matrix), with planted dropped-weight
  and dropped-conjugate variants that must differ;
* batch TR-ALS / TR-ALS-NE (Algs. 1, 2): per-mode optimality of every
  update, agreement of the two, the stopping rule;
* the multi-sweep extension of STR, the pseudo-inverse on rank-deficient
  normal equations, the counter-based initial cores, sign injection for
  KSRFT and the tensor-train special case R_1 = 1.

Every helper here is written from the definitions of Sec. 2 (pure-Python
loops over tiny tensors) and shares nothing with ``oracle/`` beyond the
data it is handed.
"""

import itertools

import numpy as np
import pytest

import workloads as W
from oracle import batch_als, randomized as rs, rng, streaming as st, tensor_ring as tr


# ---------------------------------------------------------------------------
# brute-force helpers (definitions of Sec. 2, first index fastest)
# ---------------------------------------------------------------------------

def _decode(j, sizes):
    out = []
    for s in sizes:
        out.append(j % s)
        j //= s
    return out


def subchain_rows(cores, n):
    """G^{!=n}_[2] entry by entry: row j = lin(i_{n+1}, .., i_{n-1}) (cyclic,
    first fastest), column r + R_n s = (G_{n+1}(i_{n+1}) .. G_{n-1}(i_{n-1}))[s, r]."""
    N = len(cores)
    order = [(n + 1 + k) % N for k in range(N - 1)]
    sizes = [cores[k].shape[1] for k in order]
    Rn, Rn1 = cores[n].shape[0], cores[n].shape[2]
    J = int(np.prod(sizes))
    S = np.zeros((J, Rn * Rn1))
    for j in range(J):
        M = np.eye(cores[order[0]].shape[0])
        for k, i in zip(order, _decode(j, sizes)):
            M = M @ cores[k][:, i, :]
        for s in range(Rn1):
            for r in range(Rn):
                S[j, r + Rn * s] = M[s, r]
    return S


def unfold(X, n):
    """X_[n] entry by entry: column j = lin over modes n+1, .., N-1, 0, .., n-1."""
    N = X.ndim
    order = [(n + 1 + k) % N for k in range(N - 1)]
    sizes = [X.shape[k] for k in order]
    J = int(np.prod(sizes))
    out = np.zeros((X.shape[n], J), dtype=X.dtype)
    for j in range(J):
        idx = [0] * N
        for k, i in zip(order, _decode(j, sizes)):
            idx[k] = i
        for i in range(X.shape[n]):
            idx[n] = i
            out[i, j] = X[tuple(idx)]
    return out


def full_tr(cores):
    dims = [G.shape[1] for G in cores]
    X = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        M = np.eye(cores[0].shape[0])
        for G, i in zip(cores, idx):
            M = M @ G[:, i, :]
        X[idx] = np.trace(M)
    return X


def unfold_core(G):
    """G_(2)[i, r + R s] = G[r, i, s]."""
    R0, I, R1 = G.shape
    out = np.zeros((I, R0 * R1))
    for i in range(I):
        for s in range(R1):
            for r in range(R0):
                out[i, r + R0 * s] = G[r, i, s]
    return out


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _problem(dims, ranks, T, t_init, seed, noise):
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, seed, noise=noise)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    return cores, X, W.perturb(init, 0.3, np.random.default_rng(seed + 100))


# ---------------------------------------------------------------------------
# Alg. 4: Gauss-Seidel order (replay invariant)
# ---------------------------------------------------------------------------

def _replay_deviation(cls, dims=(4, 3), ranks=(2, 3, 2), t_init=4, t_new=3, nb=3, sweeps=1):
    """Runs ``cls`` and rebuilds every P_n, Q_n from the logged cores: mode n of
    a step uses the cores of modes < n after the step, G_N^new of the step,
    and the cores of modes n+1..N-2 as they were before the step."""
    N = len(ranks)
    _, X, init = _problem(dims, ranks, t_init + nb * t_new, t_init, 7, 0.2)
    o = cls(X[..., :t_init], [G.copy() for G in init])
    P_ref, Q_ref = [], []
    for n in range(N - 1):
        S = subchain_rows(init, n)
        P_ref.append(unfold(X[..., :t_init], n) @ S)
        Q_ref.append(S.T @ S)
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        before = [c.copy() for c in o.cores]
        o.update(xb, sweeps=sweeps) if sweeps > 1 else o.update(xb)
        after = [c.copy() for c in o.cores]
        g_new = after[N - 1][:, -t_new:, :]
        for n in range(N - 1):
            used = [after[k] if k < n else (g_new if k == N - 1 else before[k])
                    for k in range(N)]
            S = subchain_rows(used, n)
            P_ref[n] = P_ref[n] + unfold(xb, n) @ S
            Q_ref[n] = Q_ref[n] + S.T @ S
    return max(max(relerr(o.P[n], P_ref[n]), relerr(o.Q[n], Q_ref[n])) for n in range(N - 1))


class _JacobiOrder(st.STR):
    """Planted mistake: every mode reads the cores of the step's start."""

    def update(self, X_new, sweeps=1):
        self._start = [c.copy() for c in self.cores]
        return super().update(X_new, sweeps)

    def _mode(self, n, X_new, ZN_new):
        N = self.N
        view = [self._start[k] if k < n else self.cores[k] for k in range(N)]
        view[N - 1] = self.G_new
        S = tr.subchain_unfold2(tr.subchain(view, n))
        self.P[n] = self.P[n] + tr.unfold_mode(X_new, n) @ S
        Zs = [ZN_new if k == N - 1 else self.Z[k] for k in tr.chain_order(N, n)]
        self.Q[n] = self.Q[n] + tr.h_unfold(tr.gram_chain(Zs))
        G = self.cores[n]
        self.cores[n] = tr.core_fold2(self.P[n] @ st.pinv(self.Q[n]), G.shape[0], G.shape[2])
        self.Z[n] = tr.gram_tensor(self.cores[n])


class _StaleGram(st.STR):
    """Planted mistake: the Gram tensors are refreshed only at the end of the
    step, so Q_n's increment uses Z_{n-1} of the old core."""

    def update(self, X_new, sweeps=1):
        self._start_Z = [z.copy() for z in self.Z]
        return super().update(X_new, sweeps)

    def _mode(self, n, X_new, ZN_new):
        N = self.N
        keep = [z for z in self.Z]
        self.Z = [self._start_Z[k] if k < n else keep[k] for k in range(N)]
        super()._mode(n, X_new, ZN_new)
        fresh = self.Z[n]
        self.Z = keep
        self.Z[n] = fresh


def test_str_replay_gauss_seidel_order():
    assert _replay_deviation(st.STR) < 1e-12


def test_str_replay_order4():
    assert _replay_deviation(st.STR, dims=(3, 2, 3), ranks=(2, 2, 3, 2), t_init=3, t_new=2) < 1e-12


def test_replay_rejects_jacobi_order_and_stale_gram():
    assert _replay_deviation(_JacobiOrder) > 1e-6
    assert _replay_deviation(_StaleGram) > 1e-6


# ---------------------------------------------------------------------------
# Multi-sweep extension (one batch, several passes, old part held fixed)
# ---------------------------------------------------------------------------

def test_multisweep_one_equals_default():
    _, X, init = _problem((4, 5), (2, 3, 2), 14, 6, 3, 0.2)
    a = st.STR(X[..., :6], [G.copy() for G in init])
    b = st.STR(X[..., :6], [G.copy() for G in init])
    a.update(X[..., 6:10])
    b.update(X[..., 6:10], sweeps=1)
    for x, y in zip(a.cores + a.P + a.Q, b.cores + b.P + b.Q):
        assert np.array_equal(x, y)


def test_multisweep_frozen_cores_is_idempotent():
    _, X, init = _problem((4, 5), (2, 3, 2), 14, 6, 4, 0.2)
    a = st.STR(X[..., :6], [G.copy() for G in init], freeze_nontemporal=True)
    b = st.STR(X[..., :6], [G.copy() for G in init], freeze_nontemporal=True)
    a.update(X[..., 6:10])
    b.update(X[..., 6:10], sweeps=3)
    assert a.cores[-1].shape == b.cores[-1].shape
    for x, y in zip(a.cores + a.P + a.Q, b.cores + b.P + b.Q):
        assert np.allclose(x, y, rtol=0, atol=1e-12 * max(1.0, np.abs(y).max()))


def test_multisweep_exact_recovery():
    cores, X = W.random_tr_problem((4, 3, 12), (2, 3, 2), 5)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :4, :]
    s = st.STR(X[..., :4], init)
    s.update(X[..., 4:8], sweeps=3)
    s.update(X[..., 8:12], sweeps=2)
    assert s.rel_error(X) < 1e-12


def test_multisweep_counts_old_slices_once():
    """After two passes, P_n = P_n^old + X_[n]^new S_n with S_n built from the
    cores of the second pass (modes < n after it, modes > n after the first
    pass), and the temporal core holds t_old + t_new slices."""
    _, X, init = _problem((4, 3), (2, 3, 2), 10, 5, 9, 0.3)
    N = 3
    o = st.STR(X[..., :5], [G.copy() for G in init])
    o.update(X[..., 5:7])
    P_old = [p.copy() for p in o.P]
    Q_old = [q.copy() for q in o.Q]
    mid = st.STR(X[..., :5], [G.copy() for G in init])
    mid.update(X[..., 5:7])
    xb = X[..., 7:10]
    mid.update(xb, sweeps=1)
    o.update(xb, sweeps=2)
    assert o.cores[-1].shape[1] == 10
    g_new = o.cores[-1][:, -3:, :]
    for n in range(N - 1):
        used = [o.cores[k] if k < n else (g_new if k == N - 1 else mid.cores[k])
                for k in range(N)]
        S = subchain_rows(used, n)
        assert relerr(o.P[n], P_old[n] + unfold(xb, n) @ S) < 1e-12
        assert relerr(o.Q[n], Q_old[n] + S.T @ S) < 1e-12
    assert _replay_deviation(st.STR, sweeps=1) < 1e-12


# ---------------------------------------------------------------------------
# Rank-deficient normal equations: the dagger of Alg. 4
# ---------------------------------------------------------------------------

def test_pinv_on_rank_deficient_q():
    """A rank index of the ring that both neighbouring cores leave unused
    (G_1(i)[:, R_2 - 1] = 0 and G_2(i)[R_2 - 1, :] = 0) makes whole columns
    of the subchains of modes 1 and 2 zero, so their Q_n are singular at
    every step.  The dagger then gives the minimum-norm solution: G_(2) Q = P
    still holds and G_(2) is zero on Q's null space, which keeps the unused
    index unused."""
    _, X, init = _problem((5, 4), (3, 2, 2), 12, 6, 11, 0.2)
    init[0][:, :, -1] = 0.0
    init[1][-1, :, :] = 0.0
    s = st.STR(X[..., :6], [G.copy() for G in init])
    for b in range(2):
        s.update(X[..., 6 + 3 * b:9 + 3 * b])
    for n in range(2):
        Q, P = s.Q[n], s.P[n]
        G2 = unfold_core(s.cores[n])
        null = np.where(np.abs(np.diag(Q)) == 0)[0]
        assert null.size > 0
        assert np.allclose(G2 @ Q, P, rtol=0, atol=1e-10 * np.abs(P).max())
        assert np.all(G2[:, null] == 0) and np.all(P[:, null] == 0)


def test_pinv_on_zero_core():
    _, X, init = _problem((5, 4), (2, 2, 2), 10, 6, 12, 0.2)
    init[1] = np.zeros_like(init[1])
    s = st.STR(X[..., :6], [G.copy() for G in init])
    s.update(X[..., 6:10])
    # every subchain through the zero core vanishes: Q = 0, P = 0, G = 0
    assert np.all(s.cores[0] == 0) and np.all(s.G_new == 0)


# ---------------------------------------------------------------------------
# rSTR temporal step (Algs. 7-9) against least squares built from scratch
# ---------------------------------------------------------------------------

def _sampled_rows(cores, idxs, n):
    """Row s: subchain row at the sample's indices (product of slices)."""
    N = len(cores)
    order = [(n + 1 + k) % N for k in range(N - 1)]
    Rn, Rn1 = cores[n].shape[0], cores[n].shape[2]
    m = len(idxs[0])
    A = np.zeros((m, Rn * Rn1), dtype=cores[order[0]].dtype)
    for s in range(m):
        M = np.eye(cores[order[0]].shape[0], dtype=A.dtype)
        for k in order:
            M = M @ cores[k][:, idxs[k][s], :]
        for q in range(Rn1):
            for r in range(Rn):
                A[s, r + Rn * q] = M[q, r]
    return A


def _temporal_fibres(X, idxs):
    N = X.ndim
    m = len(idxs[0])
    return np.stack([X[tuple(int(idxs[k][s]) for k in range(N - 1)) + (slice(None),)]
                     for s in range(m)], axis=1)            # t_new x m


def _leverage_qr(G):
    A = unfold_core(G)
    Qm, Rm = np.linalg.qr(A)
    rank = int(np.sum(np.abs(np.diag(Rm)) > 1e-10 * np.abs(np.diag(Rm)).max()))
    return np.sum(Qm[:, :rank] ** 2, axis=1) / rank


@pytest.mark.parametrize("sketch", ["uniform", "leverage"])
def test_rstr_temporal_rows_weighted_least_squares(sketch):
    dims, ranks, t_init, t_new, m = (12, 10), (2, 2, 2), 6, 4, 40
    _, X, init = _problem(dims, ranks, t_init + t_new, t_init, 13, 0.2)
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch=sketch, seed=5)
    before = [c.copy() for c in o.cores]
    idxs = [i.copy() for i in o.idxs]
    xb = X[..., t_init:]
    o.update(xb)
    N = 3
    A = _sampled_rows(before, idxs, N - 1)
    XS = _temporal_fibres(xb, idxs)
    if sketch == "leverage":
        p = [_leverage_qr(before[k]) for k in range(N - 1)]
        for k in range(N - 1):
            assert np.allclose(p[k], rs.leverage_distribution(before[k]), rtol=1e-10, atol=0)
        w = 1.0 / (m * p[0][idxs[0]] * p[1][idxs[1]])
    else:
        w = np.full(m, dims[0] * dims[1] / m)
    G_w = np.linalg.solve((A.T * w) @ A, (A.T * w) @ XS.T).T
    got = unfold_core(o.G_new)
    assert relerr(got, G_w) < 1e-10
    if sketch == "leverage":
        # planted mistake: the leverage weights dropped in the temporal solve
        G_u = np.linalg.solve(A.T @ A, A.T @ XS.T).T
        assert relerr(G_u, G_w) > 1e-4


def _dft(I):
    a = np.arange(I)
    return np.exp(-2j * np.pi * np.outer(a, a) / I) / np.sqrt(I)


def _mix_kron(X, D):
    """vec(Xhat) = (F_N D_N (x) .. (x) F_1 D_1) vec(X), first index fastest."""
    K = np.ones((1, 1))
    for n in range(X.ndim):
        K = np.kron(_dft(X.shape[n]) * D[n][None, :], K)
    return (K @ X.reshape(-1, order="F")).reshape(X.shape, order="F")


@pytest.mark.parametrize("literal", [True, False])
def test_ksrft_temporal_rows(literal):
    """Alg. 9's temporal rows from an explicit Kronecker mixing: the printed
    form Re(Xhat_S)(Re(Ghat_S^T))^dagger (default), or the real-constrained
    least squares of the complex sketch (flag)."""
    dims, ranks, t_init, t_new, m = (4, 5), (2, 2, 2), 5, 3, 30
    _, X, init = _problem(dims, ranks, t_init + t_new, t_init, 17, 0.2)
    seed = 23
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch="ksrft", seed=seed,
                temporal_literal=literal)
    before = [c.copy() for c in o.cores]
    idxs = [i.copy() for i in o.idxs]
    xb = X[..., t_init:]
    o.update(xb)
    N = 3
    D = [rng.signs(seed, 1, j, xb.shape[j]) for j in range(N)]
    Xh = _mix_kron(xb, D)
    # undo the temporal mixing (D_N F_N^* of Alg. 6's last step)
    FN = _dft(t_new) * D[N - 1][None, :]
    Xt = np.tensordot(Xh, np.linalg.inv(FN), axes=([N - 1], [1]))
    XS = _temporal_fibres(Xt, idxs)                          # complex t_new x m
    Gh = []
    for k in range(N - 1):
        F = _dft(dims[k]) * D[k][None, :]
        Gh.append(np.einsum("ab,rbs->ras", F, before[k]))
    A = _sampled_rows(Gh + [before[N - 1]], idxs, N - 1)    # complex m x d
    if literal:
        ref = np.linalg.solve(A.real.T @ A.real, A.real.T @ XS.real.T).T
    else:
        lhs = A.real.T @ A.real + A.imag.T @ A.imag
        rhs = XS.real @ A.real + XS.imag @ A.imag
        ref = np.linalg.solve(lhs, rhs.T).T
        # planted mistake: no conjugation in the Re-Gram and the product
        bad = np.linalg.solve((A.T @ A).real, (XS @ A).real.T).T
        assert relerr(bad, ref) > 1e-4
    assert relerr(unfold_core(o.G_new), ref) < 1e-9


def test_ksrft_sign_injection():
    """Signs injected for the next step replace the generator's D_j: the
    generator's own signs injected give bit-identical results; flipped ones
    give others."""
    dims, ranks, t_init, t_new, m = (4, 5), (2, 2, 2), 5, 3, 30
    _, X, init = _problem(dims, ranks, t_init + 2 * t_new, t_init, 19, 0.2)
    mk = lambda: rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m,  # noqa: E731
                         sketch="ksrft", seed=4)
    a, b, c = mk(), mk(), mk()
    xb = X[..., t_init:t_init + t_new]
    sizes = list(dims) + [t_new]
    gen = [rng.signs(4, 1, j, sizes[j]) for j in range(3)]
    b.set_samples(signs=gen)
    flipped = [d.copy() for d in gen]
    flipped[0][0] *= -1
    c.set_samples(signs=flipped)
    for o in (a, b, c):
        o.update(xb)
    for x, y in zip(a.cores, b.cores):
        assert np.array_equal(x, y)
    assert relerr(c.cores[0], a.cores[0]) > 1e-8
    assert np.array_equal(c.D[0], flipped[0])


# ---------------------------------------------------------------------------
# Batch TR-ALS (Alg. 1) and TR-ALS-NE (Alg. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("solver", ["tr_als", "tr_als_ne"])
def test_batch_als_each_mode_is_least_squares_optimal(solver):
    """After mode n's update the gradient of 1/2||TR(G) - X||^2 with respect
    to G_(2) vanishes: (TR(G) - X)_[n] G^{!=n}_[2] = 0 (brute force)."""
    cores, X = W.random_tr_problem((4, 3, 5), (2, 2, 2), 31, noise=0.3)
    start = W.perturb(cores, 0.5, np.random.default_rng(1))
    worst = []

    def check(n, cur):
        E = full_tr(cur) - X
        S = subchain_rows(cur, n)
        g = unfold(E, n) @ S
        worst.append(np.linalg.norm(g) / (np.linalg.norm(X) * np.linalg.norm(S)))

    getattr(batch_als, solver)(X, start, max_sweeps=2, tol=0.0, on_mode=check)
    assert len(worst) == 6 and max(worst) < 1e-12


def test_batch_als_ne_equals_als():
    cores, X = W.random_tr_problem((5, 4, 6), (2, 3, 2), 32, noise=0.2)
    start = W.perturb(cores, 0.3, np.random.default_rng(2))
    a, ea = batch_als.tr_als(X, start, max_sweeps=6, tol=0.0)
    b, eb = batch_als.tr_als_ne(X, start, max_sweeps=6, tol=0.0)
    assert len(ea) == len(eb) == 7
    for x, y in zip(a, b):
        assert relerr(y, x) < 1e-9
    assert all(e1 <= e0 * (1 + 1e-12) for e0, e1 in zip(eb, eb[1:]))


def test_batch_als_stopping_rule():
    cores, X = W.random_tr_problem((5, 4, 6), (2, 2, 2), 33, noise=0.05)
    start = W.perturb(cores, 0.2, np.random.default_rng(3))
    _, errs = batch_als.tr_als_ne(X, start, max_sweeps=100, tol=1e-6)
    d = np.abs(np.diff(errs))
    assert d[-1] < 1e-6 and np.all(d[:-1] >= 1e-6)
    _, errs = batch_als.tr_als_ne(X, start, max_sweeps=3, tol=0.0)
    assert len(errs) == 4


def test_batch_als_recovers_exact_tr_from_counter_start():
    cores, X = W.random_tr_problem((6, 5, 7), (2, 2, 2), 34)
    start = rng.init_cores(77, (6, 5, 7), (2, 2, 2))
    _, errs = batch_als.tr_als_ne(X, start, max_sweeps=200, tol=1e-14)
    assert errs[-1] < 1e-6


# ---------------------------------------------------------------------------
# Counter-based initial cores (Irwin-Hall normals)
# ---------------------------------------------------------------------------

def test_initial_core_stream_moments_and_layout():
    z = rng.irwin_hall_normals(2024, 3, 200000)
    assert np.all(np.abs(z) <= 6.0)
    # mean 0 and variance 1 (12 uniforms of variance 1/12 each)
    assert abs(z.mean()) < 5 / np.sqrt(200000)
    assert abs(z.var() - 1.0) < 0.02
    # the excess kurtosis of Irwin-Hall(12) is -6/(5*12) = -0.1
    k = np.mean(z ** 4) / z.var() ** 2 - 3.0
    assert abs(k + 0.1) < 0.05
    cs = rng.init_cores(5, (3, 4, 2), (2, 3, 1))
    assert [c.shape for c in cs] == [(2, 3, 3), (3, 4, 1), (1, 2, 2)]
    flat = rng.irwin_hall_normals(5, 1, 12)
    assert np.array_equal(cs[1][:, :, 0].reshape(-1, order="F"), flat)
    assert not np.array_equal(rng.irwin_hall_normals(5, 0, 12), flat)


# ---------------------------------------------------------------------------
# Tensor train: R_1 = 1 (remark after Alg. 4)
# ---------------------------------------------------------------------------

def test_tensor_train_special_case():
    """With R_1 = 1 the ring closes through a 1 x 1 product, so the TR format
    is a TT: X(i) = G_1(i_1) .. G_N(i_N) (row vector times matrices times a
    column vector); STR keeps the exact TT at its fixed point and the replay
    invariant holds."""
    dims, ranks = (5, 4, 9), (1, 3, 2)
    cores, X = W.random_tr_problem(dims, ranks, 35)
    for idx in itertools.product(*[range(d) for d in dims]):
        v = cores[0][0, idx[0], :]
        v = v @ cores[1][:, idx[1], :]
        v = v @ cores[2][:, idx[2], 0]
        assert abs(X[idx] - v) <= 1e-12 * max(1.0, abs(v))
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :3, :]
    s = st.STR(X[..., :3], init)
    s.update(X[..., 3:6])
    s.update(X[..., 6:9])
    assert s.rel_error(X) < 1e-12
    assert _replay_deviation(st.STR, dims=(4, 3), ranks=(1, 2, 3)) < 1e-12
