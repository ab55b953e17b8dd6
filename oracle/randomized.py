"""rSTR -- randomized streaming TR decomposition (Alg. 5) with the uniform
(Alg. 7), leverage-score (Alg. 8) and KSRFT (Alg. 9) sketches, FP64.

TEST INFRASTRUCTURE (CPU oracle).  Steps follow Algs. 7-9 in the paper's
order; the sampled subchain and fibres follow Alg. 3 (SSIT) and the KSRFT
mixing follows Alg. 6.

Readings taken where the paper is silent or ambiguous:
  * X_S[n] holds m mode-n fibres, one per sample row s (the m rows of the
    sampled subchain), not the Cartesian product of the index lists.
  * The rescaling D is applied by default (weight J_n/m per sample for the
    uniform and KSRFT sketches, 1/(m q(j)) for leverage sampling), with J_n
    the number of rows of the sketched matrix: the temporal extent is t_init
    at initialisation and t_new in a time step.  ``rescale=False`` gives the
    "ignored" reading of Sec. 3.3.
  * idxs(:, k) is drawn once per core and refreshed right after G_k is
    updated; the temporal column is redrawn over the new batch after the
    temporal update, and gathers read G_N^new.
  * Leverage distributions use rank(G_{k(2)}) from an SVD with cut-off
    max(size) * eps * sigma_max.
  * KSRFT: F_j is the unitary DFT F[a, b] = exp(-2 pi i a b / I_j) / sqrt(I_j);
    after each re-mix the sampled mixed cores are re-gathered with the
    existing indices; the P/Q updates read
        P_n += Xhat_S[n] conj(Ghat_S[2]),  Q_n += Ghat_S[2]^T conj(Ghat_S[2])
    at initialisation and in every step; the temporal rows are the printed
    form of the KSRFT paragraph of Sec. 3.3 and of Alg. 9,
        G_N^new = Re(Xhat_S) (Re(Ghat_S^T))^dagger
    (a constant sketch weight does not change this least-squares solution);
    ``temporal_literal=False`` gives instead the real-constrained normal
    equations of the complex sketch,
        G_N^new = Re(Xhat_S conj(Ghat_S)) Re(Ghat_S^T conj(Ghat_S))^dagger,
    the form the paper uses for the non-temporal cores.
  * ``set_samples`` replaces the generator's draws (test hook): injected
    indices are used until each row is redrawn right after its core is
    updated; injected signs replace the D_j of the next time step.
"""

import numpy as np

from . import rng
from . import tensor_ring as tr
from .streaming import pinv

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------------------
# Sketch ingredients
# ---------------------------------------------------------------------------

def leverage_distribution(G):
    """p_k(i) = l_i(G_{k(2)}) / rank(G_{k(2)}) (Lemma on leverage estimation,
    Sec. 3.3), with l_i the squared row norms of an orthonormal basis of the
    column space (Def. leverage scores)."""
    A = tr.core_unfold2(G)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.full(A.shape[0], 1.0 / A.shape[0])
    rank = int(np.sum(s > max(A.shape) * EPS * s[0]))
    lev = np.sum(U[:, :rank] ** 2, axis=1)
    return lev / rank


def dft(I):
    """Unitary DFT of dimension I (Def. KSRFT)."""
    a = np.arange(I)
    return np.exp(-2j * np.pi * np.outer(a, a) / I) / np.sqrt(I)


def mix_core(G, d):
    """Ghat = G x_2 (F D) (Alg. 6, mixing of the TR-cores)."""
    FD = dft(G.shape[1]) * d[None, :]
    return np.einsum("ab,rbs->ras", FD, G)


def mix_tensor(X, ds):
    """Xhat = X x_1 (F_1 D_1) x_2 ... x_N (F_N D_N) (Alg. 6)."""
    Y = X.astype(np.complex128)
    for n, d in enumerate(ds):
        Y = tr.ttm(Y, dft(X.shape[n]) * d[None, :], n)
    return Y


def unmix(XS, d):
    """D_n F_n^* applied to the sampled mode-n fibres (Alg. 6, last step)."""
    F = dft(XS.shape[0])
    return d[:, None] * (F.conj().T @ XS)


def sampled_subchain(GS, n):
    """Alg. 3: start from identity slices of size R_{n+1} and take the
    slices-Hadamard product with the sampled cores k = n+1..N, 1..n-1."""
    N = len(GS)
    m = GS[0].shape[1]
    R = GS[n].shape[2]
    T = np.repeat(np.eye(R, dtype=GS[n].dtype)[:, None, :], m, axis=1)
    for k in list(range(n + 1, N)) + list(range(0, n)):
        T = tr.slices_hadamard(T, GS[k])
    return T                                        # (R_{n+1}, m, R_n)


def sampled_fibres(X, idxs, n):
    """Alg. 3, last step, as m mode-n fibres: column s is
    X[idxs[0][s], .., :, .., idxs[N-1][s]] with mode n free (I_n x m)."""
    Xm = np.moveaxis(X, n, 0)
    sel = tuple(idxs[k] for k in range(X.ndim) if k != n)
    return Xm[(slice(None),) + sel]


# ---------------------------------------------------------------------------
# rSTR
# ---------------------------------------------------------------------------

class RSTR:
    """State and steps of rSTR-U / rSTR-L / rSTR-K (Algs. 7 / 8 / 9)."""

    def __init__(self, X_init, cores0, m, sketch="uniform", seed=0,
                 rescale=True, temporal_literal=True):
        assert sketch in ("uniform", "leverage", "ksrft")
        self.N = N = X_init.ndim
        self.m, self.sketch, self.seed = int(m), sketch, int(seed)
        self.rescale, self.temporal_literal = rescale, temporal_literal
        self.cores = [np.array(G, dtype=np.float64, copy=True) for G in cores0]
        self.dims = [G.shape[1] for G in self.cores[:N - 1]]
        self.step = 0
        t0 = X_init.shape[N - 1]
        src_X = X_init
        if sketch == "ksrft":
            self.D = [rng.signs(self.seed, 0, j, X_init.shape[j]) for j in range(N)]
            self.Ghat = [mix_core(G, d) for G, d in zip(self.cores, self.D)]
            src_X = mix_tensor(X_init, self.D)
        if sketch == "leverage":
            self.p = [leverage_distribution(G) for G in self.cores]
        self.next_signs = None
        self.idxs = [self._draw(0, k, self.cores[k].shape[1]) for k in range(N)]
        self.GS = [self._gather(k, self.cores[k]) for k in range(N)]
        self.P, self.Q = [], []
        for n in range(N - 1):
            dP, dQ = self._increments(src_X, n, t0)
            self.P.append(dP)
            self.Q.append(dQ)
        self.G_new = None

    # -- sampling -----------------------------------------------------------
    def _draw(self, step, k, size):
        if self.sketch == "leverage":
            return rng.distribution_indices(self.seed, step, k, self.m, self.p[k])
        return rng.uniform_indices(self.seed, step, k, self.m, size)

    def _gather(self, k, G):
        src = self.Ghat[k] if self.sketch == "ksrft" else G
        return src[:, self.idxs[k], :]

    def _weights(self, n, t):
        """Diagonal of D_n^2 (eq. sampDS and the leverage rescaling)."""
        if not self.rescale:
            return np.ones(self.m)
        if self.sketch == "leverage":
            q = np.ones(self.m)
            for k in range(self.N):
                if k != n:
                    q = q * self.p[k][self.idxs[k]]
            return 1.0 / (self.m * q)
        J = t * int(np.prod([self.dims[k] for k in range(self.N - 1) if k != n]))
        if n == self.N - 1:
            J = int(np.prod(self.dims))
        return np.full(self.m, J / self.m)

    # -- one mode's P/Q increment (Alg. 5 / 7 / 8 / 9 non-temporal step) ----
    def _increments(self, src_X, n, t):
        A = tr.subchain_unfold2(sampled_subchain(self.GS, n))     # m x R^2
        XS = sampled_fibres(src_X, self.idxs, n)                 # I_n x m
        w = self._weights(n, t)
        if self.sketch == "ksrft":
            XS = unmix(XS, self.D[n])
            dP = XS @ (w[:, None] * A.conj())
            dQ = A.T @ (w[:, None] * A.conj())
        else:
            dP = XS @ (w[:, None] * A)
            dQ = A.T @ (w[:, None] * A)
        return dP, dQ

    # -- one time step --------------------------------------------------------
    def update(self, X_new):
        N = self.N
        self.step += 1
        s = self.step
        t_new = X_new.shape[N - 1]
        src_X = X_new
        if self.sketch == "ksrft":
            if self.next_signs is not None:
                self.D = [np.asarray(d, dtype=np.float64) for d in self.next_signs]
                assert all(len(d) == X_new.shape[j] for j, d in enumerate(self.D))
                self.next_signs = None
            else:
                self.D = [rng.signs(self.seed, s, j, X_new.shape[j]) for j in range(N)]
            src_X = mix_tensor(X_new, self.D)
            for k in range(N - 1):
                self.Ghat[k] = mix_core(self.cores[k], self.D[k])
                self.GS[k] = self._gather(k, self.cores[k])

        # temporal mode
        A = tr.subchain_unfold2(sampled_subchain(self.GS, N - 1))  # m x R_N R_1
        XS = sampled_fibres(src_X, self.idxs, N - 1)               # t_new x m
        w = self._weights(N - 1, t_new)
        if self.sketch == "ksrft":
            XS = unmix(XS, self.D[N - 1])
            if self.temporal_literal:
                GN2 = XS.real @ pinv(A.T.real)
            else:
                GN2 = (XS @ (w[:, None] * A.conj())).real @ \
                    pinv((A.T @ (w[:, None] * A.conj())).real)
        else:
            d = np.sqrt(w)
            GN2 = (XS * d[None, :]) @ pinv((d[:, None] * A).T)
        GN = self.cores[N - 1]
        G_new = tr.core_fold2(GN2, GN.shape[0], GN.shape[2])
        self.cores[N - 1] = np.concatenate([GN, G_new], axis=1)
        self.G_new = G_new
        if self.sketch == "leverage":
            self.p[N - 1] = leverage_distribution(G_new)
        if self.sketch == "ksrft":
            self.Ghat[N - 1] = mix_core(G_new, self.D[N - 1])
        self.idxs[N - 1] = self._draw(s, N - 1, t_new)
        self.GS[N - 1] = self._gather(N - 1, G_new)

        # non-temporal modes
        for n in range(N - 1):
            dP, dQ = self._increments(src_X, n, t_new)
            self.P[n] = self.P[n] + dP
            self.Q[n] = self.Q[n] + dQ
            G = self.cores[n]
            if self.sketch == "ksrft":
                Gn2 = self.P[n].real @ pinv(self.Q[n].real)
            else:
                Gn2 = self.P[n] @ pinv(self.Q[n])
            self.cores[n] = tr.core_fold2(Gn2, G.shape[0], G.shape[2])
            if self.sketch == "leverage":
                self.p[n] = leverage_distribution(self.cores[n])
            if self.sketch == "ksrft":
                self.Ghat[n] = mix_core(self.cores[n], self.D[n])
            self.idxs[n] = self._draw(s, n, self.cores[n].shape[1])
            self.GS[n] = self._gather(n, self.cores[n])
        return self

    def set_samples(self, idxs=None, signs=None):
        """Test hook: ``idxs`` (N rows of m indices; row N-1 indexes the newest
        temporal block) replaces the current samples and the sampled cores are
        re-gathered; ``signs`` (N vectors of +-1, the temporal one as long as
        the next batch) replaces the D_j that the next step would draw."""
        N = self.N
        if idxs is not None:
            self.idxs = [np.asarray(idxs[k], dtype=np.int64).copy() for k in range(N)]
            for k in range(N - 1):
                self.GS[k] = self._gather(k, self.cores[k])
            newest = self.G_new if self.G_new is not None else self.cores[N - 1]
            self.GS[N - 1] = self._gather(N - 1, newest)
        if signs is not None:
            self.next_signs = [np.asarray(d, dtype=np.float64).copy() for d in signs]

    def rel_error(self, X_all):
        return tr.rel_error(X_all, self.cores)
