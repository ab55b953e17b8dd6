"""STR -- streaming TR decomposition (Alg. 4), FP64, step by step.

TEST INFRASTRUCTURE (CPU oracle).

Readings of the paper taken here (each is also listed in the design notes):
  * Init also forms Z_N from the initial temporal core, because the Q_n
    initialisation of Alg. 4 uses Z_N although only Z_1..Z_{N-1} are listed.
  * The Q_n increment uses Z_N^new, the Gram tensor of the new temporal rows
    only (Sec. 3.1, definition of H^{!=n}_new), not the Z_N over all rows that
    Alg. 4 recomputes after the append.
  * The pseudo-inverse (dagger) is taken literally, as an SVD pseudo-inverse
    with the cut-off max(size) * eps * sigma_max.
  * One call of ``update`` is one time step of Alg. 4: the temporal mode, then
    n = 1..N-1 in order, each mode using the cores already updated in the
    same step.
  * ``sweeps`` > 1 (an extension, not in the paper) repeats that pass on the
    same batch.  Every repetition starts again from the P_n^old, Q_n^old held
    before the batch (Sec. 3.1 splits P_n, Q_n into an old part and the new
    batch's part, eq. partial), recomputes the new temporal rows from the
    current non-temporal cores (replacing the previous pass's rows instead
    of appending more) and re-forms the new batch's increments with the
    refreshed cores, so the old slices are never counted twice.
"""

import numpy as np

from . import tensor_ring as tr

EPS = np.finfo(np.float64).eps


def pinv(A):
    """Pseudo-inverse (the dagger of Alg. 4) with singular values below
    max(size) * eps * sigma_max treated as zero."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros(A.T.shape)
    tol = max(A.shape) * EPS * s[0]
    keep = s > tol
    return (Vt[keep].T / s[keep]) @ U[:, keep].T


class STR:
    """State and steps of Alg. 4.

    Attributes (0-based mode index n = 0..N-1, N-1 is the temporal mode):
      cores[n]  TR-cores, shape (R_n, I_n, R_{n+1}); cores[N-1] grows in time
      Z[n]      Gram tensors (Alg. 4 initialisation / refresh)
      P[n], Q[n] complementary matrices of the non-temporal modes (Sec. 3.1,
                the normal equation), shapes (I_n, R_n R_{n+1}) and
                (R_n R_{n+1}, R_n R_{n+1})
      G_new     temporal rows added by the last step (Alg. 4, G_N^new)
    """

    def __init__(self, X_init, cores0, freeze_nontemporal=False):
        """``freeze_nontemporal`` is a test hook: the P_n/Q_n increments are
        accumulated as usual but the non-temporal cores are not re-solved, the
        setting in which the derivation of eq. partial is exact."""
        self.freeze = freeze_nontemporal
        self.N = N = X_init.ndim
        assert len(cores0) == N
        self.cores = [np.array(G, dtype=np.float64, copy=True) for G in cores0]
        assert self.cores[N - 1].shape[1] == X_init.shape[N - 1]
        # Alg. 4, initialisation: Gram tensors (plus Z_N, see module notes)
        self.Z = [tr.gram_tensor(G) for G in self.cores]
        self.P, self.Q = [], []
        for n in range(N - 1):
            S = tr.subchain_unfold2(tr.subchain(self.cores, n))
            self.P.append(tr.unfold_mode(X_init, n) @ S)
            H = tr.gram_chain([self.Z[k] for k in tr.chain_order(N, n)])
            self.Q.append(tr.h_unfold(H))
        self.G_new = None
        self.steps = 0

    # -- Alg. 4, update stage for the temporal mode -------------------------
    def _temporal(self, X_new):
        N = self.N
        H = tr.gram_chain([self.Z[k] for k in range(N - 2, -1, -1)])
        S = tr.subchain_unfold2(tr.subchain(self.cores, N - 1))
        GN2_new = tr.unfold_mode(X_new, N - 1) @ S @ pinv(tr.h_unfold(H))
        GN = self.cores[N - 1]
        G_new = tr.core_fold2(GN2_new, GN.shape[0], GN.shape[2])
        self.cores[N - 1] = np.concatenate([GN, G_new], axis=1)
        self.G_new = G_new
        return tr.gram_tensor(G_new)                 # Z_N^new

    # -- Alg. 4, update stage for the non-temporal modes --------------------
    def _mode(self, n, X_new, ZN_new):
        N = self.N
        cores_new = list(self.cores)
        cores_new[N - 1] = self.G_new                # G^{!=n}_new (eq. partial2)
        S = tr.subchain_unfold2(tr.subchain(cores_new, n))
        self.P[n] = self.P[n] + tr.unfold_mode(X_new, n) @ S
        Zs = [ZN_new if k == N - 1 else self.Z[k] for k in tr.chain_order(N, n)]
        self.Q[n] = self.Q[n] + tr.h_unfold(tr.gram_chain(Zs))
        if self.freeze:
            return
        G = self.cores[n]
        Gn2 = self.P[n] @ pinv(self.Q[n])
        self.cores[n] = tr.core_fold2(Gn2, G.shape[0], G.shape[2])
        self.Z[n] = tr.gram_tensor(self.cores[n])

    def update(self, X_new, sweeps=1):
        """One time step of Alg. 4 for the batch X_new (I_1 x .. x t_new);
        ``sweeps`` passes over the batch (see the module notes)."""
        N = self.N
        P_old = [P.copy() for P in self.P]
        Q_old = [Q.copy() for Q in self.Q]
        t_new = X_new.shape[N - 1]
        for k in range(int(sweeps)):
            if k > 0:
                self.cores[N - 1] = self.cores[N - 1][:, :-t_new, :]
                self.P = [P.copy() for P in P_old]
                self.Q = [Q.copy() for Q in Q_old]
            ZN_new = self._temporal(X_new)
            for n in range(N - 1):
                self._mode(n, X_new, ZN_new)
        self.Z[N - 1] = tr.gram_tensor(self.cores[N - 1])
        self.steps += 1
        return self

    def rel_error(self, X_all):
        return tr.rel_error(X_all, self.cores)
