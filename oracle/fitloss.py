"""TR fit loss 1/2 ||TR(G) - X||_F^2 and its core gradients, FP64.

TEST INFRASTRUCTURE (CPU oracle).

The loss is the objective of eq. trmin squared and halved, as in the ALS
subproblem eq. tr_als.  Its gradient with respect to G_{n(2)} follows from
the normal equation of Sec. 3.1 (eq. partial):
    d loss / d G_{n(2)} = G_{n(2)} Q_n - P_n,
    P_n = X_[n] G^{!=n}_[2],  Q_n = (G^{!=n}_[2])^T G^{!=n}_[2],
which equals (TR(G) - X)_[n] G^{!=n}_[2]; both forms are provided so that
the tests can pin one against the other and against finite differences.
"""

import numpy as np

from . import tensor_ring as tr


def fit_loss(X, cores):
    """1/2 ||TR(G) - X||_F^2 by direct residual."""
    E = tr.tr_reconstruct(cores) - X
    return 0.5 * float(np.sum(E * E))


def P_Q(X, cores, n):
    """Batch P_n and Q_n over the whole tensor (eq. partial), with Q_n both
    from the subchain and from the Gram-tensor chain (Prop. subchain Gram)."""
    S = tr.subchain_unfold2(tr.subchain(cores, n))
    P = tr.unfold_mode(X, n) @ S
    Q = S.T @ S
    return P, Q


def Q_chain(cores, n):
    Z = [tr.gram_tensor(G) for G in cores]
    return tr.h_unfold(tr.gram_chain([Z[k] for k in tr.chain_order(len(cores), n)]))


def grad_normal_eq(X, cores):
    """[G_{n(2)} Q_n - P_n folded to core layout for n = 1..N]."""
    out = []
    for n, G in enumerate(cores):
        P, _ = P_Q(X, cores, n)
        Q = Q_chain(cores, n)
        g2 = tr.core_unfold2(G) @ Q - P
        out.append(tr.core_fold2(g2, G.shape[0], G.shape[2]))
    return out


def grad_residual(X, cores):
    """[(TR(G) - X)_[n] G^{!=n}_[2] folded to core layout]."""
    E = tr.tr_reconstruct(cores) - X
    out = []
    for n, G in enumerate(cores):
        S = tr.subchain_unfold2(tr.subchain(cores, n))
        g2 = tr.unfold_mode(E, n) @ S
        out.append(tr.core_fold2(g2, G.shape[0], G.shape[2]))
    return out
