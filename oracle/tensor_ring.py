"""Tensor-ring primitives written out from their definitions (Sec. 1 and 2).

TEST INFRASTRUCTURE (CPU oracle).  Plain FP64 NumPy; nothing here is tuned.

Every array index is 0-based.  A TR-core G_n has shape (R_n, I_n, R_{n+1})
and lateral slice G_n(i) = G_n[:, i, :] (Sec. 1).  When a tensor is flattened
its first index runs fastest: this is the paper's multi-index
  overline(i_1 ... i_N) = 1 + sum_n (i_n - 1) prod_{j<n} I_j
(Sec. 2, opening paragraph), shifted to 0-based.
"""

import itertools

import numpy as np


# ---------------------------------------------------------------------------
# Multi-index and unfoldings (Sec. 2, opening paragraph and Def. of unfoldings)
# ---------------------------------------------------------------------------

def lin(idx, dims):
    """0-based multi-index with the first index fastest (Sec. 2)."""
    out, stride = 0, 1
    for i, d in zip(idx, dims):
        out += int(i) * stride
        stride *= int(d)
    return out


def _unfold(X, row_axes, col_axes):
    """Matrix with rows lin(row_axes) and columns lin(col_axes), first listed
    axis fastest in each, as every unfolding of Sec. 2 is defined."""
    rows = int(np.prod([X.shape[a] for a in row_axes])) if row_axes else 1
    Y = np.transpose(X, list(row_axes) + list(col_axes))
    return Y.reshape(rows, -1, order="F")


def unfold_classical(X, n):
    """Classical mode-n unfolding X_(n): row i_n, column
    lin(i_1..i_{n-1}, i_{n+1}..i_N) (Sec. 2, Def. of unfoldings)."""
    N = X.ndim
    return _unfold(X, [n], [k for k in range(N) if k != n])


def unfold_mode(X, n):
    """Mode-n unfolding X_[n]: row i_n, column lin(i_{n+1}..i_N, i_1..i_{n-1})
    -- the cyclic order (Sec. 2, Def. of unfoldings)."""
    N = X.ndim
    return _unfold(X, [n], list(range(n + 1, N)) + list(range(0, n)))


def unfold_n(X, n):
    """n-unfolding X_<n>: rows lin(i_1..i_n), columns lin(i_{n+1}..i_N)
    (Sec. 2, Def. of unfoldings); ``n`` counts leading modes (1-based)."""
    return _unfold(X, list(range(n)), list(range(n, X.ndim)))


def fold_mode(M, n, shape):
    """Inverse of ``unfold_mode`` for a tensor of the given shape."""
    N = len(shape)
    order = [n] + list(range(n + 1, N)) + list(range(0, n))
    Y = M.reshape([shape[a] for a in order], order="F")
    return np.transpose(Y, np.argsort(order))


def ttm(X, U, n):
    """Tensor-times-matrix X x_n U, U of shape (J, I_n) (Sec. 2, Def. TTM):
    (X x_n U)(.., j, ..) = sum_{i_n} X(.., i_n, ..) U(j, i_n)."""
    Y = np.tensordot(U, X, axes=([1], [n]))      # j first
    return np.moveaxis(Y, 0, n)


# ---------------------------------------------------------------------------
# TR format (Sec. 1)
# ---------------------------------------------------------------------------

def tr_entry(cores, idx):
    """X(i_1..i_N) = Trace(G_1(i_1) G_2(i_2) ... G_N(i_N)) (Sec. 1)."""
    M = np.eye(cores[0].shape[0])
    for G, i in zip(cores, idx):
        M = M @ G[:, i, :]
    return float(np.trace(M))


def tr_full_bruteforce(cores):
    """Whole TR tensor by evaluating the trace formula entry by entry.
    For tiny tensors only (pure-Python loop)."""
    dims = [G.shape[1] for G in cores]
    X = np.empty(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        X[idx] = tr_entry(cores, idx)
    return X


def core_unfold2(G):
    """Classical mode-2 unfolding of a core, G_{n(2)}: row i, column r + R_n*s
    holds G_n[r, i, s] (Sec. 2, Def. of unfoldings, applied to a 3rd-order
    tensor)."""
    return unfold_classical(G, 1)


def core_fold2(G2, Rn, Rn1):
    """Inverse of ``core_unfold2``: G[r, i, s] = G2[i, r + Rn*s]."""
    I = G2.shape[0]
    return np.ascontiguousarray(
        np.transpose(G2.reshape(I, Rn, Rn1, order="F"), (1, 0, 2)))


# ---------------------------------------------------------------------------
# Products of Sec. 2
# ---------------------------------------------------------------------------

def outer(A, B):
    """Outer product A o B (Sec. 2, Def. outer product)."""
    return np.multiply.outer(A, B)


def contract_2413(A, B):
    """General contracted tensor product A x_{2,4}^{1,3} B of
    A (I1 x J x R1 x K) and B (J x I2 x K x R2) (Sec. 2, Def. general
    contracted tensor product):
        (A x B)(i1, i2, r1, r2) = sum_{j,k} A(i1, j, r1, k) B(j, i2, k, r2)."""
    return np.einsum("ajrk,jbks->abrs", A, B)


def subchain_product(A, B):
    """Mode-2 subchain product A [x]_2 B of A (I1 x J1 x K) and B (K x J2 x I2)
    (Sec. 2, Def. subchain product): slice lin(j1, j2) is A(j1) B(j2), with j1
    fastest."""
    I1, J1, _ = A.shape
    _, J2, I2 = B.shape
    C = np.einsum("ajk,kbc->ajbc", A, B)           # [a, j1, j2, c]
    return C.reshape(I1, J1 * J2, I2, order="F")


def slices_hadamard(A, B):
    """Mode-2 slices-Hadamard product A (*)_2 B: slice j is A(j) B(j)
    (Sec. 2, Def. slices-Hadamard product)."""
    return np.einsum("ajk,kjc->ajc", A, B)


def subchain(cores, n):
    """Subchain tensor G^{!=n} of shape (R_{n+1}, prod_{j!=n} I_j, R_n): slice
    lin(i_{n+1}..i_N, i_1..i_{n-1}) is
        G_{n+1}(i_{n+1}) ... G_N(i_N) G_1(i_1) ... G_{n-1}(i_{n-1})
    (Sec. 2, Def. subchain tensor), built as the chain of subchain products
    G_{n+1} [x]_2 ... [x]_2 G_N [x]_2 G_1 [x]_2 ... [x]_2 G_{n-1}
    (eq. subchain_new in Sec. 3.1)."""
    N = len(cores)
    order = list(range(n + 1, N)) + list(range(0, n))
    T = cores[order[0]]
    for k in order[1:]:
        T = subchain_product(T, cores[k])
    return T


def subchain_bruteforce(cores, n):
    """Same tensor as ``subchain`` but evaluated slice by slice from the
    definition (pure-Python loop; tiny inputs only)."""
    N = len(cores)
    order = list(range(n + 1, N)) + list(range(0, n))
    dims = [cores[k].shape[1] for k in order]
    J = int(np.prod(dims))
    out = np.empty((cores[n].shape[2], J, cores[n].shape[0]))
    for idx in itertools.product(*[range(d) for d in reversed(dims)]):
        idx = idx[::-1]                         # first listed index fastest
        M = np.eye(cores[order[0]].shape[0])
        for k, i in zip(order, idx):
            M = M @ cores[k][:, i, :]
        out[:, lin(idx, dims), :] = M
    return out


def subchain_unfold2(T):
    """Mode-2 unfolding T_[2] of a (R_{n+1} x J x R_n) subchain tensor: row j,
    column r + R_n*s holds T[s, j, r] (Sec. 2, Def. of unfoldings)."""
    return unfold_mode(T, 1)


# ---------------------------------------------------------------------------
# Gram tensors and their chains (Alg. 2, Prop. subchain Gram)
# ---------------------------------------------------------------------------

def gram_tensor(G):
    """Z = sum_i G(i)^T o G(i)^T of shape (R_{n+1}, R_n, R_{n+1}, R_n)
    (Alg. 2, second step; Alg. 4 initialisation):
        Z[a, b, c, d] = sum_i G[b, i, a] G[d, i, c]."""
    Z = 0.0
    for i in range(G.shape[1]):
        Gt = G[:, i, :].T
        Z = Z + outer(Gt, Gt)
    return Z


def gram_chain(Zs):
    """Left-to-right chain Zs[0] x_{2,4}^{1,3} Zs[1] x ... (Alg. 2, Alg. 4)."""
    H = Zs[0]
    for Z in Zs[1:]:
        H = contract_2413(H, Z)
    return H


def chain_order(N, n):
    """Order of Gram tensors in H^{!=n}: Z_{n-1} .. Z_1, Z_N .. Z_{n+1}
    (Alg. 2, H^{!=n}; Alg. 4 initialisation of Q_n), 0-based."""
    return list(range(n - 1, -1, -1)) + list(range(N - 1, n, -1))


def h_unfold(H):
    """H_<2>: the 2-unfolding of a 4th-order Gram chain (Prop. subchain Gram);
    its row/column order is that of G_{n(2)}'s columns."""
    return unfold_n(H, 2)


def tr_reconstruct(cores):
    """Whole tensor via the identity X_[N] = G_{N(2)} (G^{!=N}_[2])^T, the
    basis of the ALS subproblem (eq. tr_als in Sec. 2).  Cross-checked against
    ``tr_full_bruteforce`` in the oracle tests."""
    N = len(cores)
    S = subchain_unfold2(subchain(cores, N - 1))
    XN = core_unfold2(cores[N - 1]) @ S.T
    shape = [G.shape[1] for G in cores]
    return fold_mode(XN, N - 1, shape)


def rel_error(X, cores):
    """Relative error ||X - TR(G)||_F / ||X||_F by direct reconstruction
    (Sec. 4, the error measure of the experimental protocol)."""
    E = X - tr_reconstruct(cores)
    return float(np.linalg.norm(E.ravel()) / np.linalg.norm(X.ravel()))
