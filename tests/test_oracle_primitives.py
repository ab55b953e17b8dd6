"""Pins of the oracle's tensor primitives (Sec. 1-2) against brute force,
closed forms and textbook identities."""

import itertools

import numpy as np
import pytest

from oracle import tensor_ring as tr
import workloads as W


def _cores(dims, ranks, seed=0):
    r = np.random.default_rng(seed)
    N = len(dims)
    return [r.standard_normal((ranks[n], dims[n], ranks[(n + 1) % N])) for n in range(N)]


# all sizes distinct so that a transposed index cannot pass
CASES = [((3, 4, 5), (2, 3, 4)), ((3, 2, 4, 5), (2, 3, 2, 4)), ((2, 3, 2, 3, 2), (2, 1, 3, 2, 2))]


def test_lin_index_first_fastest():
    dims = (3, 4, 5)
    X = np.arange(60.0).reshape(dims, order="F")
    for idx in itertools.product(range(3), range(4), range(5)):
        assert X[idx] == tr.lin(idx, dims)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_unfoldings_elementwise(dims, ranks):
    X = np.random.default_rng(1).standard_normal(dims)
    N = len(dims)
    for n in range(N):
        Xc, Xm = tr.unfold_classical(X, n), tr.unfold_mode(X, n)
        cyc = list(range(n + 1, N)) + list(range(n))
        rest = [k for k in range(N) if k != n]
        for idx in itertools.product(*[range(d) for d in dims]):
            j_cls = tr.lin([idx[k] for k in rest], [dims[k] for k in rest])
            j_cyc = tr.lin([idx[k] for k in cyc], [dims[k] for k in cyc])
            assert Xc[idx[n], j_cls] == X[idx]
            assert Xm[idx[n], j_cyc] == X[idx]
        for m in range(1, N):
            Xn = tr.unfold_n(X, m)
            idx = tuple(d - 1 for d in dims)
            assert Xn[tr.lin(idx[:m], dims[:m]), tr.lin(idx[m:], dims[m:])] == X[idx]
        assert np.array_equal(tr.fold_mode(Xm, n, dims), X)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_tr_reconstruction_matches_trace_bruteforce(dims, ranks):
    cores = _cores(dims, ranks)
    Xb = tr.tr_full_bruteforce(cores)
    assert np.allclose(tr.tr_reconstruct(cores), Xb, rtol=0, atol=1e-12 * np.abs(Xb).max())
    # the input generator's synthesis is pinned to the same definition
    assert np.allclose(W.synthesize_tr(cores), Xb, rtol=0, atol=1e-12 * np.abs(Xb).max())


@pytest.mark.parametrize("dims,ranks", CASES)
def test_subchain_matches_definition(dims, ranks):
    cores = _cores(dims, ranks)
    for n in range(len(dims)):
        assert np.allclose(tr.subchain(cores, n), tr.subchain_bruteforce(cores, n), atol=1e-12)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_unfolding_identity(dims, ranks):
    """X_[n] = G_{n(2)} (G^{!=n}_[2])^T for X = TR(G) (eq. tr_als)."""
    cores = _cores(dims, ranks)
    X = tr.tr_full_bruteforce(cores)
    for n in range(len(dims)):
        S = tr.subchain_unfold2(tr.subchain_bruteforce(cores, n))
        lhs = tr.unfold_mode(X, n)
        rhs = tr.core_unfold2(cores[n]) @ S.T
        assert np.allclose(lhs, rhs, atol=1e-12 * np.abs(lhs).max())


@pytest.mark.parametrize("dims,ranks", CASES)
def test_prop_subchain_gram(dims, ranks):
    """Prop. subchain Gram: the contracted chain of Gram tensors equals the
    explicit Gram of the subchain, in G_{n(2)}'s column order."""
    cores = _cores(dims, ranks)
    Z = [tr.gram_tensor(G) for G in cores]
    for n in range(len(dims)):
        S = tr.subchain_unfold2(tr.subchain_bruteforce(cores, n))
        H = tr.h_unfold(tr.gram_chain([Z[k] for k in tr.chain_order(len(dims), n)]))
        ref = S.T @ S
        assert np.allclose(H, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_gram_tensor_elementwise():
    G = np.random.default_rng(3).standard_normal((2, 5, 3))
    Z = tr.gram_tensor(G)
    for a, b, c, d in itertools.product(range(3), range(2), range(3), range(2)):
        assert np.isclose(Z[a, b, c, d], sum(G[b, i, a] * G[d, i, c] for i in range(5)))


def test_contract_2413_elementwise():
    r = np.random.default_rng(4)
    A = r.standard_normal((2, 3, 4, 5))
    B = r.standard_normal((3, 6, 5, 7))
    C = tr.contract_2413(A, B)
    for i1, i2, r1, r2 in itertools.product(range(2), range(6), range(4), range(7)):
        ref = sum(A[i1, j, r1, k] * B[j, i2, k, r2] for j in range(3) for k in range(5))
        assert np.isclose(C[i1, i2, r1, r2], ref)


def test_subchain_and_hadamard_products_slicewise():
    r = np.random.default_rng(5)
    A = r.standard_normal((2, 3, 4))
    B = r.standard_normal((4, 5, 3))
    C = tr.subchain_product(A, B)
    for j1, j2 in itertools.product(range(3), range(5)):
        assert np.allclose(C[:, j1 + 3 * j2, :], A[:, j1, :] @ B[:, j2, :])
    B2 = r.standard_normal((4, 3, 2))
    D = tr.slices_hadamard(A, B2)
    for j in range(3):
        assert np.allclose(D[:, j, :], A[:, j, :] @ B2[:, j, :])


def test_rank_one_ring_is_outer_product():
    """R = 1: TR(G) is the outer product of the core fibres, and the Gram
    chain is the product of squared norms."""
    dims = (3, 4, 5)
    cores = _cores(dims, (1, 1, 1), seed=7)
    vecs = [G[0, :, 0] for G in cores]
    X = np.einsum("i,j,k->ijk", *vecs)
    assert np.allclose(tr.tr_full_bruteforce(cores), X)
    Z = [tr.gram_tensor(G) for G in cores]
    H = tr.h_unfold(tr.gram_chain([Z[k] for k in tr.chain_order(3, 0)]))
    assert np.isclose(H[0, 0], np.dot(vecs[1], vecs[1]) * np.dot(vecs[2], vecs[2]))


def test_diagonal_cores_give_cp_sum():
    """Diagonal slices: Trace(prod diag) = sum_r prod_n u_{n,r}(i_n)."""
    r = np.random.default_rng(8)
    dims, R = (3, 4, 2, 5), 3
    U = [r.standard_normal((R, d)) for d in dims]
    cores = []
    for u in U:
        G = np.zeros((R, u.shape[1], R))
        for k in range(R):
            G[k, :, k] = u[k]
        cores.append(G)
    X = np.einsum("ra,rb,rc,rd->abcd", *U)
    assert np.allclose(tr.tr_full_bruteforce(cores), X)


def test_ttm_multi_mode_identity():
    """Y = X x_1 U_1 ... x_N U_N has Y_[n] = U_n X_[n] (U_{n-1} (x) .. U_1 (x)
    U_N (x) .. U_{n+1})^T (Sec. 2, Multi-TTM)."""
    r = np.random.default_rng(9)
    dims = (3, 4, 2)
    X = r.standard_normal(dims)
    Us = [r.standard_normal((d + 1, d)) for d in dims]
    Y = X
    for n, U in enumerate(Us):
        Y = tr.ttm(Y, U, n)
    N = 3
    for n in range(N):
        order = list(range(n - 1, -1, -1)) + list(range(N - 1, n, -1))
        K = np.ones((1, 1))
        for k in order:
            K = np.kron(K, Us[k])
        assert np.allclose(tr.unfold_mode(Y, n), Us[n] @ tr.unfold_mode(X, n) @ K.T)


def test_ttm_elementwise():
    r = np.random.default_rng(10)
    X = r.standard_normal((3, 4, 2))
    U = r.standard_normal((5, 4))
    Y = tr.ttm(X, U, 1)
    for i, j, k in itertools.product(range(3), range(5), range(2)):
        assert np.isclose(Y[i, j, k], sum(X[i, q, k] * U[j, q] for q in range(4)))
