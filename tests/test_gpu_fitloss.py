"""GPU parity of the TR fit loss and its hand-written backward
(G_{n(2)} Q_n - P_n) against the FP64 oracle and finite differences."""

import numpy as np
import pytest

import workloads as W
from oracle import fitloss
from parity import dev

pytestmark = pytest.mark.gpu


def _torch_cores(cores, dtype):
    import torch
    return [torch.tensor(np.ascontiguousarray(G), dtype=dtype, device="cuda",
                         requires_grad=True) for G in cores]


def _run(P, X, cores, dtype):
    import torch
    from paper_2307_00719_amd.autograd import TRFitLoss
    Xt = torch.tensor(np.ascontiguousarray(X), dtype=dtype, device="cuda")
    ct = _torch_cores(cores, dtype)
    loss = TRFitLoss.apply(Xt, *ct)
    loss.backward()
    torch.cuda.synchronize()
    return float(loss), [c.grad.double().cpu().numpy() for c in ct]


@pytest.mark.parametrize("dims,ranks", [((6, 5, 7), (2, 3, 4)), ((9, 4, 5, 3), (3, 2, 2, 3)),
                                        ((17, 33, 6), (5, 4, 3))])
def test_fitloss_f64_parity(trlib, dims, ranks):
    cores, X = W.random_tr_problem(dims, ranks, 2, noise=0.3)
    pt = [G + 0.1 * np.random.default_rng(1).standard_normal(G.shape) for G in cores]
    loss, grads = _run(trlib, X, pt, __import__("torch").float64)
    ref_loss = fitloss.fit_loss(X, pt)
    ref = fitloss.grad_normal_eq(X, pt)
    print(f"[fitloss {dims}] loss rel {abs(loss - ref_loss) / ref_loss:.2e}", flush=True)
    assert abs(loss - ref_loss) <= 1e-11 * ref_loss
    for g, r in zip(grads, ref):
        assert dev(g, r) < 1e-10


def test_fitloss_finite_differences_gpu(trlib):
    """Central differences of the GPU loss itself (FP64) on the 8x8x8x4
    sub-instance of the c5 recipe."""
    import torch
    w = W.make("c5", dims=(8, 8, 8), T=4)
    point = W.c5_point(w)
    loss, grads = _run(trlib, w.X, point, torch.float64)
    r = np.random.default_rng(3)
    for k in range(4):
        for _ in range(3):
            idx = tuple(r.integers(0, s) for s in point[k].shape)
            h = 1e-6 * max(1.0, abs(point[k][idx]))
            cp = [c.copy() for c in point]
            cm = [c.copy() for c in point]
            cp[k][idx] += h
            cm[k][idx] -= h
            lp, _ = _run(trlib, w.X, cp, torch.float64)
            lm, _ = _run(trlib, w.X, cm, torch.float64)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][idx]) <= 1e-6 * max(1.0, abs(grads[k][idx]))


def test_fitloss_f32_c5_full(trlib):
    """FP32 forward/backward on the whole 64 x 64 x 64 x 50 evaluation (TR-ranks
    16) against the FP64 oracle's loss and G_{n(2)} Q_n - P_n: loss within
    1e-5 relative, every gradient entry within 1e-4 (parity.dev)."""
    import torch
    w = W.make("c5")
    point = W.c5_point(w)
    loss, grads = _run(trlib, w.X, point, torch.float32)
    ref_loss = fitloss.fit_loss(w.X, point)
    ref = fitloss.grad_normal_eq(w.X, point)
    devs = [dev(g, r) for g, r in zip(grads, ref)]
    print(f"[fitloss c5 f32] loss rel {abs(loss - ref_loss) / ref_loss:.2e} grads {devs}",
          flush=True)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert max(devs) < 1e-4


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("dims,ranks", [((20, 7, 9), (3, 3, 1)), ((19, 23, 5), (3, 2, 4)),
                                        ((5, 6, 7, 4), (2, 3, 2, 2))])
def test_mttkrp_and_gram_chain_entry_points(trlib, dt, dims, ranks):
    """tr_mttkrp and tr_gram_chain against P_n = X_[n] G^{!=n}_[2] and the
    explicit subchain Gram, for every mode."""
    import torch
    from oracle import tensor_ring as tr
    cores, X = W.random_tr_problem(dims, ranks, 4, noise=0.2)
    tdt = torch.float64 if dt == "f64" else torch.float32
    code = 0 if dt == "f64" else 1
    Xt = torch.from_numpy(np.asfortranarray(X)).to(tdt).cuda()
    ct = [torch.from_numpy(np.asfortranarray(G)).to(tdt).cuda() for G in cores]
    # Gram tensors in the paper's layout (R_{k+1} x R_k x R_{k+1} x R_k,
    # column-major), the input of tr_gram_chain
    Zt = [torch.from_numpy(np.asfortranarray(tr.gram_tensor(G)).ravel(order="F")).cuda()
          for G in cores]
    wsb = trlib.tr_workspace_bytes(list(dims), list(ranks), dt)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st_ = torch.cuda.current_stream().cuda_stream
    tol = 1e-12 if dt == "f64" else 2e-6
    for n in range(len(dims)):
        d = ranks[n] * ranks[(n + 1) % len(dims)]
        P = torch.zeros((dims[n], d), dtype=torch.float64, device="cuda")
        Q = torch.zeros((d, d), dtype=torch.float64, device="cuda")
        trlib.tr_mttkrp(list(dims), list(ranks), code, n, Xt.data_ptr(),
                        [c.data_ptr() for c in ct], P.data_ptr(), 0, ws.data_ptr(), wsb, st_)
        trlib.tr_gram_chain(list(dims), list(ranks), n, [z.data_ptr() for z in Zt],
                            Q.data_ptr(), 0, ws.data_ptr(), wsb, st_)
        Q2 = Q.clone()
        trlib.tr_gram_chain(list(dims), list(ranks), n, [z.data_ptr() for z in Zt],
                            Q2.data_ptr(), 1, ws.data_ptr(), wsb, st_)
        torch.cuda.synchronize()
        S = tr.subchain_unfold2(tr.subchain(cores, n))
        Pr, Qr = tr.unfold_mode(X, n) @ S, S.T @ S
        ep = dev(P.cpu().numpy(), Pr)
        eq = max(dev(Q.cpu().numpy(), Qr), dev(Q2.cpu().numpy(), 2 * Qr))
        print(f"[mttkrp {dims} n={n} {dt}] P {ep:.2e} Q {eq:.2e}", flush=True)
        assert ep < tol and eq < 1e-12


@pytest.mark.parametrize("dims,ranks", [((37, 45, 40, 33), (5, 7, 3, 6)),
                                        ((50, 64, 600), (4, 6, 5))])
def test_fitloss_f32_bulk_shapes(trlib, dims, ranks):
    """FP32 gradients through the formed-subchain MTTKRP (order <= 4, ranks
    <= 16, I_f <= 64, at least 32 rows, twice as many outer indices as
    workgroups): ragged row counts (37, 45, 40, 33; 600 = 9 full 64-row
    groups + 24), I_f below 64 (37, 45, 50: zero padded), unequal ranks, and
    every chain shape of orders 3 and 4 (U only, V only, both, two factors
    on one side).
    Loss within 1e-5 relative, gradients within 1e-4 (parity.dev)."""
    import torch
    cores, X = W.random_tr_problem(dims, ranks, 9, noise=0.3)
    pt = [G + 0.1 * np.random.default_rng(5).standard_normal(G.shape) for G in cores]
    loss, grads = _run(trlib, X, pt, torch.float32)
    ref_loss = fitloss.fit_loss(X, pt)
    ref = fitloss.grad_normal_eq(X, pt)
    devs = [dev(g, r) for g, r in zip(grads, ref)]
    print(f"[fitloss bulk {dims}] loss rel {abs(loss - ref_loss) / ref_loss:.2e} grads {devs}",
          flush=True)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert max(devs) < 1e-4
