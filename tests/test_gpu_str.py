"""GPU parity of the STR update (Alg. 4) through the C ABI against the FP64
oracle, on the same seeded inputs.

Tolerances (FP64 path): relative fit error within 1e-10 (relative) of the
oracle's after every batch; P_n, Q_n and cores within 1e-11 (1e-10 for the
cores of ragged shapes) entry by entry (parity.dev: each entry relative to
its own size or to the array's RMS size).  FP32-operand path (MTTKRP in
FP32 MFMA, everything else FP64): fit error within 1e-5 relative, P_n
within 1e-5, cores within 1e-4.
"""

import numpy as np
import pytest

import workloads as W
from parity import dev
from oracle import streaming as st

pytestmark = pytest.mark.gpu


def run_pair(P, X, init, t_init, t_new, nb, dt="f64", device_input=False, log="", sweeps=1):
    o = st.STR(X[..., :t_init], [G.copy() for G in init])
    g = P.TRStream(X[..., :t_init], init, compute_dtype=dt, sweeps=sweeps)
    worst = 0.0
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb, sweeps=sweeps)
        if device_input:
            import torch
            g.update(torch.from_numpy(np.asfortranarray(xb)).cuda())
        else:
            g.update(xb)
        T = t_init + (b + 1) * t_new
        eo = o.rel_error(X[..., :T])
        eg = g.reconstruct_error(X[..., :T])
        worst = max(worst, abs(eg - eo) / eo)
    out = dict(err_dev=worst, err=eg)
    gc = g.cores()
    out["cores"] = max(dev(a, b) for a, b in zip(gc, o.cores))
    pq = 0.0
    for n in range(X.ndim - 1):
        Pg, Qg = g.PQ(n)
        pq = max(pq, dev(Pg, o.P[n]), dev(Qg, o.Q[n]))
    out["PQ"] = pq
    g.close()
    print(f"[parity {log} {dt}] {out}", flush=True)
    return out


def _init(cores, t_init, noise, seed):
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    return W.perturb(init, noise, np.random.default_rng(seed))


def test_c1_parity_f64(trlib):
    w = W.make("c1", init_noise=1e-2)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, w.n_batches, log="c1")
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-11


SHAPES = [
    # (dims, ranks, t_init, t_new, nb): ragged sizes, several tiles, N = 3..5
    ((37, 23), (3, 4, 2), 9, 7, 3),
    ((70, 33), (2, 3, 5), 12, 3, 4),
    ((9, 7, 5), (2, 3, 2, 3), 8, 4, 3),
    ((5, 4, 3, 3), (2, 2, 3, 2, 2), 6, 2, 3),
    ((130, 17), (1, 2, 1), 5, 5, 2),
    ((21, 19), (5, 4, 6), 40, 11, 2),
    # Q of 42 x 42 and 49 x 49: three and four ragged 16 x 16 tiles a side
    ((24, 22), (7, 6, 7), 20, 6, 2),
    # R_p = 8 with R_{p+1} = 7 and 8: the Gram workgroups of the fused launch
    # also form the chain product's columns (odd R_{p+1}: a partial last tile)
    ((19, 21), (8, 7, 8), 12, 5, 3),
    # Q of 72 x 72 to 90 x 90 (d > 64): past the fused per-mode launch, so the
    # side kernel (its own Gram tile workgroups, chain, upper-triangle inverse)
    # runs on the second stream
    ((20, 18), (9, 8, 10), 25, 6, 2),
    # order 4 with d = 81..90: three Gram factors chained through the side
    # kernel's two ping-pong buffers
    ((6, 5, 7), (9, 9, 10, 9), 12, 3, 3),
]


@pytest.mark.parametrize("dims,ranks,t_init,t_new,nb", SHAPES)
def test_parity_shapes_f64(trlib, dims, ranks, t_init, t_new, nb):
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, 11, noise=0.05)
    init = _init(cores, t_init, 0.05, 3)
    r = run_pair(trlib, X, init, t_init, t_new, nb, log=str(dims))
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-10


def test_exact_recovery_gpu(trlib):
    dims, ranks = (33, 29), (3, 2, 4)
    cores, X = W.random_tr_problem(dims + (30,), ranks, 5)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :10, :]
    g = trlib.TRStream(X[..., :10], init)
    for b in range(4):
        g.update(X[..., 10 + 5 * b:15 + 5 * b])
    assert g.reconstruct_error(X) < 1e-12


def test_c1_parity_f32(trlib):
    w = W.make("c1", init_noise=1e-2)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, w.n_batches, dt="f32", log="c1")
    assert r["err_dev"] < 1e-5 and r["PQ"] < 1e-5 and r["cores"] < 1e-4


def test_device_input_and_cast(trlib):
    w = W.make("c1", init_noise=1e-2)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, device_input=True, log="dev")
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11
    # an FP32 device batch is cast up for the FP64 path
    import torch
    g = trlib.TRStream(w.X_init(), w.cores_init)
    o = st.STR(w.X_init(), [G.copy() for G in w.cores_init])
    xb = w.batch(0).astype(np.float32)
    g.update(torch.from_numpy(np.asfortranarray(xb)).cuda())
    o.update(xb.astype(np.float64))
    assert max(dev(a, b) for a, b in zip(g.cores(), o.cores)) < 1e-11


def test_c2_full_size_parity(trlib):
    """The full 256 x 256 slices, t_new = 20, in the launch configuration the
    benchmark times; the oracle follows every batch."""
    w = W.make("c2", T=160, init_noise=1e-3)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, log="c2")
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-10
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, dt="f32", log="c2")
    assert r["err_dev"] < 1e-5 and r["PQ"] < 1e-5 and r["cores"] < 1e-4


def test_get_cores_roundtrip_and_determinism(trlib):
    w = W.make("c1", init_noise=1e-2)
    g = trlib.TRStream(w.X_init(), w.cores_init)
    for a, b in zip(g.cores(), w.cores_init):
        assert np.array_equal(a, b)
    h = trlib.TRStream(w.X_init(), w.cores_init)
    for b in range(3):
        g.update(w.batch(b))
        h.update(w.batch(b))
    for a, b in zip(g.cores(), h.cores()):
        assert np.array_equal(a, b)


def test_zero_batch(trlib):
    w = W.make("c1", init_noise=1e-2)
    g = trlib.TRStream(w.X_init(), w.cores_init)
    g.update(w.batch(0))
    before = g.cores()
    P0 = [g.PQ(n) for n in range(2)]
    g.update(np.zeros_like(w.batch(1), order="F"))
    after = g.cores()
    assert np.all(after[-1][:, -w.t_new:, :] == 0)
    for n in range(2):
        P1, Q1 = g.PQ(n)
        assert np.array_equal(P1, P0[n][0]) and np.allclose(Q1, P0[n][1], rtol=0, atol=0)
        assert dev(after[n], before[n]) < 1e-12


def test_nonfinite_and_bad_arguments(trlib):
    w = W.make("c1", init_noise=1e-2)
    g = trlib.TRStream(w.X_init(), w.cores_init)
    bad = w.batch(0).copy(order="F")
    bad[3, 4, 1] = np.nan
    with pytest.raises(trlib.TRError) as e:
        g.update(bad)
    assert e.value.status == "TR_ERR_NONFINITE"
    assert g.num_slices() == w.t_init
    g.update(w.batch(0))                       # the handle is still usable
    assert g.num_slices() == w.t_init + w.t_new
    with pytest.raises(trlib.TRError) as e:
        g.reconstruct_error(w.X[..., :w.t_init])
    assert e.value.status == "TR_ERR_SHAPE"
    import torch
    d = trlib.TRStream(w.X_init(), w.cores_init, check_finite=True)
    xb = torch.from_numpy(np.asfortranarray(bad)).cuda()
    with pytest.raises(trlib.TRError):
        d.update(xb)
    assert d.num_slices() == w.t_init


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_order4_c3_shape(trlib, dt):
    """The 64 x 64 x 64 stream with TR-ranks 10 (d = 100 for every mode, the
    two-stream path with an order-4 Gram chain) over three batches of 10."""
    w = W.make("c3", T=70, init_noise=1e-3)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, dt=dt, log="c3 order 4")
    if dt == "f64":
        assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-10
    else:
        assert r["err_dev"] < 1e-5 and r["PQ"] < 1e-5 and r["cores"] < 1e-4


MULTI = [
    ((20, 20), (3, 3, 3), 10, 5, 3, 3),
    ((9, 7, 5), (2, 3, 2, 3), 8, 4, 2, 2),
    ((20, 18), (9, 8, 10), 25, 6, 2, 2),      # d > 64: the two-stream path
]


@pytest.mark.parametrize("dims,ranks,t_init,t_new,nb,sweeps", MULTI)
def test_multi_pass_updates(trlib, dims, ranks, t_init, t_new, nb, sweeps):
    """Several passes over each batch (the extension of Sec. 3.1's split
    P_n = P_n^old + P_n^new): every pass restarts from the P_n, Q_n held
    before the batch, against the oracle's STR.update(sweeps=...)."""
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, 17, noise=0.05)
    init = _init(cores, t_init, 0.05, 4)
    r = run_pair(trlib, X, init, t_init, t_new, nb, log=f"{dims} x{sweeps}", sweeps=sweeps)
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-10
    one = run_pair(trlib, X, init, t_init, t_new, nb, log=f"{dims} x1")
    assert r["err"] != one["err"]


def test_tensor_train_stream_c2_size(trlib):
    """Streaming tensor train (the remark after Alg. 4: R_1 = 1 makes the TR
    a TT): the 256 x 256 stream with TT-ranks (1, 8, 8), so the temporal
    core's rows have R_N R_1 = 8 entries and mode 1's d = R_1 R_2 = 8, in the
    benchmark's launch configuration, over three batches of 20."""
    dims, ranks, t_init, t_new, nb = (256, 256), (1, 8, 8), 100, 20, 3
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(dims + (T,), ranks, 23, noise=0.01)
    init = _init(cores, t_init, 1e-3, 5)
    r = run_pair(trlib, X, init, t_init, t_new, nb, log="TT c2")
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-11 and r["cores"] < 1e-10
    r = run_pair(trlib, X, init, t_init, t_new, nb, dt="f32", log="TT c2")
    assert r["err_dev"] < 1e-5 and r["PQ"] < 1e-5 and r["cores"] < 1e-4


def test_tensor_train_exact_recovery(trlib):
    cores, X = W.random_tr_problem((40, 30, 25), (1, 4, 3), 8)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :10, :]
    g = trlib.TRStream(X[..., :10], init)
    for b in range(3):
        g.update(X[..., 10 + 5 * b:15 + 5 * b])
    assert g.reconstruct_error(X) < 1e-12
    g.close()
