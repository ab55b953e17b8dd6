"""Checkpoint / resume and sample injection through the C ABI.

* tr_stream_save + tr_stream_load: a stream resumed from a file continues
  bit for bit like the uninterrupted stream (same kernels, same fixed-order
  reductions), for STR and the three sketches, orders 3 and 4.
* tr_stream_set_samples: indices injected on both sides (GPU and the FP64
  oracle) replace the generator's draw for the next update; the results
  then agree with the oracle to the parity tolerances of the randomized
  tests (FP64: 1e-10 relative).
"""

import numpy as np
import pytest

import workloads as W
from parity import dev
from oracle import randomized as rs

pytestmark = pytest.mark.gpu




def _problem(dims, ranks, t_init, nb, t_new, seed):
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, seed, noise=0.05)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    return W.perturb(init, 0.05, np.random.default_rng(seed + 1)), X


CKPT = [
    (None, (14, 12), (2, 3, 2), "f64"),
    (None, (9, 8, 7), (2, 3, 2, 2), "f64"),
    (None, (14, 12), (2, 3, 2), "f32"),
    ("uniform", (14, 12), (2, 3, 2), "f64"),
    ("leverage", (30, 25), (2, 2, 2), "f64"),
    ("ksrft", (14, 12), (2, 3, 2), "f64"),
    ("ksrft", (9, 8, 7), (2, 3, 2, 2), "bf16"),
]


@pytest.mark.parametrize("sketch,dims,ranks,dt", CKPT)
def test_save_load_resumes_bitwise(trlib, tmp_path, sketch, dims, ranks, dt):
    t_init, t_new, nb, m = 8, 4, 4, 60
    init, X = _problem(dims, ranks, t_init, nb, t_new, 11)
    kw = dict(compute_dtype=dt, sketch=sketch, sketch_size=m if sketch else 0)
    batch = lambda b: X[..., t_init + b * t_new:t_init + (b + 1) * t_new]  # noqa: E731
    print(f"[ckpt] sketch={sketch} dims={dims} ranks={ranks} dt={dt}", flush=True)
    g1 = trlib.TRStream(X[..., :t_init], init, seed=5, **kw)
    for b in range(2):
        g1.update(batch(b))
    path = str(tmp_path / "state.trs")
    g1.save(path)
    g2 = trlib.TRStream.load(path, dims, ranks, **kw)
    assert g2.num_slices() == g1.num_slices() == t_init + 2 * t_new
    for b in range(2, nb):
        g1.update(batch(b))
        g2.update(batch(b))
    for a, c in zip(g1.cores(), g2.cores()):
        assert np.array_equal(a, c)
    for n in range(len(ranks) - 1):
        for a, c in zip(g1.PQ(n), g2.PQ(n)):
            assert np.array_equal(a, c)
    if sketch:
        assert np.array_equal(g1.samples(), g2.samples())
    T = t_init + nb * t_new
    assert g1.reconstruct_error(X[..., :T]) == g2.reconstruct_error(X[..., :T])
    g1.close()
    g2.close()


def test_load_rejects_other_shape_and_altered_file(trlib, tmp_path):
    init, X = _problem((14, 12), (2, 3, 2), 8, 1, 4, 3)
    g = trlib.TRStream(X[..., :8], init)
    path = tmp_path / "s.trs"
    g.save(str(path))
    g.close()
    with pytest.raises(trlib.TRError) as e:
        trlib.TRStream.load(str(path), (14, 12), (2, 2, 2))
    assert e.value.code == 2
    with pytest.raises(trlib.TRError) as e:
        trlib.TRStream.load(str(path), (14, 12), (2, 3, 2), compute_dtype="f32")
    assert e.value.code == 2
    raw = bytearray(path.read_bytes())
    raw[-9] ^= 0x40                               # one bit of the last Gram matrix
    bad = tmp_path / "bad.trs"
    bad.write_bytes(bytes(raw))
    with pytest.raises(trlib.TRError) as e:
        trlib.TRStream.load(str(bad), (14, 12), (2, 3, 2))
    assert e.value.code == 1
    short = tmp_path / "short.trs"
    short.write_bytes(bytes(raw[:-100]))
    with pytest.raises(trlib.TRError) as e:
        trlib.TRStream.load(str(short), (14, 12), (2, 3, 2))
    assert e.value.code == 1
    h = trlib.TRStream.load(str(path), (14, 12), (2, 3, 2))
    assert h.num_slices() == 8
    h.close()


def _inject(o, g, S):
    g.set_samples(S)
    N = o.N
    for k in range(N):
        o.idxs[k] = S[k].astype(np.int64)
    if o.sketch != "ksrft":
        for k in range(N - 1):
            o.GS[k] = o._gather(k, o.cores[k])


@pytest.mark.parametrize("sketch,dims,ranks", [
    ("uniform", (20, 18), (3, 2, 3)),
    ("leverage", (40, 30), (2, 2, 2)),
    ("ksrft", (12, 10, 6), (2, 2, 3, 2)),
])
def test_injected_samples_match_oracle(trlib, sketch, dims, ranks):
    t_init, t_new, nb, m = 8, 5, 3, 50
    init, X = _problem(dims, ranks, t_init, nb, t_new, 21)
    N = len(ranks)
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch=sketch, seed=9)
    g = trlib.TRStream(X[..., :t_init], init, sketch=sketch, sketch_size=m, seed=9)
    rng = np.random.default_rng(2024)
    sizes = list(dims) + [t_init]
    for b in range(nb):
        S = np.stack([rng.integers(0, sizes[k], m) for k in range(N)]).astype(np.int32)
        assert not np.array_equal(S, g.samples())
        _inject(o, g, S)
        assert np.array_equal(g.samples(), S)
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
        sizes[-1] = t_new
        sg = g.samples()
        assert all(np.array_equal(sg[k], o.idxs[k]) for k in range(N))
    T = t_init + nb * t_new
    eo, eg = o.rel_error(X[..., :T]), g.reconstruct_error(X[..., :T])
    cores = max(dev(a, c) for a, c in zip(g.cores(), o.cores))
    pq = max(max(dev(g.PQ(n)[0], o.P[n].real), dev(g.PQ(n)[1], o.Q[n].real))
             for n in range(N - 1))
    print(f"[inject {sketch}] err dev {abs(eg - eo) / eo:.2e} cores {cores:.2e} PQ {pq:.2e}",
          flush=True)
    assert abs(eg - eo) <= 1e-10 * eo and cores < 1e-9 and pq < 1e-10
    g.close()


def test_set_samples_rejects_out_of_range(trlib):
    init, X = _problem((14, 12), (2, 3, 2), 8, 1, 4, 4)
    g = trlib.TRStream(X[..., :8], init, sketch="uniform", sketch_size=30, seed=1)
    before = g.samples()
    S = before.copy()
    S[0, 3] = 14                                  # core 0 has 14 indices
    with pytest.raises(trlib.TRError) as e:
        g.set_samples(S)
    assert e.value.code == 1
    S = before.copy()
    S[2, 0] = 8                                   # the temporal block has 8 slices
    with pytest.raises(trlib.TRError):
        g.set_samples(S)
    S[2, 0] = -1
    with pytest.raises(trlib.TRError):
        g.set_samples(S)
    assert np.array_equal(g.samples(), before)
    g.close()
    h = trlib.TRStream(X[..., :8], init)
    with pytest.raises(trlib.TRError):
        h.set_samples(before)
    h.close()


def test_injected_signs_match_oracle(trlib):
    """KSRFT with the D_k of each step injected on both sides (the sign
    diagonals of Def. KSRFT taken from outside instead of the generator):
    the results agree with the oracle to the FP64 parity tolerances, and
    differ from the run with the generator's signs."""
    dims, ranks, t_init, t_new, nb, m = (12, 10, 6), (2, 2, 3, 2), 8, 5, 3, 50
    init, X = _problem(dims, ranks, t_init, nb, t_new, 23)
    N = len(ranks)
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch="ksrft", seed=3)
    g = trlib.TRStream(X[..., :t_init], init, sketch="ksrft", sketch_size=m, seed=3)
    h = trlib.TRStream(X[..., :t_init], init, sketch="ksrft", sketch_size=m, seed=3)
    rng = np.random.default_rng(99)
    sizes = list(dims) + [t_new]
    for b in range(nb):
        D = [np.where(rng.random(sizes[k]) < 0.5, 1, -1).astype(np.int8) for k in range(N)]
        g.set_samples(signs=D)
        o.set_samples(signs=D)
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
        h.update(xb)
        sg = g.samples()
        assert all(np.array_equal(sg[k], o.idxs[k]) for k in range(N))
    T = t_init + nb * t_new
    eo, eg, eh = (o.rel_error(X[..., :T]), g.reconstruct_error(X[..., :T]),
                  h.reconstruct_error(X[..., :T]))
    cores = max(dev(a, c) for a, c in zip(g.cores(), o.cores))
    pq = max(max(dev(g.PQ(n)[0], o.P[n].real), dev(g.PQ(n)[1], o.Q[n].real))
             for n in range(N - 1))
    print(f"[inject signs] err gpu {eg:.10e} oracle {eo:.10e} generator {eh:.10e} "
          f"cores {cores:.2e} PQ {pq:.2e}", flush=True)
    assert abs(eg - eo) <= 1e-10 * eo and cores < 1e-9 and pq < 1e-10
    assert eg != eh
    # a temporal sign vector that does not match the next batch is refused
    D = [np.ones(sizes[k], dtype=np.int8) for k in range(N - 1)] + [np.ones(3, dtype=np.int8)]
    g.set_samples(signs=D)
    with pytest.raises(trlib.TRError) as e:
        g.update(X[..., :t_new])
    assert e.value.code == 2
    bad = [d.copy() for d in D]
    bad[0][0] = 0
    with pytest.raises(trlib.TRError) as e:
        g.set_samples(signs=bad)
    assert e.value.code == 1
    g.close()
    h.close()
    u = trlib.TRStream(X[..., :t_init], init, sketch="uniform", sketch_size=m, seed=3)
    with pytest.raises(trlib.TRError):
        u.set_samples(signs=D)
    u.close()
