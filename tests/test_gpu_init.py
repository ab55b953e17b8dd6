"""The GPU initialiser and the batch solver: batch TR-ALS with normal
equations (Alg. 2) on the device against the FP64 oracle's ``tr_als_ne``,
both started from the same counter-based random cores (Irwin-Hall normals,
stream kind 2 of the seed; ``oracle.rng.init_cores`` on the host).

* tr_stream_init with no cores: the sweeps run, the error after each, the
  stopping sweep and the cores agree with the oracle; the stream then tracks
  like the oracle's STR started from the oracle's cores;
* tr_batch_als: a cold start, and the warm ("Hot") start from given cores
  over all slices seen so far, the batch reference of Sec. 4.

ALS is deterministic, so the two sides follow the same iterates up to
rounding; the tolerances are those of the STR parity tests (1e-10 on the
errors, 1e-9 entry by entry on the cores).
"""

import numpy as np
import pytest

import workloads as W
from oracle import batch_als, rng, streaming as st
from parity import dev

pytestmark = pytest.mark.gpu


def oracle_init(X_init, ranks, seed, sweeps, tol):
    dims = list(X_init.shape)
    cores0 = rng.init_cores(seed, dims, ranks)
    return batch_als.tr_als_ne(X_init, cores0, max_sweeps=sweeps, tol=tol)


@pytest.mark.parametrize("cfg,T,sweeps", [("c1", 40, 100), ("c2", 160, 12)])
def test_initialiser_matches_oracle(trlib, cfg, T, sweeps):
    w = W.make(cfg, T=T)
    X = w.X
    ranks = list(w.ranks)
    X_init = w.X_init()
    seed = 77
    oc, oerr = oracle_init(X_init, ranks, seed, sweeps, 1e-8)
    g = trlib.TRStream(X_init, None, ranks=ranks, seed=seed, init_max_sweeps=sweeps,
                       init_tol=1e-8)
    stt = g.stats()
    cdev = max(dev(a, b) for a, b in zip(g.cores(), oc))
    print(f"[init {cfg}] sweeps gpu {stt['init_sweeps']} oracle {len(oerr) - 1}, err gpu "
          f"{stt['init_rel_err']:.10e} oracle {oerr[-1]:.10e}, cores {cdev:.2e}", flush=True)
    assert stt["init_sweeps"] == len(oerr) - 1
    assert abs(stt["init_rel_err"] - oerr[-1]) <= 1e-10 * oerr[-1]
    assert cdev < 1e-9
    # the stream continues like the oracle's STR from the oracle's cores
    o = st.STR(X_init, [G.copy() for G in oc])
    for b in range(2):
        xb = w.batch(b)
        o.update(xb)
        g.update(xb)
    Tn = w.t_init + 2 * w.t_new
    eo, eg = o.rel_error(X[..., :Tn]), g.reconstruct_error(X[..., :Tn])
    print(f"[init {cfg}] after 2 batches: err gpu {eg:.10e} oracle {eo:.10e}", flush=True)
    assert abs(eg - eo) <= 1e-10 * eo
    g.close()


def test_batch_als_cold_and_hot(trlib):
    dims, ranks, T = (18, 15, 30), (3, 2, 3), 30
    cores, X = W.random_tr_problem(dims, ranks, 12, noise=0.05)
    seed, sweeps = 5, 40
    oc, oerr = oracle_init(X, ranks, seed, sweeps, 1e-10)
    gc, gerr = trlib.tr_batch_als(X, ranks, None, max_sweeps=sweeps, tol=1e-10, seed=seed)
    print(f"[batch cold] sweeps gpu {len(gerr) - 1} oracle {len(oerr) - 1}, err gpu "
          f"{gerr[-1]:.10e} oracle {oerr[-1]:.10e}", flush=True)
    assert len(gerr) == len(oerr)
    assert dev(gerr, np.asarray(oerr)) < 1e-10
    assert max(dev(a, b) for a, b in zip(gc, oc)) < 1e-9
    # warm ("Hot") start over a longer tensor from the previous cores, the
    # temporal core extended by the generating rows of the new slices
    cores2, X2 = W.random_tr_problem(dims[:-1] + (40,), ranks, 12, noise=0.05)
    start = [G.copy() for G in oc]
    start[-1] = np.concatenate([oc[-1], cores2[-1][:, 30:, :]], axis=1)
    oc2, oerr2 = batch_als.tr_als_ne(X2, start, max_sweeps=5, tol=0.0)
    gc2, gerr2 = trlib.tr_batch_als(X2, ranks, start, max_sweeps=5, tol=0.0)
    print(f"[batch hot] err gpu {gerr2[-1]:.10e} oracle {oerr2[-1]:.10e}", flush=True)
    assert len(gerr2) == 6 and dev(gerr2, np.asarray(oerr2)) < 1e-10
    assert max(dev(a, b) for a, b in zip(gc2, oc2)) < 1e-9


def test_initialiser_rejects_bad_options(trlib):
    w = W.make("c1")
    with pytest.raises(trlib.TRError) as e:
        trlib.TRStream(w.X_init(), None, ranks=[3, 3, 3], init_max_sweeps=-1)
    assert e.value.code == 1
