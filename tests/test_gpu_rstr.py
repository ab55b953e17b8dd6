"""GPU parity of rSTR-U / rSTR-L (Algs. 7 and 8) against the FP64 oracle.

Both sides draw the same samples from the counter-based generator, so the
comparison is element by element: sample indices bit-exact, and (FP64 path)
P_n, Q_n, cores and fit error within 1e-10 relative.  The GPU solves the
temporal least-squares problem through its normal equations, the oracle
through the pseudo-inverse of the sketched matrix, which bounds the
agreement by cond(G_S)^2 eps.
"""

import numpy as np
import pytest

import workloads as W
from parity import dev
from oracle import randomized as rs

pytestmark = pytest.mark.gpu




def run_pair(P, X, init, t_init, t_new, nb, m, sketch, seed=7, dt="f64", log=""):
    o = rs.RSTR(X[..., :t_init], [G.copy() for G in init], m=m, sketch=sketch, seed=seed)
    g = P.TRStream(X[..., :t_init], init, compute_dtype=dt, sketch=sketch, sketch_size=m,
                   seed=seed)
    N = X.ndim
    s0 = g.samples()
    assert all(np.array_equal(s0[k], o.idxs[k]) for k in range(N)), "initial samples differ"
    worst = 0.0
    for b in range(nb):
        xb = X[..., t_init + b * t_new:t_init + (b + 1) * t_new]
        o.update(xb)
        g.update(xb)
        T = t_init + (b + 1) * t_new
        eo, eg = o.rel_error(X[..., :T]), g.reconstruct_error(X[..., :T])
        worst = max(worst, abs(eg - eo) / eo)
        sg = g.samples()
        same = all(np.array_equal(sg[k], o.idxs[k]) for k in range(N))
        assert same, f"samples differ after batch {b}"
    out = dict(err_dev=worst, err=eg)
    out["cores"] = max(dev(a, b) for a, b in zip(g.cores(), o.cores))
    pq = 0.0
    for n in range(N - 1):
        Pg, Qg = g.PQ(n)
        pq = max(pq, dev(Pg, o.P[n]), dev(Qg, o.Q[n]))
    out["PQ"] = pq
    g.close()
    print(f"[rstr {sketch} {log} {dt}] {out}", flush=True)
    return out


CASES = [
    ((20, 18), (3, 2, 3), 8, 5, 3, 60),
    ((9, 8, 7), (2, 3, 2, 2), 6, 4, 3, 50),
    ((40, 30), (2, 2, 2), 10, 10, 3, 40),      # I > R^2: leverage is not uniform
]


@pytest.mark.parametrize("sketch", ["uniform", "leverage"])
@pytest.mark.parametrize("dims,ranks,t_init,t_new,nb,m", CASES)
def test_rstr_parity_f64(trlib, sketch, dims, ranks, t_init, t_new, nb, m):
    T = t_init + nb * t_new
    cores, X = W.random_tr_problem(tuple(dims) + (T,), ranks, 3, noise=0.05)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :t_init, :]
    init = W.perturb(init, 0.05, np.random.default_rng(1))
    r = run_pair(trlib, X, init, t_init, t_new, nb, m, sketch, log=str(dims))
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-10 and r["cores"] < 1e-9


@pytest.mark.parametrize("sketch", ["uniform", "leverage"])
def test_rstr_exact_recovery(trlib, sketch):
    cores, X = W.random_tr_problem((30, 25, 20), (2, 3, 2), 4)
    init = [G.copy() for G in cores]
    init[-1] = init[-1][:, :8, :]
    g = trlib.TRStream(X[..., :8], init, sketch=sketch, sketch_size=80, seed=3)
    for b in range(3):
        g.update(X[..., 8 + 4 * b:12 + 4 * b])
    assert g.reconstruct_error(X) < 1e-11


@pytest.mark.parametrize("sketch,R", [("uniform", 10), ("leverage", 10), ("leverage", 5)])
def test_rstr_c3_shape(trlib, sketch, R):
    """The 64^3 slices and t_new = 10 of the randomized workload, m = 10 R^2;
    R = 5 makes the leverage distribution non-uniform (64 > 25)."""
    w = W.make("c3", T=70, R=R, init_noise=1e-2)
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, 10 * R * R, sketch,
                 log=f"c3 R={R}")
    assert r["err_dev"] < 1e-10 and r["PQ"] < 1e-10 and r["cores"] < 1e-9
    r = run_pair(trlib, w.X, w.cores_init, w.t_init, w.t_new, 3, 10 * R * R, sketch, dt="f32",
                 log=f"c3 R={R}")
    assert r["err_dev"] < 1e-5 and r["PQ"] < 1e-5 and r["cores"] < 1e-4
