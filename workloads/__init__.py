"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module only draws data; it performs none of the tracking method's
arithmetic.  Tensors are returned as float64 arrays indexed X[i_1, .., i_N]
in Fortran (first-index-fastest) memory order, so a temporal batch
X[..., t0:t1] is one contiguous block, as the C ABI expects.

Workloads (sizes per the streaming protocol of Sec. 4: an initial part, then
batches of t_new temporal slices):

  c1  20 x 20 x 40,  t_init 10, t_new 5,  R 3,  Gaussian cores,
      X = TR(G) + 1e-3 N(0,1)
  c2  256 x 256 x 1000, t_init 100, t_new 20, R 8, Gaussian cores,
      X = TR(G) + N(0, s^2), s = 1e-2 ||TR(G)||_F / sqrt(numel)
  c3  64 x 64 x 64 x 400, t_init 40, t_new 10, R 10, sketch m = 10 R^2,
      Gaussian cores, 1e-2 relative noise as c2
  c4  120 x 160 x 3 x 600, t_init 60, t_new 20, R 12, KSRFT m = 10 R^2;
      video-like: a sum of 12 separable products of cosines with random
      frequencies in {1..4} and phases, channel weights in [0, 1], scaled to
      max |X| = 1, plus U(-0.05, 0.05) noise (CP rank 12, hence exact TR rank
      12 with diagonal cores)
  c5  64 x 64 x 64 x 50 (one batch), R 16; fit loss at true cores plus
      0.1 N(0,1)

Gaussian-core data follow the synthetic recipe of Sec. 4.2 (TR-cores with
i.i.d. standard normal entries).  c4 stands in for the paper's video data
set, which is not available here.

Initial cores for streaming runs are the generating cores plus a seeded
perturbation of relative size ``init_noise`` (default 1e-4, standing in for
the converged batch TR-ALS initialisation of the experimental protocol in
Sec. 4): the paper lets any method produce the initial decomposition as long
as every tracker starts from the same one (remark after Alg. 4).

Seeds: numpy.random.default_rng([2307, 719, cfg, stream]) with stream
0 = cores, 1 = noise, 2 = initial-core perturbation, 3 = c5 perturbation,
4 = c4 field parameters.
"""

from dataclasses import dataclass, field

import numpy as np

CONFIGS = {
    "c1": dict(cfg=1, dims=(20, 20), T=40, t_init=10, t_new=5, R=3, sketch=None, m=0),
    "c2": dict(cfg=2, dims=(256, 256), T=1000, t_init=100, t_new=20, R=8, sketch=None, m=0),
    "c3": dict(cfg=3, dims=(64, 64, 64), T=400, t_init=40, t_new=10, R=10,
               sketch="uniform", m=1000),
    "c4": dict(cfg=4, dims=(120, 160, 3), T=600, t_init=60, t_new=20, R=12,
               sketch="ksrft", m=1440),
    "c5": dict(cfg=5, dims=(64, 64, 64), T=50, t_init=0, t_new=50, R=16, sketch=None, m=0),
}


def rng_for(cfg, stream):
    return np.random.default_rng([2307, 719, int(cfg), int(stream)])


def gaussian_cores(dims, ranks, rng):
    """TR-cores G_n of shape (R_n, I_n, R_{n+1}) with N(0,1) entries."""
    N = len(dims)
    return [rng.standard_normal((ranks[n], dims[n], ranks[(n + 1) % N]))
            for n in range(N)]


def synthesize_tr(cores):
    """Data tensor of the TR format, X(i) = Trace(prod_n G_n(i_n)), formed by
    contracting the cores one after the other (data synthesis only)."""
    T = cores[0]                                   # (R_1, I_1, R_2)
    for G in cores[1:-1]:
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    # T: (R_1, I_1, ..., I_{N-1}, R_N); close the ring with the last core
    R1, RN = T.shape[0], T.shape[-1]
    lead = T.shape[1:-1]
    J = int(np.prod(lead))
    Tm = np.moveaxis(T, 0, -1).reshape(J, RN * R1, order="F")  # [(i), b + RN*a]
    GN = cores[-1]                                 # (R_N, I_N, R_1)
    GNm = np.transpose(GN, (0, 2, 1)).reshape(RN * R1, GN.shape[1], order="F")
    X = (GNm.T @ Tm.T).T                          # Fortran-contiguous (J, I_N)
    return X.reshape(tuple(lead) + (GN.shape[1],), order="F")


def _add_noise(X0, e_flat):
    """X0 + e in place; e_flat is laid out in X0's first-index-fastest order."""
    X = np.asfortranarray(X0)
    Xf = X.reshape(-1, order="F")
    np.add(Xf, e_flat, out=Xf)
    return X


def perturb(cores, rel, rng):
    """cores + rel * std(core) * N(0,1), per core."""
    out = []
    for G in cores:
        s = float(np.std(G)) if G.size else 1.0
        out.append(G + rel * s * rng.standard_normal(G.shape))
    return out


def video_field(dims_t, R, rng):
    """c4 recipe: rank-R sum of separable cosine products (diagonal TR cores)."""
    I1, I2, C, T = dims_t
    f = rng.integers(1, 5, size=(R, 3))
    ph = rng.uniform(0.0, 2 * np.pi, size=(R, 3))
    a = rng.uniform(0.5, 1.0, size=R)
    w = rng.uniform(0.0, 1.0, size=(R, C))
    u1 = np.cos(2 * np.pi * f[:, 0:1] * np.arange(I1)[None, :] / I1 + ph[:, 0:1])
    u2 = np.cos(2 * np.pi * f[:, 1:2] * np.arange(I2)[None, :] / I2 + ph[:, 1:2])
    u4 = np.cos(2 * np.pi * f[:, 2:3] * np.arange(T)[None, :] / T + ph[:, 2:3])
    factors = [a[:, None] * u1, u2, w, u4]        # each (R, I_n)
    cores = []
    for U in factors:
        G = np.zeros((R, U.shape[1], R))
        for r in range(R):
            G[r, :, r] = U[r]
        cores.append(G)
    return cores


@dataclass
class Workload:
    name: str
    dims: tuple                  # all N dims, temporal last (full length)
    ranks: tuple                 # R_1..R_N
    t_init: int
    t_new: int
    sketch: object
    m: int
    cores_true: list
    X: np.ndarray                # full stream, Fortran order
    cores_init: list = field(default_factory=list)
    sketch_seed: int = 0         # key of the sample / sign generator

    @property
    def N(self):
        return len(self.dims)

    @property
    def n_batches(self):
        return (self.dims[-1] - self.t_init) // self.t_new

    def X_init(self):
        return self.X[..., :self.t_init]

    def batch(self, b):
        t0 = self.t_init + b * self.t_new
        return self.X[..., t0:t0 + self.t_new]


def make(name, init_noise=1e-4, dims=None, T=None, t_init=None, t_new=None, R=None,
         noise=None):
    """Build a named workload; keyword overrides give smaller variants of the
    same recipe for tests (``noise`` overrides the noise level)."""
    c = dict(CONFIGS[name])
    dims_s = tuple(dims) if dims is not None else c["dims"]
    T = c["T"] if T is None else T
    t_init = c["t_init"] if t_init is None else t_init
    t_new = c["t_new"] if t_new is None else t_new
    R = c["R"] if R is None else R
    full = tuple(dims_s) + (T,)
    N = len(full)
    ranks = (R,) * N
    cfg = c["cfg"]
    if name == "c4":
        cores = video_field(full, R, rng_for(cfg, 4))
        X0 = synthesize_tr(cores)
        scale = float(np.max(np.abs(X0)))
        X0 = X0 / scale
        cores = [cores[0] / scale] + cores[1:]
        lvl = 0.05 if noise is None else noise
        X = _add_noise(X0, rng_for(cfg, 1).uniform(-lvl, lvl, size=X0.size))
    else:
        cores = gaussian_cores(full, ranks, rng_for(cfg, 0))
        X0 = synthesize_tr(cores)
        if name == "c1":
            lvl = 1e-3 if noise is None else noise
            X = _add_noise(X0, lvl * rng_for(cfg, 1).standard_normal(X0.size))
        else:
            lvl = 1e-2 if noise is None else noise
            s = lvl * np.linalg.norm(X0.ravel(order="K")) / np.sqrt(X0.size)
            e = rng_for(cfg, 1).standard_normal(X0.size)
            X = _add_noise(X0, np.multiply(e, s, out=e))
    X = np.asfortranarray(X)
    w = Workload(name, full, ranks, t_init, t_new, c["sketch"], c["m"], cores, X)
    w.sketch_seed = 2307719 * 10 + cfg
    if t_init > 0:
        init = [G.copy() for G in cores]
        init[-1] = init[-1][:, :t_init, :]
        w.cores_init = perturb(init, init_noise, rng_for(cfg, 2)) if init_noise else init
    return w


def c5_point(w, rel=0.1):
    """c5 evaluation point: true cores + rel * N(0,1)."""
    r = rng_for(5, 3)
    return [G + rel * r.standard_normal(G.shape) for G in w.cores_true]


def random_tr_problem(dims, ranks, seed, noise=0.0):
    """Small ad-hoc problem for tests: Gaussian cores and X = TR(G) + noise."""
    r = np.random.default_rng(seed)
    cores = gaussian_cores(dims, ranks, r)
    X = synthesize_tr(cores)
    if noise:
        X = X + noise * r.standard_normal(X.shape)
    return cores, np.asfortranarray(X)
