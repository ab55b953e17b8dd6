"""Counter-based random numbers for the randomized variants (Algs. 3, 6-9).

TEST INFRASTRUCTURE (CPU oracle).

The paper draws indices with replacement (Randsample in Algs. 3, 7-9) and
random signs (the D_j of the KSRFT definition) without fixing a generator.
Both this oracle and the HIP library implement, independently, the same
counter-based generator so that their draws coincide:

  splitmix64(x): z = x + 0x9E3779B97F4A7C15 (mod 2^64)
                 z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
                 z = (z ^ (z >> 27)) * 0x94D049BB133111EB
                 return z ^ (z >> 31)
  (the SplitMix64 output function of Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014)

  key(seed, step, core, kind) = splitmix64(seed ^ splitmix64(
                                 (step << 32) | (core << 16) | kind))
  word s of a stream          = splitmix64(key + s)
  uniform u_s                 = (word >> 11) * 2^-53          in [0, 1)
  sign                        = +1 if the top bit of the word is 0, else -1
  uniform index over [I]      = floor(u_s * I)                (IEEE double)
  index from a distribution p = min{i : cdf[i] > u_s}, cdf summed left to
                                right in double, last entry set to 1

``step`` is 0 at initialisation and t at time step t; ``core`` is the 0-based
core whose samples (kind 0) or signs (kind 1) are drawn.

Initial TR-cores (the random start of the batch TR-ALS that initialises a
stream, Sec. 4 protocol) use kind 2: entry e of core k (column-major, e =
r + R_k (i + I_k s)) is the Irwin-Hall approximation of a standard normal,
    z_e = (u_{12e} + u_{12e+1} + ... + u_{12e+11}) - 6,
summed left to right in double precision (mean 0, variance 1).  It needs
no transcendental function, so two independent implementations give the
same bits.
"""

import numpy as np

KIND_INDEX = 0
KIND_SIGN = 1
KIND_INIT = 2

_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function on Python ints (reference definition)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_array(x):
    """Vectorised SplitMix64 on uint64 arrays (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def stream_key(seed, step, core, kind):
    tag = ((int(step) << 32) | (int(core) << 16) | int(kind)) & _M64
    return splitmix64((int(seed) & _M64) ^ splitmix64(tag))


def words(seed, step, core, kind, count):
    key = np.uint64(stream_key(seed, step, core, kind))
    with np.errstate(over="ignore"):
        ctr = key + np.arange(count, dtype=np.uint64)
    return splitmix64_array(ctr)


def uniforms(seed, step, core, count):
    w = words(seed, step, core, KIND_INDEX, count)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_indices(seed, step, core, count, I):
    """Randsample(I, m) with replacement, uniform (Alg. 7)."""
    u = uniforms(seed, step, core, count)
    return np.floor(u * float(I)).astype(np.int64)


def distribution_indices(seed, step, core, count, p):
    """Randsample(I, m, true, p): m draws with replacement from p (Alg. 8)."""
    u = uniforms(seed, step, core, count)
    cdf = np.cumsum(np.asarray(p, dtype=np.float64))
    cdf[-1] = 1.0
    return np.searchsorted(cdf, u, side="right").astype(np.int64)


def signs(seed, step, core, count):
    """Random sign-flip diagonal of D_j (Def. KSRFT): entries +-1."""
    w = words(seed, step, core, KIND_SIGN, count)
    return np.where((w >> np.uint64(63)) == 0, 1.0, -1.0)


def irwin_hall_normals(seed, core, count):
    """Approximately N(0,1) draws of the initial-core stream (kind 2, step 0):
    z_e = sum_{j<12} u_{12e+j} - 6, summed left to right."""
    w = words(seed, 0, core, KIND_INIT, 12 * count)
    u = (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u = u.reshape(count, 12)
    z = np.zeros(count)
    for j in range(12):
        z = z + u[:, j]
    return z - 6.0


def init_cores(seed, dims, ranks):
    """Initial TR-cores G_k (R_k x I_k x R_{k+1}) filled column-major from the
    kind-2 stream of core k."""
    N = len(dims)
    out = []
    for k in range(N):
        shape = (ranks[k], dims[k], ranks[(k + 1) % N])
        z = irwin_hall_normals(seed, k, int(np.prod(shape)))
        out.append(z.reshape(shape, order="F"))
    return out
