// gfx950 kernels of the randomized variant (rSTR, Alg. 5 with the uniform
// and leverage-score sketches of Algs. 7 and 8, and the sampled subchain /
// fibres of Alg. 3).
//
// Sample draws use a counter-based generator built on the SplitMix64 output
// function (Steele, Lea & Flood, OOPSLA 2014):
//   key(seed, step, core, kind) = mix(seed ^ mix((step<<32)|(core<<16)|kind))
//   word s = mix(key + s),  u = (word >> 11) * 2^-53,
//   uniform index = floor(u * I),  index from p = min{i : cdf[i] > u}
// with cdf summed left to right in FP64 and its last entry set to 1.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tr_internal.h"

namespace trk {

uint64_t rng_key(uint64_t seed, uint64_t step, uint64_t core, uint64_t kind) {
  const uint64_t tag = (step << 32) | (core << 16) | kind;
  return mix64(seed ^ mix64(tag));
}

__device__ inline double rng_uniform(uint64_t key, uint64_t s) {
  return (double)(mix64(key + s) >> 11) * 0x1.0p-53;
}

// Random start of the batch TR-ALS: entry e = r + Ra (i + I s) of a core
// (column-major numbering) is the Irwin-Hall sum of twelve uniforms of the
// stream `key` minus six, z_e = u_{12e} + ... + u_{12e+11} - 6, summed left
// to right (mean 0, variance 1; no transcendental function, so the bits do
// not depend on a math library), written to the slice-major state row i.
__global__ void k_init_normal(uint64_t key, int Ra, int64_t I, int Rb, double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)Ra * I * Rb;
  if (e >= n) return;
  double z = 0.0;
  for (int j = 0; j < 12; ++j) z += rng_uniform(key, (uint64_t)(12 * e + j));
  z -= 6.0;
  const int r = (int)(e % Ra);
  const int64_t rest = e / Ra;
  const int64_t i = rest % I;
  const int sidx = (int)(rest / I);
  G[i * (int64_t)(Ra * Rb) + r + (int64_t)Ra * sidx] = z;
}

hipError_t launch_init_normal(uint64_t key, int Ra, int64_t I, int Rb, double* G,
                              hipStream_t st) {
  const int64_t n = (int64_t)Ra * I * Rb;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_normal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, Ra,
                     I, Rb, G);
  return hipGetLastError();
}

// Randsample(I, m) with replacement, uniform (Alg. 7).
__global__ void k_draw_uniform(uint64_t key, int m, int64_t I, int* __restrict__ idx) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const double u = rng_uniform(key, (uint64_t)s);
  const double x = u * (double)I;
  idx[s] = (int)floor(x);
}

hipError_t launch_draw_uniform(uint64_t key, int m, int64_t I, int* idx, hipStream_t st) {
  hipLaunchKernelGGL(k_draw_uniform, dim3((m + 255) / 256), dim3(256), 0, st, key, m, I, idx);
  return hipGetLastError();
}

// Randsample(I, m, true, p) (Alg. 8): thread 0 forms the cdf left to right,
// then every thread inverts its uniform by binary search.
// distributions of up to this many entries keep their cdf in LDS
constexpr int DRAW_LDS = 4096;

__global__ __launch_bounds__(256) void k_draw_dist(uint64_t key, int m, int64_t I,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ cdf,
                                                   int* __restrict__ idx) {
  __shared__ double sc[DRAW_LDS];
  if (I <= DRAW_LDS) {
    // the same sequential running sum, in LDS, and every search step an LDS
    // read (the draws are those of the global-memory form below)
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) sc[i] = p[i];
    __syncthreads();
    if (threadIdx.x == 0) {
      double c = 0.0;
      for (int64_t i = 0; i < I; ++i) {
        c += sc[i];
        sc[i] = c;
      }
      sc[I - 1] = 1.0;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < m; s += blockDim.x) {
      const double u = rng_uniform(key, (uint64_t)s);
      int lo = 0, hi = (int)I - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sc[mid] > u)
          hi = mid;
        else
          lo = mid + 1;
      }
      idx[s] = lo;
    }
    return;
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double c = 0.0;
    for (int64_t i = 0; i < I; ++i) {
      c += p[i];
      cdf[i] = c;
    }
    cdf[I - 1] = 1.0;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < m; s += blockDim.x) {
    const double u = rng_uniform(key, (uint64_t)s);
    int64_t lo = 0, hi = I - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (cdf[mid] > u)
        hi = mid;
      else
        lo = mid + 1;
    }
    idx[s] = (int)lo;
  }
}

hipError_t launch_draw_dist(uint64_t key, int m, int64_t I, const double* p, double* cdf,
                            int* idx, hipStream_t st) {
  hipLaunchKernelGGL(k_draw_dist, dim3(1), dim3(256), 0, st, key, m, I, p, cdf, idx);
  return hipGetLastError();
}

// Leverage-based distribution of a core (Lemma on leverage estimation,
// Def. leverage scores): p_i = l_i / sum_j l_j (sum_j l_j = rank G_(2)) with
//   l_i = g_i Zinv g_i^T   (I > d: Zinv = (G_(2)^T G_(2))^dagger, the
//                            inverse or, for a rank-deficient core, the
//                            pseudo-inverse of the elimination's fallback),
//   l_i = 1                (I <= d and G_(2) of full row rank: the row Gram
//                            K = G_(2) G_(2)^T passed the elimination),
//   l_i = (K K^dagger)_ii  (I <= d and K rank-deficient: the elimination
//                            fell back to the pseudo-inverse, *fell_back).
// The scores are the diagonal of the projector onto the column space of
// G_(2) in every case.  A zero core (every score 0) gives the uniform
// distribution.
__global__ __launch_bounds__(256) void k_leverage(const double* __restrict__ G, int64_t I, int d,
                                                  const double* __restrict__ Zinv,
                                                  const double* __restrict__ K,
                                                  const int* __restrict__ fell_back,
                                                  double* __restrict__ p) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const bool rowk = K && fell_back && *fell_back;
  double part = 0.0;
  for (int64_t i = tid; i < I; i += 256) {
    double l = 1.0;
    if (!K) {
      const double* g = G + i * d;
      l = 0.0;
      for (int c = 0; c < d; ++c) {
        double t = 0.0;
        for (int c2 = 0; c2 < d; ++c2) t += Zinv[(size_t)c * d + c2] * g[c2];
        l += g[c] * t;
      }
    } else if (rowk) {
      // diagonal of the projector K K^+ onto the row space of G G^T
      l = 0.0;
      for (int64_t j = 0; j < I; ++j) l += K[i * I + j] * Zinv[j * I + i];
    }
    p[i] = l;
    part += l;
  }
  red[tid] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double tot = red[0];
  for (int64_t i = tid; i < I; i += 256) p[i] = tot > 0.0 ? p[i] / tot : 1.0 / (double)I;
}

hipError_t launch_leverage(const double* G, int64_t I, int d, const double* Zinv,
                           const double* K, const int* fell_back, double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_leverage, dim3(1), dim3(256), 0, st, G, I, d, Zinv, K, fell_back, p);
  return hipGetLastError();
}

// Sampled subchain rows (Alg. 3): for sample s of mode n, row s of
// G^{!=n}_S[2] is the subchain row at the multi-index (idx_q[s])_{q != n}:
//   A[s][r + R_n*srow] = (G_{n+1}(.) ... G_{n-1}(.))[srow, r]
// and its weight w[s] (the diagonal of D_n^2): wconst for the uniform sketch,
// 1 / (m prod_{q != n} p_q[idx_q[s]]) when `probs` is given.
// One sampled row per 16-lane group (lane b of the group holds column b of
// the running row product), so a slice product is 16 independent column
// loads per lane and 16 shuffles inside the group.
__global__ __launch_bounds__(256) void k_sample_rows(Geom g, CoreView cv,
                                                     const int* __restrict__ idxs, int m,
                                                     const double* const* probs, double wconst,
                                                     double* __restrict__ A,
                                                     double* __restrict__ w) {
  const int N = g.N;
  const int Rn = g.R[g.n], Rn1 = g.R[g.n + 1 == N ? 0 : g.n + 1];
  const int d = g.d;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = threadIdx.x & 15;
  const int e = tid >> 4;                              // (sample, row) pair
  const bool live = e < m * Rn1;
  const int ec = live ? e : 0;
  const int s = ec / Rn1, srow = ec - s * Rn1;
  // row srow of G_{n+1}(.) ... G_{n-1}(.), column b in this lane
  int q = g.n + 1 == N ? 0 : g.n + 1;
  double v;
  {
    const int iq = idxs[(size_t)q * m + s];
    const int Rq1 = g.R[q + 1 == N ? 0 : q + 1];
    const double* G0 = (const double*)cv.ptr[q] + iq * cv.si[q] + srow * cv.sr[q];
    const double x = G0[(b < Rq1 ? b : 0) * cv.ss[q]];
    v = b < Rq1 ? x : 0.0;
  }
  for (int j = 1; j < N - 1; ++j) {
    q = q + 1 == N ? 0 : q + 1;
    const int iq = idxs[(size_t)q * m + s];
    const double* H = (const double*)cv.ptr[q] + iq * cv.si[q];
    const int Rq = g.R[q], Rq2 = g.R[q + 1 == N ? 0 : q + 1];
    const int bc = b < Rq2 ? b : 0;
    double h[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int ac = a < Rq ? a : 0;                 // loads stay inside the slice
      const double x = H[ac * cv.sr[q] + bc * cv.ss[q]];
      h[a] = (a < Rq && b < Rq2) ? x : 0.0;
    }
    double u = 0.0;
#pragma unroll
    for (int a = 0; a < 16; ++a) u = fma(__shfl(v, a, 16), h[a], u);
    v = u;
  }
  if (live && b < Rn) A[(size_t)s * d + b + Rn * srow] = v;
  if (live && srow == 0 && b == 0) {
    double ws = wconst;
    if (probs) {
      double qq = 1.0;
      for (int k = 0; k < N; ++k)
        if (k != g.n) qq *= probs[k][idxs[(size_t)k * m + s]];
      ws = 1.0 / ((double)m * qq);
    }
    w[s] = ws;
  }
}

hipError_t launch_sample_rows(const Geom& g, const CoreView& cv, const int* idxs, int m,
                              const double* const* probs, double wconst, double* A, double* w,
                              hipStream_t st) {
  for (int k = 0; k < g.N; ++k)
    if (g.R[k] > 16) return hipErrorInvalidValue;
  const int Rn1 = g.R[g.n + 1 == g.N ? 0 : g.n + 1];
  const int64_t nthr = (int64_t)m * Rn1 * 16;
  dim3 grid((unsigned)((nthr + 255) / 256));
  hipLaunchKernelGGL(k_sample_rows, grid, dim3(256), 0, st, g, cv, idxs, m, probs, wconst, A, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sketched product: part[split][i][c] = sum over the split's samples s of
//   X_S[i][s] * w[s] * A[s][c],
// X_S[:, s] the mode-n fibre of X at the sampled indices (Alg. 3, read as m
// fibres).  Same tiling as the MTTKRP: KC samples per chunk staged in LDS,
// 16x16x4 MFMAs, each wave owning output blocks wave, wave+4, ...
// ---------------------------------------------------------------------------
typedef double d4s __attribute__((ext_vector_type(4)));
typedef float f4s __attribute__((ext_vector_type(4)));

__device__ inline d4s mfma_s(double a, double b, d4s c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4s mfma_s(float a, float b, f4s c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct SAcc;
template <> struct SAcc<double> {
  typedef double type;
  typedef d4s vec;
  static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct SAcc<float> {
  typedef float type;
  typedef f4s vec;
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T, int MAXB>
__global__ __launch_bounds__(256) void k_sketch_gemm(Geom g, int MT, int cpw, const T* __restrict__ X,
                                                     const int* __restrict__ idxs, int m,
                                                     const double* __restrict__ A,
                                                     const double* __restrict__ w,
                                                     typename SAcc<T>::type* __restrict__ part) {
  typedef typename SAcc<T>::vec V4;
  constexpr int KCP = KC + 1;
  extern __shared__ __align__(16) char smem[];
  const int d = g.d;
  const int NB = (d + 15) >> 4, NTP = NB * 16;
  int64_t* off = (int64_t*)smem;                       // [KC]
  T* Bs = (T*)(off + KC);                              // [KC][NTP]
  T* As = Bs + KC * NTP;                               // [MT][KCP]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int split = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * MT;
  const int nblk = (MT >> 4) * NB;
  const int s_beg = split * cpw * KC;
  const int s_end = s_beg + cpw * KC < m ? s_beg + cpw * KC : m;
  // X strides of every mode
  int64_t stride[MAXN];
  {
    int64_t acc = 1;
    for (int q = 0; q < g.N; ++q) {
      stride[q] = acc;
      acc *= g.I[q];
    }
  }
  V4 acc[MAXB];
#pragma unroll
  for (int bi = 0; bi < MAXB; ++bi) acc[bi] = V4{0, 0, 0, 0};
  for (int sb = s_beg; sb < s_end; sb += KC) {
    if (tid < KC) {
      const int s = sb + tid;
      int64_t o = -1;
      if (s < s_end) {
        o = 0;
        for (int q = 0; q < g.N; ++q)
          if (q != g.n) o += (int64_t)idxs[(size_t)q * m + s] * stride[q];
      }
      off[tid] = o;
    }
    __syncthreads();
    // staging in batches of 8 elements per thread with every load of a
    // batch in flight (indices clamped in range, the selects after the loads)
    for (int e0 = tid; e0 < KC * NTP; e0 += 256 * 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e / NTP, c = e - kk * NTP;
        const int s = sb + kk;
        const bool ok = e < KC * NTP && s < s_end && c < d;
        const int sc = s < s_end ? s : s_end - 1, cc = c < d ? c : d - 1;
        const double x = w[sc] * A[(size_t)sc * d + cc];
        v[u] = ok ? (T)x : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        if (e < KC * NTP) Bs[e] = v[u];
      }
    }
    for (int e0 = tid; e0 < MT * KC; e0 += 256 * 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e % KC, mm = e / KC;
        const int64_t mg = m0 + mm;
        const bool ok = e < MT * KC && mg < g.In && off[kk] >= 0;
        const T x = X[ok ? off[kk] + mg * stride[g.n] : 0];
        v[u] = ok ? x : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e % KC, mm = e / KC;
        if (e < MT * KC) As[mm * KCP + kk] = v[u];
      }
    }
    __syncthreads();
    const int ar = lane & 15, ak = lane >> 4;
    for (int k0 = 0; k0 < KC; k0 += 4) {
#pragma unroll
      for (int bi = 0; bi < MAXB; ++bi) {
        const int b = wave + 4 * bi;
        if (b < nblk) {
          const int rb = b / NB, cb = b - rb * NB;
          acc[bi] = mfma_s(As[(rb * 16 + ar) * KCP + k0 + ak], Bs[(k0 + ak) * NTP + cb * 16 + ar],
                           acc[bi]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < MAXB; ++bi) {
    const int b = wave + 4 * bi;
    if (b < nblk) {
      const int rb = b / NB, cb = b - rb * NB;
      const int col = cb * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t mg = m0 + rb * 16 + SAcc<T>::row(lane, v);
        if (mg < g.In && col < d) part[((size_t)split * g.In + mg) * d + col] = acc[bi][v];
      }
    }
  }
}

SketchPlan plan_sketch(const Geom& g, int m, int xdtype) {
  SketchPlan p;
  const int NB = (g.d + 15) / 16;
  int MT = (int)((g.In + 15) / 16) * 16;
  if (MT > 64) MT = 64;
  while (MT > 16 && (MT / 16) * NB > 64) MT -= 16;
  p.MT = MT;
  p.mtiles = (int)((g.In + MT - 1) / MT);
  const int chunks = (m + KC - 1) / KC;
  p.cpw = 1;
  p.nsplit = chunks;
  p.psize = xdtype == F64 ? 8 : 4;
  return p;
}

template <typename T, int MAXB>
static hipError_t launch_sketch_t(const Geom& g, const SketchPlan& p, const void* X,
                                  const int* idxs, int m, const double* A, const double* w,
                                  void* part, hipStream_t st) {
  const int NTP = ((g.d + 15) / 16) * 16;
  const size_t lds = KC * sizeof(int64_t) + (size_t)KC * NTP * sizeof(T) +
                     (size_t)p.MT * (KC + 1) * sizeof(T);
  auto fn = k_sketch_gemm<T, MAXB>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(p.nsplit, p.mtiles), dim3(256), lds, st, g, p.MT, p.cpw,
                     (const T*)X, idxs, m, A, w, (typename SAcc<T>::type*)part);
  return hipGetLastError();
}

hipError_t launch_sketch_gemm(const Geom& g, const SketchPlan& p, const void* X, int xdt,
                              const int* idxs, int m, const double* A, const double* w,
                              void* part, hipStream_t st) {
  const int nblk = (p.MT / 16) * ((g.d + 15) / 16);
  const int per = (nblk + 3) / 4;
  if (xdt == F64) {
    if (per <= 4) return launch_sketch_t<double, 4>(g, p, X, idxs, m, A, w, part, st);
    if (per <= 8) return launch_sketch_t<double, 8>(g, p, X, idxs, m, A, w, part, st);
    return launch_sketch_t<double, 16>(g, p, X, idxs, m, A, w, part, st);
  }
  if (xdt == F32) {
    if (per <= 4) return launch_sketch_t<float, 4>(g, p, X, idxs, m, A, w, part, st);
    if (per <= 8) return launch_sketch_t<float, 8>(g, p, X, idxs, m, A, w, part, st);
    return launch_sketch_t<float, 16>(g, p, X, idxs, m, A, w, part, st);
  }
  return hipErrorInvalidValue;
}

// out[c1*d + c2] = sum_s w[s] A[s][c1] A[s][c2] (w == nullptr: weights 1),
// the weighted Gram of the sampled rows (the sketched Q_n of Alg. 5).  One
// workgroup of 16 waves per upper-triangle 16x16 tile: wave j takes the
// k-steps (4 rows each) j, j+16, ... on FP64 16x16x4 MFMAs with 8 k-steps of
// loads in flight and two accumulators; the 16 wave sums are added in LDS
// in a fixed order and the tile and its mirror are written, so the result
// is exactly symmetric.
constexpr int WG_WAVES = 16;

__global__ __launch_bounds__(64 * WG_WAVES) void k_wgram(const double* __restrict__ A,
                                                         const double* __restrict__ w,
                                                         int64_t rows, int d,
                                                         double* __restrict__ out) {
  __shared__ double red[WG_WAVES][256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int nb = (d + 15) >> 4;
  int rb = 0, cb = blockIdx.x;
  while (cb >= nb - rb) {
    cb -= nb - rb;
    ++rb;
  }
  cb += rb;
  const int c1 = min(rb * 16 + l16, d - 1), c2 = min(cb * 16 + l16, d - 1);
  const int64_t nks = (rows + 3) / 4, rl = rows > 0 ? rows - 1 : 0;
  constexpr int KB = 8;
  d4s acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  for (int64_t k0 = wave; k0 < nks; k0 += KB * WG_WAVES) {
    double av[KB], bv[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int64_t i = (k0 + WG_WAVES * q) * 4 + g4;
      const int64_t ic = i < rows ? i : rl;
      const double wi = w ? w[ic] : 1.0;
      const double xa = A[ic * d + c1], xb = A[ic * d + c2];
      const bool ok = i < rows;
      av[q] = ok ? wi * xa : 0.0;
      bv[q] = ok ? xb : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KB; q += 2) {
      acc0 = mfma_s(av[q], bv[q], acc0);
      acc1 = mfma_s(av[q + 1], bv[q + 1], acc1);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][SAcc<double>::row(lane, v) * 16 + l16] = acc0[v] + acc1[v];
  __syncthreads();
  if (tid < 256) {
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < WG_WAVES; ++j) sum += red[j][tid];
    const int r = rb * 16 + (tid >> 4), c = cb * 16 + (tid & 15);
    // on a diagonal tile only the upper entry of each pair writes (both
    // positions): one writer per element, exactly symmetric
    if (r < d && c < d && r <= c) {
      out[(size_t)r * d + c] = sum;
      out[(size_t)c * d + r] = sum;
    }
  }
}

hipError_t launch_wgram(const double* A, const double* w, int64_t rows, int d, double* out,
                        hipStream_t st) {
  const int nb = (d + 15) / 16;
  hipLaunchKernelGGL(k_wgram, dim3(nb * (nb + 1) / 2), dim3(64 * WG_WAVES), 0, st, A, w, rows, d,
                     out);
  return hipGetLastError();
}

// Row Gram K = G_(2) G_(2)^T (I x I) of slice-major rows, for the rank check
// of the leverage distribution when I <= d.
__global__ __launch_bounds__(256) void k_row_gram(const double* __restrict__ G, int64_t I, int d,
                                                  double* __restrict__ K) {
  // 16 lanes per entry, each summing every 16th column, then a fixed-order
  // butterfly over the 16 lanes: the partials of (i, j) and (j, i) are the
  // same products in the same order, so K is exactly symmetric
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t e = t >> 4;
  const int l = threadIdx.x & 15;
  const bool ok = e < I * I;
  const int64_t ec = ok ? e : 0;
  const int64_t i = ec / I, j = ec - i * I;
  double s = 0.0;
  for (int c = l; c < d; c += 16) s += G[i * d + c] * G[j * d + c];
  s += __shfl_xor(s, 8, 16);
  s += __shfl_xor(s, 4, 16);
  s += __shfl_xor(s, 2, 16);
  s += __shfl_xor(s, 1, 16);
  if (ok && l == 0) K[e] = s;
}

hipError_t launch_row_gram(const double* G, int64_t I, int d, double* K, hipStream_t st) {
  hipLaunchKernelGGL(k_row_gram, dim3((unsigned)((I * I * 16 + 255) / 256)), dim3(256), 0, st, G,
                     I, d, K);
  return hipGetLastError();
}

}  // namespace trk
