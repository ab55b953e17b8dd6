// gfx950 kernels of the KSRFT-sketched variant (rSTR-K, Alg. 9, with the
// mixing of Alg. 6 and the sampling of Alg. 3).
//
// F_j is the unitary DFT of size I_j, F[a, b] = exp(-2 pi i a b / I_j) /
// sqrt(I_j), and D_j a diagonal of random signs (Def. KSRFT); the mixed
// tensor and cores are Xhat = X x_1 (F_1 D_1) ... x_N (F_N D_N) and
// Ghat_k = G_k x_2 (F_k D_k).  Complex quantities are kept as two real
// planes (real part first).  Only real parts of P_n and Q_n enter the
// solves (Alg. 9), so the sketched products are formed as real GEMMs over
// the stacked planes:
//   Re(Q) = Re(A)^T W Re(A) + Im(A)^T W Im(A),
//   Z = Xhat_S W conj(A) = [Re Xhat_S | Im Xhat_S] [[W Re A, -W Im A],
//                                                    [W Im A,  W Re A]],
// and the mode-n unmixing D_n F_n^* is applied to Z (an I_n x I_n product)
// rather than to the sampled fibres: Re(D_n F_n^* Z) is the increment of
// Re(P_n).  The mixing of X is the dense contraction of the method; it runs
// on MFMA in the compute precision (BF16 with FP32 accumulation for the
// mixed-precision path).

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "bf16_round.h"
#include <stdint.h>

#include "tr_internal.h"

namespace trk {

typedef double kd4 __attribute__((ext_vector_type(4)));
typedef float kf4 __attribute__((ext_vector_type(4)));
typedef __bf16 kbf8 __attribute__((ext_vector_type(8)));

// MFMA operand traits: KPL consecutive K values per lane, 4*KPL per step.
template <typename TM> struct Mf;
template <> struct Mf<double> {
  static constexpr int KPL = 1;
  typedef double frag;
  typedef kd4 acc;
  typedef double out;
  static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ inline acc op(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mf<float> {
  static constexpr int KPL = 1;
  typedef float frag;
  typedef kf4 acc;
  typedef float out;
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ inline acc op(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mf<__bf16> {
  static constexpr int KPL = 8;
  typedef kbf8 frag;
  typedef kf4 acc;
  typedef float out;
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ inline acc op(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <typename TM>
__device__ inline typename Mf<TM>::frag load_frag(const TM* p) {
  if constexpr (Mf<TM>::KPL == 1) {
    return *p;
  } else {
    kbf8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[i];
    return v;
  }
}

template <typename T>
__device__ inline double to_double(T x) {
  return (double)x;
}
template <>
__device__ inline double to_double<__hip_bfloat16>(__hip_bfloat16 x) {
  return (double)__bfloat162float(x);
}
template <typename TM>
__device__ inline TM from_double(double x) {
  return (TM)x;
}
template <>
__device__ inline __bf16 from_double<__bf16>(double x) {
  return __builtin_bit_cast(__bf16, bf16_bits_rne(x));
}

// cos / sin of 2 pi r / I for the integer r = (a b) mod I.
__device__ inline void twiddle(int64_t r, int64_t I, double* c, double* s) {
  sincospi(2.0 * (double)r / (double)I, s, c);
}

// ---------------------------------------------------------------------------
// Random signs of D_j: +1 when the top bit of the stream word is 0.
// ---------------------------------------------------------------------------
__global__ void k_signs(uint64_t key, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (mix64(key + (uint64_t)i) >> 63) == 0 ? 1.0 : -1.0;
}

hipError_t launch_signs(uint64_t key, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_signs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, n, out);
  return hipGetLastError();
}

__global__ void k_signs_all(SignsAll a) {
  const int k = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.n[k]) a.out[k][i] = (mix64(a.key[k] + (uint64_t)i) >> 63) == 0 ? 1.0 : -1.0;
}

hipError_t launch_signs_all(const SignsAll& a, hipStream_t st) {
  if (a.count < 1 || a.count > MAXN) return hipErrorInvalidValue;
  int64_t nmax = 1;
  for (int k = 0; k < a.count; ++k) nmax = a.n[k] > nmax ? a.n[k] : nmax;
  hipLaunchKernelGGL(k_signs_all, dim3((unsigned)((nmax + 255) / 256), (unsigned)a.count),
                     dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mixing matrix of one mode as a real (2I x Kp) row-major matrix acting on
// stacked planes: real input [[Re W], [Im W]], complex input
// [[Re W, -Im W], [Im W, Re W]], W = F D; columns past pin*I are zero.
// ---------------------------------------------------------------------------
// K of a mixing matrix (pin I) padded to the 64-row staging chunks.
__host__ __device__ inline int mix_kp(int64_t I, int pin) { return (pin * (int)I + 63) / 64 * 64; }

template <typename TM>
__device__ inline void mix_weight(int64_t I, int pin, const double* __restrict__ D, int Kp,
                                  TM* __restrict__ W, int64_t e);

template <typename TM>
__global__ void k_mix_weights(int64_t I, int pin, const double* __restrict__ D, int Kp,
                              TM* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < 2 * I * Kp) mix_weight(I, pin, D, Kp, W, e);
}

template <typename TM>
__global__ void k_mix_weights_all(MixWeightsAll a) {
  const int k = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int Kp = mix_kp(a.I[k], a.pin[k]);
  if (e < 2 * a.I[k] * Kp) mix_weight(a.I[k], a.pin[k], a.D[k], Kp, (TM*)a.W[k], e);
}

// Entry e (row-major) of the mixing matrix.
template <typename TM>
__device__ inline void mix_weight(int64_t I, int pin, const double* __restrict__ D, int Kp,
                                  TM* __restrict__ W, int64_t e) {
  const int64_t row = e / Kp, col = e - row * Kp;
  double val = 0.0;
  if (col < pin * I) {
    const int64_t po = row / I, i = row - po * I;
    const int64_t pi = col / I, b = col - pi * I;
    double c, s;
    twiddle((i * b) % I, I, &c, &s);
    const double sc = D[b] / sqrt((double)I);
    const double wre = c * sc, wim = -s * sc;
    if (pin == 1)
      val = po == 0 ? wre : wim;
    else
      val = po == 0 ? (pi == 0 ? wre : -wim) : (pi == 0 ? wim : wre);
  }
  W[e] = from_double<TM>(val);
}

// ---------------------------------------------------------------------------
// One mode product of the mixing: out[po][.., i, ..] = sum_{pi, b}
// W[(po, i)][(pi, b)] in[pi][.., b, ..] over a column-major tensor whose
// mode has stride S and size I (C = the product of the slower modes).
// Column j = a + S c of the unfolding holds the elements a + S (b + I c).
// Workgroup: JT columns, all 2I rows; K staged in LDS in chunks of KCH
// (stored column-major, so an MFMA operand of KPL consecutive k is one
// contiguous read); W read through the cache.  Wave w owns row tiles
// w, w+4, ...
// ---------------------------------------------------------------------------
template <typename TI, typename TM, typename TO, int JT, int RTW>
__global__ __launch_bounds__(256) void k_mix_mode(const TI* __restrict__ in, int pin,
                                                  int64_t ips, TO* __restrict__ out, int64_t ops,
                                                  int64_t S, int64_t I, int64_t C,
                                                  const TM* __restrict__ W, int Kp) {
  typedef Mf<TM> M;
  typedef typename M::acc ACC;
  constexpr int KCH = 64;
  constexpr int KCP = KCH + (M::KPL == 8 ? 8 : 1);
  constexpr int NCT = JT / 16;
  __shared__ __align__(16) TM Bs[JT * KCP];
  // offset of (plane 0, i = 0) of each of the workgroup's columns
  // j = a + S c: a + S I c (-1 past the last column), decoded once here
  __shared__ int64_t colb[JT];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t J = S * C;
  const int64_t j0 = (int64_t)blockIdx.x * JT;
  const int K = pin * (int)I;
  const int M2 = 2 * (int)I;
  const int nrt = (M2 + 15) / 16;
  const int l16 = lane & 15, g4 = lane >> 4;
  if (tid < JT) {
    const int64_t j = j0 + tid;
    colb[tid] = j < J ? (j % S) + S * I * (j / S) : -1;
  }
  __syncthreads();
  ACC acc[RTW][NCT];
#pragma unroll
  for (int r = 0; r < RTW; ++r)
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[r][c] = ACC{0, 0, 0, 0};

  for (int kc = 0; kc < Kp; kc += KCH) {
    // stage B[k][j] = in[k / I][.., k % I, ..] (zero past K and J)
    for (int e = tid; e < KCH * JT; e += 256) {
      int kl, jl;
      if (S > 1) {
        jl = e % JT;
        kl = e / JT;
      } else {
        kl = e % KCH;
        jl = e / KCH;
      }
      const int k = kc + kl;
      const int64_t cb = colb[jl];
      double v = 0.0;
      if (k < K && cb >= 0) {
        const int pi = k >= (int)I ? 1 : 0, b = k - pi * (int)I;   // pin <= 2
        v = to_double(in[pi * ips + cb + S * b]);
      }
      Bs[jl * KCP + kl] = from_double<TM>(v);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KCH; ks += 4 * M::KPL) {
      const int kk = ks + g4 * M::KPL;
      typename M::frag bfr[NCT];
#pragma unroll
      for (int c = 0; c < NCT; ++c) bfr[c] = load_frag<TM>(&Bs[(c * 16 + l16) * KCP + kk]);
#pragma unroll
      for (int r = 0; r < RTW; ++r) {
        const int rt = wave + 4 * r;
        const int row = rt * 16 + l16 < M2 ? rt * 16 + l16 : M2 - 1;
        const typename M::frag afr = load_frag<TM>(&W[(int64_t)row * Kp + kc + kk]);
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[r][c] = M::op(afr, bfr[c], acc[r][c]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RTW; ++r) {
    const int rt = wave + 4 * r;
    if (rt < nrt) {
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int64_t cb = colb[c * 16 + l16];
        if (cb >= 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rt * 16 + M::row(lane, v);
            if (row < M2) {
              const int po = row >= (int)I ? 1 : 0, i = row - po * (int)I;
              out[po * ops + cb + S * i] = (TO)acc[r][c][v];
            }
          }
        }
      }
    }
  }
}

static int round_up(int x, int q) { return (x + q - 1) / q * q; }

// Mixing along a short mode (2I <= 16), where the MFMA tiles would be
// mostly padding: one thread per column j = a + S c, its pin I inputs
// rounded to the operand type TM (as the tiled kernel rounds its staged
// operands) against the 2I x Kp matrix, accumulated in the output type.
template <typename TI, typename TM, typename TO>
__global__ __launch_bounds__(256) void k_mix_small(const TI* __restrict__ in, int pin,
                                                   int64_t ips, TO* __restrict__ out,
                                                   int64_t ops, int64_t S, int I, int64_t C,
                                                   const TM* __restrict__ W, int Kp) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= S * C) return;
  const int64_t cb = (j % S) + S * I * (j / S);
  const int K = pin * I;
  TO x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    x[k] = TO(0);
    if (k < K) {
      const int pi = k >= I ? 1 : 0, b = k - pi * I;
      const TM v = from_double<TM>(to_double(in[pi * ips + cb + S * b]));
      x[k] = (TO)(float)v;
      if constexpr (sizeof(TM) == 8) x[k] = (TO)v;
    }
  }
#pragma unroll
  for (int row = 0; row < 16; ++row) {
    if (row < 2 * I) {
      TO acc = TO(0);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        TO w = TO(0);
        if (k < K) {
          const TM wv = W[row * Kp + k];
          w = (TO)(float)wv;
          if constexpr (sizeof(TM) == 8) w = (TO)wv;
        }
        acc += w * x[k];
      }
      const int po = row >= I ? 1 : 0, i = row - po * I;
      out[po * ops + cb + S * i] = acc;
    }
  }
}

template <typename TI, typename TM, typename TO, int JT>
static hipError_t launch_mix_mode_t(const void* in, int pin, int64_t ips, void* out, int64_t ops,
                                    int64_t S, int64_t I, int64_t C, const void* W, int Kp,
                                    hipStream_t st) {
  if (2 * I <= 16) {
    hipLaunchKernelGGL((k_mix_small<TI, TM, TO>), dim3((unsigned)((S * C + 255) / 256)),
                       dim3(256), 0, st, (const TI*)in, pin, ips, (TO*)out, ops, S, (int)I, C,
                       (const TM*)W, Kp);
    return hipGetLastError();
  }
  const int nrt = (int)((2 * I + 15) / 16);
  const int rtw = (nrt + 3) / 4;
  const unsigned grid = (unsigned)((S * C + JT - 1) / JT);
#define TRK_MIX(R)                                                                              \
  hipLaunchKernelGGL((k_mix_mode<TI, TM, TO, JT, R>), dim3(grid), dim3(256), 0, st,            \
                     (const TI*)in, pin, ips, (TO*)out, ops, S, I, C, (const TM*)W, Kp)
  if (rtw <= 1)
    TRK_MIX(1);
  else if (rtw <= 2)
    TRK_MIX(2);
  else if (rtw <= 3)
    TRK_MIX(3);
  else if (rtw <= 5)
    TRK_MIX(5);
  else if (rtw <= 8)
    TRK_MIX(8);
  else
    return hipErrorInvalidValue;
#undef TRK_MIX
  return hipGetLastError();
}

int mix_k_padded(int64_t I, int pin) { return mix_kp(I, pin); }

hipError_t launch_mix_weights(int64_t I, int pin, const double* D, int cdt, void* W,
                              hipStream_t st) {
  const int Kp = mix_k_padded(I, pin);
  const unsigned grid = (unsigned)((2 * I * Kp + 255) / 256);
  if (cdt == F64)
    hipLaunchKernelGGL(k_mix_weights<double>, dim3(grid), dim3(256), 0, st, I, pin, D, Kp,
                       (double*)W);
  else if (cdt == F32)
    hipLaunchKernelGGL(k_mix_weights<float>, dim3(grid), dim3(256), 0, st, I, pin, D, Kp,
                       (float*)W);
  else
    hipLaunchKernelGGL(k_mix_weights<__bf16>, dim3(grid), dim3(256), 0, st, I, pin, D, Kp,
                       (__bf16*)W);
  return hipGetLastError();
}

hipError_t launch_mix_weights_all(const MixWeightsAll& a, int cdt, hipStream_t st) {
  if (a.count < 1 || a.count > MAXN) return hipErrorInvalidValue;
  int64_t emax = 1;
  for (int k = 0; k < a.count; ++k) {
    const int64_t e = 2 * a.I[k] * mix_kp(a.I[k], a.pin[k]);
    emax = e > emax ? e : emax;
  }
  const dim3 grid((unsigned)((emax + 255) / 256), (unsigned)a.count);
  if (cdt == F64)
    hipLaunchKernelGGL(k_mix_weights_all<double>, grid, dim3(256), 0, st, a);
  else if (cdt == F32)
    hipLaunchKernelGGL(k_mix_weights_all<float>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_mix_weights_all<__bf16>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mix_mode(const void* in, int idt, int pin, int64_t ips, void* out,
                           int64_t ops, int64_t S, int64_t I, int64_t C, const void* W, int cdt,
                           hipStream_t st) {
  if (I > 256 || pin < 1 || pin > 2) return hipErrorInvalidValue;
  const int Kp = mix_k_padded(I, pin);
  if (cdt == F64) {
    if (idt != F64) return hipErrorInvalidValue;
    return launch_mix_mode_t<double, double, double, 32>(in, pin, ips, out, ops, S, I, C, W, Kp,
                                                         st);
  }
  if (cdt == F32) {
    if (idt != F32) return hipErrorInvalidValue;
    return launch_mix_mode_t<float, float, float, 64>(in, pin, ips, out, ops, S, I, C, W, Kp, st);
  }
  if (idt == BF16)
    return launch_mix_mode_t<__hip_bfloat16, __bf16, float, 64>(in, pin, ips, out, ops, S, I, C,
                                                                W, Kp, st);
  if (idt == F32)
    return launch_mix_mode_t<float, __bf16, float, 64>(in, pin, ips, out, ops, S, I, C, W, Kp,
                                                       st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Sampled mixed core slices: GS[p][s][c] = plane p of
//   (1/sqrt(I)) sum_i exp(-2 pi i idx_s i / I) D[i] G(i)[c]
// for the m samples of a core with I slice-major FP64 rows of width d; the
// twiddles of one workgroup come from an LDS table of the I roots.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mix_slices(const double* __restrict__ G, int64_t I, int d,
                                                    const double* __restrict__ D,
                                                    const int* __restrict__ idx, int m,
                                                    double* __restrict__ GS) {
  extern __shared__ double tw[];            // [I] cos, [I] sin
  for (int64_t r = threadIdx.x; r < I; r += 256) twiddle(r, I, &tw[r], &tw[I + r]);
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * d) return;
  const int s = (int)(e / d), c = (int)(e - (int64_t)s * d);
  const int64_t step = idx[s];
  double re = 0.0, im = 0.0;
  int64_t r = 0;
  for (int64_t i = 0; i < I; ++i) {
    const double g = D[i] * G[i * d + c];
    re += tw[r] * g;
    im -= tw[I + r] * g;
    r += step;
    if (r >= I) r -= I;
  }
  const double sc = 1.0 / sqrt((double)I);
  GS[e] = re * sc;
  GS[(int64_t)m * d + e] = im * sc;
}

// Tiled form for I <= 448: a workgroup owns 16 samples x 16 columns and
// stages the twiddles and D G for its columns in LDS once, so G is read once
// per workgroup instead of once per sample; same sum, same order.
constexpr int MIX_TILE_MAXI = 448;     // (2 + 16) * 448 doubles fit the 64 KiB default

__global__ __launch_bounds__(256) void k_mix_slices_t(MixSlicesAll a) {
  extern __shared__ double sm[];
  const int k = blockIdx.z;
  const double* __restrict__ G = a.G[k];
  const double* __restrict__ D = a.D[k];
  const int* __restrict__ idx = a.idx[k];
  double* __restrict__ GS = a.GS[k];
  const int I = a.I[k], d = a.d[k], m = a.m;
  double* tw = sm;                          // [I] cos, [I] sin
  double* dg = sm + 2 * I;                  // [I][16]: D[i] G[i][c0 + j]
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * 16, s0 = blockIdx.y * 16;
  if (c0 >= d) return;                      // a narrower core of the batch
  for (int r = tid; r < I; r += 256) twiddle(r, I, &tw[r], &tw[I + r]);
  for (int e = tid; e < I * 16; e += 256) {
    const int i = e >> 4, j = e & 15;
    const int c = c0 + j < d ? c0 + j : d - 1;
    dg[e] = D[i] * G[(size_t)i * d + c];
  }
  __syncthreads();
  const int j = tid & 15, sl = tid >> 4;
  const int s = s0 + sl, c = c0 + j;
  if (s >= m || c >= d) return;
  const int step = idx[s];
  // four partial sums over i (independent FMA chains), added in a fixed
  // order; r = (i step) mod I walks the twiddle table
  double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
  int r = 0;
  int i = 0;
  for (; i + 4 <= I; i += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double gv = dg[(i + u) * 16 + j];
      re[u] += tw[r] * gv;
      im[u] -= tw[I + r] * gv;
      r += step;
      if (r >= I) r -= I;
    }
  }
  for (; i < I; ++i) {
    const double gv = dg[i * 16 + j];
    re[0] += tw[r] * gv;
    im[0] -= tw[I + r] * gv;
    r += step;
    if (r >= I) r -= I;
  }
  const double sc = 1.0 / sqrt((double)I);
  const int64_t e = (int64_t)s * d + c;
  GS[e] = ((re[0] + re[1]) + (re[2] + re[3])) * sc;
  GS[(int64_t)m * d + e] = ((im[0] + im[1]) + (im[2] + im[3])) * sc;
}

hipError_t launch_mix_slices(const double* G, int64_t I, int d, const double* D, const int* idx,
                             int m, double* GS, hipStream_t st) {
  if (I > 4096) return hipErrorInvalidValue;
  if (I <= MIX_TILE_MAXI) {
    MixSlicesAll a = {};
    a.count = 1;
    a.m = m;
    a.G[0] = G;
    a.I[0] = (int)I;
    a.d[0] = d;
    a.D[0] = D;
    a.idx[0] = idx;
    a.GS[0] = GS;
    return launch_mix_slices_all(a, st);
  }
  const unsigned grid = (unsigned)(((int64_t)m * d + 255) / 256);
  hipLaunchKernelGGL(k_mix_slices, dim3(grid), dim3(256), (size_t)2 * I * sizeof(double), st, G,
                     I, d, D, idx, m, GS);
  return hipGetLastError();
}

hipError_t launch_mix_slices_all(const MixSlicesAll& a, hipStream_t st) {
  if (a.count < 1 || a.count > MAXN) return hipErrorInvalidValue;
  int imax = 1, dmax = 1;
  for (int k = 0; k < a.count; ++k) {
    if (a.I[k] > MIX_TILE_MAXI || a.I[k] < 1 || a.d[k] < 1) return hipErrorInvalidValue;
    imax = a.I[k] > imax ? a.I[k] : imax;
    dmax = a.d[k] > dmax ? a.d[k] : dmax;
  }
  dim3 grid((unsigned)((dmax + 15) / 16), (unsigned)((a.m + 15) / 16), (unsigned)a.count);
  const size_t lds = (size_t)(2 * imax + 16 * imax) * sizeof(double);
  hipLaunchKernelGGL(k_mix_slices_t, grid, dim3(256), lds, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Complex sampled subchain rows of mode n (Alg. 3 on the mixed cores): row s
// is the product of the sampled slices GS_k[s] in ring order from n+1, in
// the mode-2 unfolding layout (column r + R_n srow).  Writes the stacked
// planes Ast = [Re A; Im A] (2m x d), the product operand
// Bst = [[w Re A, -w Im A], [w Im A, w Re A]] (2m x 2d) and the 2m weights;
// with `literal` (the literal temporal reading) Bst = [[Re A, 0], [0, Re A]].
// ---------------------------------------------------------------------------
// One sampled row per 16-lane group: lane b holds column b (both planes) of
// the running product; a slice product is 16 independent column loads per
// plane and 16 shuffles inside the group.
__global__ __launch_bounds__(256) void k_sample_rows_c(Geom g, const double* const* GS, int m,
                                                       double w, int literal,
                                                       double* __restrict__ Ast,
                                                       double* __restrict__ Bst,
                                                       double* __restrict__ w2) {
  const int N = g.N, n = g.n;
  const int Rn = g.R[n], Rn1 = g.R[n + 1 == N ? 0 : n + 1];
  const int d = g.d;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = threadIdx.x & 15;
  const int e = tid >> 4;
  const bool live = e < m * Rn1;
  const int ec = live ? e : 0;
  const int s = ec / Rn1, srow = ec - s * Rn1;
  double vr, vi;
  int q = n + 1 == N ? 0 : n + 1;
  {
    const int Ra = g.R[q], Rb = g.R[q + 1 == N ? 0 : q + 1], dq = Ra * Rb;
    const double* re = GS[q] + (size_t)s * dq;
    const double* im = GS[q] + (size_t)m * dq + (size_t)s * dq;
    const int bc = b < Rb ? b : 0;
    const double xr = re[srow + Ra * bc], xi = im[srow + Ra * bc];
    vr = b < Rb ? xr : 0.0;
    vi = b < Rb ? xi : 0.0;
  }
  for (int j = 1; j < N - 1; ++j) {
    q = q + 1 == N ? 0 : q + 1;
    const int Ra = g.R[q], Rb = g.R[q + 1 == N ? 0 : q + 1], dq = Ra * Rb;
    const double* re = GS[q] + (size_t)s * dq;
    const double* im = GS[q] + (size_t)m * dq + (size_t)s * dq;
    const int bc = b < Rb ? b : 0;
    double hr[16], hi[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int ac = a < Ra ? a : 0;                 // loads stay inside the slice
      const double xr = re[ac + Ra * bc], xi = im[ac + Ra * bc];
      const bool ok = a < Ra && b < Rb;
      hr[a] = ok ? xr : 0.0;
      hi[a] = ok ? xi : 0.0;
    }
    double ur = 0.0, ui = 0.0;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const double pr = __shfl(vr, a, 16), pi = __shfl(vi, a, 16);
      ur = fma(pr, hr[a], fma(-pi, hi[a], ur));
      ui = fma(pr, hi[a], fma(pi, hr[a], ui));
    }
    vr = ur;
    vi = ui;
  }
  if (live && b < Rn) {
    const int c = b + Rn * srow;
    const double are = vr, aim = vi;
    Ast[(size_t)s * d + c] = are;
    Ast[(size_t)(m + s) * d + c] = aim;
    Bst[(size_t)s * 2 * d + c] = literal ? are : w * are;
    Bst[(size_t)s * 2 * d + d + c] = literal ? 0.0 : -w * aim;
    Bst[(size_t)(m + s) * 2 * d + c] = literal ? 0.0 : w * aim;
    Bst[(size_t)(m + s) * 2 * d + d + c] = literal ? are : w * are;
  }
  if (live && srow == 0 && b == 0) {
    w2[s] = w;
    w2[m + s] = w;
  }
}

hipError_t launch_sample_rows_c(const Geom& g, const double* const* GS, int m, double w,
                                int literal, double* Ast, double* Bst, double* w2,
                                hipStream_t st) {
  for (int k = 0; k < g.N; ++k)
    if (g.R[k] > 16) return hipErrorInvalidValue;
  const int Rn1 = g.R[g.n + 1 == g.N ? 0 : g.n + 1];
  const unsigned grid = (unsigned)(((int64_t)m * Rn1 * 16 + 255) / 256);
  hipLaunchKernelGGL(k_sample_rows_c, dim3(grid), dim3(256), 0, st, g, GS, m, w, literal, Ast, Bst,
                     w2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sketched product over stacked planes: part[split][i][c] = sum over the
// split's K indices k of Xg[i][k] B[k][c], with Xg[:, k] the mode-n fibre of
// plane k / m of the mixed tensor at the indices of sample k % m, and B a
// dense (2m x dB) FP64 matrix.  KC = 32 K indices per chunk staged in LDS in
// the MFMA operand precision; each wave owns output blocks wave, wave+4, ...
// ---------------------------------------------------------------------------
template <typename TX, typename TM, int MAXB>
__global__ __launch_bounds__(256) void k_sgemm(Geom g, int MT, int dB, int64_t pstride,
                                               const TX* __restrict__ X,
                                               const int* __restrict__ idxs, int m, int kchunks,
                                               const double* __restrict__ B,
                                               typename Mf<TM>::out* __restrict__ part) {
  typedef Mf<TM> M;
  typedef typename M::acc ACC;
  constexpr int KCH = 32;
  constexpr int KCP = KCH + (M::KPL == 8 ? 8 : 1);
  extern __shared__ __align__(16) char smem[];
  const int NB = (dB + 15) >> 4, NTP = NB * 16;
  int64_t* off = (int64_t*)smem;                       // [KCH]
  TM* Bs = (TM*)(off + KCH);                           // [NTP][KCP]
  TM* As = Bs + NTP * KCP;                             // [MT][KCP]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int split = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * MT;
  const int nblk = (MT >> 4) * NB;
  const int K2 = 2 * m;
  const int k_beg = split * kchunks * KCH;
  const int k_end = k_beg + kchunks * KCH < K2 ? k_beg + kchunks * KCH : K2;
  int64_t stride[MAXN];
  {
    int64_t a = 1;
    for (int q = 0; q < g.N; ++q) {
      stride[q] = a;
      a *= g.I[q];
    }
  }
  ACC acc[MAXB];
#pragma unroll
  for (int bi = 0; bi < MAXB; ++bi) acc[bi] = ACC{0, 0, 0, 0};
  for (int kb = k_beg; kb < k_end; kb += KCH) {
    if (tid < KCH) {
      const int k = kb + tid;
      int64_t o = -1;
      if (k < k_end) {
        const int s = k % m, p = k / m;
        o = p * pstride;
        for (int q = 0; q < g.N; ++q)
          if (q != g.n) o += (int64_t)idxs[(size_t)q * m + s] * stride[q];
      }
      off[tid] = o;
    }
    __syncthreads();
    // staging in batches of 8 elements per thread with every load of a
    // batch in flight (indices clamped in range, the selects after the loads)
    for (int e0 = tid; e0 < KCH * NTP; e0 += 256 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e / NTP, c = e - kk * NTP;
        const int k = kb + kk;
        const bool ok = e < KCH * NTP && k < k_end && c < dB;
        const int kc = k < k_end ? k : k_end - 1, cc = c < dB ? c : dB - 1;
        const double x = B[(size_t)kc * dB + cc];
        v[u] = ok ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e / NTP, c = e - kk * NTP;
        if (e < KCH * NTP) Bs[c * KCP + kk] = from_double<TM>(v[u]);
      }
    }
    for (int e0 = tid; e0 < MT * KCH; e0 += 256 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e % KCH, mm = e / KCH;
        const int64_t mg = m0 + mm;
        const bool ok = e < MT * KCH && mg < g.In && off[kk] >= 0;
        const int64_t o = ok ? off[kk] + mg * stride[g.n] : 0;
        const double x = (double)X[o];
        v[u] = ok ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        const int kk = e % KCH, mm = e / KCH;
        if (e < MT * KCH) As[mm * KCP + kk] = from_double<TM>(v[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KCH; ks += 4 * M::KPL) {
      const int kk = ks + g4 * M::KPL;
#pragma unroll
      for (int bi = 0; bi < MAXB; ++bi) {
        int b = wave + 4 * bi;
        b = b < nblk ? b : nblk - 1;
        const int rb = b / NB, cb = b - rb * NB;
        acc[bi] = M::op(load_frag<TM>(&As[(rb * 16 + l16) * KCP + kk]),
                        load_frag<TM>(&Bs[(cb * 16 + l16) * KCP + kk]), acc[bi]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < MAXB; ++bi) {
    const int b = wave + 4 * bi;
    if (b < nblk) {
      const int rb = b / NB, cb = b - rb * NB;
      const int col = cb * 16 + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t mg = m0 + rb * 16 + M::row(lane, v);
        if (mg < g.In && col < dB) part[((size_t)split * g.In + mg) * dB + col] = acc[bi][v];
      }
    }
  }
}

SgemmPlan plan_sgemm(const Geom& g, int m, int dB, int cdt) {
  SgemmPlan p;
  const int NB = (dB + 15) / 16;
  int MT = (int)((g.In + 15) / 16) * 16;
  if (MT > 64) MT = 64;
  const int maxblk = cdt == F64 ? 32 : 64;
  while (MT > 16 && (MT / 16) * NB > maxblk) MT -= 16;
  p.MT = MT;
  p.mtiles = (int)((g.In + MT - 1) / MT);
  p.psize = cdt == F64 ? 8 : 4;
  p.nblk = (MT / 16) * NB;
  // K splits: about 512 workgroups, partials at most 16 MiB
  const int chunks = (2 * m + 31) / 32;
  int64_t ns = (512 + p.mtiles - 1) / p.mtiles;
  const int64_t budget = ((int64_t)16 << 20) / ((int64_t)g.In * dB * p.psize);
  if (ns > budget) ns = budget;
  if (ns > chunks) ns = chunks;
  if (ns < 1) ns = 1;
  p.kchunks = (int)((chunks + ns - 1) / ns);
  p.nsplit = (chunks + p.kchunks - 1) / p.kchunks;
  return p;
}

template <typename TX, typename TM, int MAXB>
static hipError_t launch_sgemm_t(const Geom& g, const SgemmPlan& p, int dB, int64_t pstride,
                                 const void* X, const int* idxs, int m, const double* B,
                                 void* part, hipStream_t st) {
  constexpr int KCP = 32 + (Mf<TM>::KPL == 8 ? 8 : 1);
  const int NTP = ((dB + 15) / 16) * 16;
  const size_t lds = 32 * sizeof(int64_t) + (size_t)(NTP + p.MT) * KCP * sizeof(TM);
  auto fn = k_sgemm<TX, TM, MAXB>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(p.nsplit, p.mtiles), dim3(256), lds, st, g, p.MT, dB, pstride,
                     (const TX*)X, idxs, m, p.kchunks, B, (typename Mf<TM>::out*)part);
  return hipGetLastError();
}

template <typename TX, typename TM>
static hipError_t launch_sgemm_b(const Geom& g, const SgemmPlan& p, int dB, int64_t pstride,
                                 const void* X, const int* idxs, int m, const double* B,
                                 void* part, hipStream_t st) {
  const int per = (p.nblk + 3) / 4;
  if (per <= 4) return launch_sgemm_t<TX, TM, 4>(g, p, dB, pstride, X, idxs, m, B, part, st);
  if (per <= 8) return launch_sgemm_t<TX, TM, 8>(g, p, dB, pstride, X, idxs, m, B, part, st);
  return launch_sgemm_t<TX, TM, 16>(g, p, dB, pstride, X, idxs, m, B, part, st);
}

hipError_t launch_sgemm(const Geom& g, const SgemmPlan& p, int dB, int64_t pstride,
                        const void* X, int cdt, const int* idxs, int m, const double* B,
                        void* part, hipStream_t st) {
  if (p.nblk > 64) return hipErrorInvalidValue;
  if (cdt == F64)
    return launch_sgemm_b<double, double>(g, p, dB, pstride, X, idxs, m, B, part, st);
  if (cdt == F32) return launch_sgemm_b<float, float>(g, p, dB, pstride, X, idxs, m, B, part, st);
  return launch_sgemm_b<float, __bf16>(g, p, dB, pstride, X, idxs, m, B, part, st);
}

// ---------------------------------------------------------------------------
// Unmixing of mode n applied to Z = [Re | Im] (I x 2d, FP64):
//   dP[i][c] = D[i] / sqrt(I) sum_j (cos(2 pi i j / I) Re Z[j][c]
//                                    - sin(2 pi i j / I) Im Z[j][c])
// = Re(D_n F_n^* Z).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_unmix(const double* __restrict__ Z, int64_t I, int d,
                                               const double* __restrict__ D,
                                               double* __restrict__ dP) {
  extern __shared__ double tw[];            // [I] cos, [I] sin
  for (int64_t r = threadIdx.x; r < I; r += 256) twiddle(r, I, &tw[r], &tw[I + r]);
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= I * d) return;
  const int64_t i = e / d;
  const int c = (int)(e - i * d);
  double acc = 0.0;
  int64_t r = 0;
  for (int64_t j = 0; j < I; ++j) {
    acc += tw[r] * Z[j * 2 * d + c] - tw[I + r] * Z[j * 2 * d + d + c];
    r += i;
    if (r >= I) r -= I;
  }
  dP[e] = D[i] * acc / sqrt((double)I);
}

hipError_t launch_unmix(const double* Z, int64_t I, int d, const double* D, double* dP,
                        hipStream_t st) {
  if (I > 4096) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((I * d + 255) / 256);
  hipLaunchKernelGGL(k_unmix, dim3(grid), dim3(256), (size_t)2 * I * sizeof(double), st, Z, I, d,
                     D, dP);
  return hipGetLastError();
}

}  // namespace trk
