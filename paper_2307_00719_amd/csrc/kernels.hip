// gfx950 kernels of the streaming tensor-ring tracker.
//
// Notation (0-based, mode N-1 temporal): a TR-core G_k has lateral slices
// G_k(i) of size R_k x R_{k+1} (Sec. 1).  For mode n the subchain slice of a
// column k = l + L*rr of X_[n] is
//     S(k) = G_{n+1}(i_{n+1}) ... G_{N-1}(i_{N-1}) G_0(i_0) ... G_{n-1}(i_{n-1})
// (Def. subchain tensor) and G^{!=n}_[2][k, r + R_n*s] = S(k)[s, r]
// (the mode-2 unfolding of Sec. 2).  The per-batch products of Alg. 4 are
// P_n += X_[n] G^{!=n}_[2] (the MTTKRP-like product) and the Gram chain of
// Prop. subchain Gram.

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "bf16_round.h"
#include <stdint.h>

#include <algorithm>

#include "tr_internal.h"

namespace trk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Accumulator type and the row held by register v of `lane` in a 16x16
// MFMA result block (column lane % 16): the FP64 16x16x4 instruction keeps
// rows lane/16 + 4v, the FP32 one rows 4(lane/16) + v.
template <typename T> struct Acc;
template <> struct Acc<double> {
  typedef double type;
  typedef d4 vec;
  static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Acc<float> {
  typedef float type;
  typedef f4 vec;
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

Geom make_geom(int N, const int64_t* I, const int* R, int n) {
  Geom g;
  g.N = N;
  g.n = n;
  for (int k = 0; k < MAXN; ++k) {
    g.I[k] = k < N ? I[k] : 1;
    g.R[k] = k < N ? R[k] : 1;
  }
  g.L = 1;
  for (int k = 0; k < n; ++k) g.L *= I[k];
  g.In = I[n];
  g.Rr = 1;
  for (int k = n + 1; k < N; ++k) g.Rr *= I[k];
  g.d = R[n] * R[(n + 1) % N];
  return g;
}

static int pad16(int64_t x) { return (int)((x + 15) / 16) * 16; }

// ---------------------------------------------------------------------------
// Subchain row: v = e_s^T S(k), i.e. row s of S(k), of length R_n.
// idx holds i_q for every q != n of column k.  (Reconstruction kernel.)
// ---------------------------------------------------------------------------
template <typename TC, int RM>
__device__ inline void subchain_row(const Geom& g, const CoreView& cv, const int* idx, int s,
                                    TC (&v)[RM]) {
  const int N = g.N;
  int q = g.n + 1 == N ? 0 : g.n + 1;
  {
    const TC* G = (const TC*)cv.ptr[q] + idx[q] * cv.si[q] + s * cv.sr[q];
    const int Rq1 = g.R[q + 1 == N ? 0 : q + 1];
    const int64_t ss = cv.ss[q];
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = (b < Rq1) ? G[b * ss] : TC(0);
  }
  for (int j = 1; j < N - 1; ++j) {
    q = q + 1 == N ? 0 : q + 1;
    const TC* H = (const TC*)cv.ptr[q] + idx[q] * cv.si[q];
    const int Rq = g.R[q];
    const int Rq1 = g.R[q + 1 == N ? 0 : q + 1];
    const int64_t sr = cv.sr[q], ss = cv.ss[q];
    TC u[RM];
#pragma unroll
    for (int b = 0; b < RM; ++b) {
      TC acc = TC(0);
      if (b < Rq1) {
#pragma unroll
        for (int a = 0; a < RM; ++a)
          if (a < Rq) acc += v[a] * H[a * sr + b * ss];
      }
      u[b] = acc;
    }
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = u[b];
  }
}

// Decode column k of X_[n] into its X offset (without the i_n term) and the
// multi-index of every other mode.
__device__ inline int64_t decode_column(const Geom& g, int64_t k, int* idx) {
  int64_t l = k % g.L, rr = k / g.L;
  const int64_t off = l + g.L * g.In * rr;
  for (int q = 0; q < g.n; ++q) {
    idx[q] = (int)(l % g.I[q]);
    l /= g.I[q];
  }
  for (int q = g.n + 1; q < g.N; ++q) {
    idx[q] = (int)(rr % g.I[q]);
    rr /= g.I[q];
  }
  idx[g.n] = 0;
  return off;
}

MttkrpPlan plan_mttkrp(const Geom& g, int xdtype, int max_wg, bool bulk) {
  MttkrpPlan p;
  const int N = g.N;
  p.zform = 0;
  p.prv = 0;
  p.prv_in = 0;
  p.ng = 1;
  p.MT = 16;
  p.mtiles = (int)((g.In + 15) / 16);
  p.psize = (xdtype == F64) ? 8 : 4;
  p.f = g.n == 0 ? 1 : 0;
  const int f = p.f;
  const int df = g.R[f] * g.R[(f + 1) % N];
  p.nbf = (df + 15) / 16;
  p.KS = p.nbf <= 4 ? 4 : (p.nbf <= 8 ? 2 : 1);
  const int64_t If = g.I[f];
  p.Q = (int)((If + 4 * p.KS - 1) / (4 * p.KS));
  p.Kout = g.L * g.Rr / If;
  if (g.n == 0) {
    p.sf = g.I[0];      // X[m + I_0*(i_1 + I_1*o)]
    p.sm = 1;
  } else {
    p.sf = 1;           // X[i_0 + I_0*l_hi + m*L + L*In*rr]
    p.sm = g.L;
  }
  // outer indices per workgroup: about 512 workgroups, and the partials
  // (one I_n x d block per chunk) at most half the bytes of X
  const int64_t xbytes = g.L * g.Rr * g.In * (xdtype == F64 ? 8 : (xdtype == F32 ? 4 : 2));
  int64_t chunks = (512 + p.mtiles - 1) / p.mtiles;
  const int64_t by_bytes = xbytes / (2 * (int64_t)g.In * g.d * p.psize);
  if (chunks > by_bytes) chunks = by_bytes;
  if (max_wg > 0 && chunks > max_wg / p.mtiles) chunks = max_wg / p.mtiles;
  if (chunks > p.Kout) chunks = p.Kout;
  if (chunks < 1) chunks = 1;
  if (const char* e = getenv("TRSTREAM_NSPLIT")) {
    int64_t v = atoll(e);
    if (v > 0) chunks = v < p.Kout ? v : p.Kout;
  }
  p.upw = (p.Kout + chunks - 1) / chunks;
  p.nsplit = (int)((p.Kout + p.upw - 1) / p.upw);
  if (bulk && xdtype == F32 && If <= 64) {
    bool small = N <= 4;
    for (int k = 0; k < N; ++k) small = small && g.R[k] <= 16;
    // one 8-wave workgroup per CU (its two Z buffers take 136 KiB of LDS):
    // about 256 workgroups (fewer under max_wg) of 64 rows, or of 32 or 16
    // when I_n is that small, at least two outer indices each
    const int rows_wg = g.In <= 16 ? 16 : (g.In <= 32 ? 32 : 64);
    const int64_t mg = (g.In + rows_wg - 1) / rows_wg;
    int64_t zc = 256 / mg;
    if (max_wg > 0 && zc > max_wg / mg) zc = max_wg / mg;
    if (zc < 1) zc = 1;
    if (small && p.Kout >= 2 * zc) {
      p.zform = 1;
      p.MT = rows_wg;
      p.upw = (p.Kout + zc - 1) / zc;
      p.nsplit = (int)((p.Kout + p.upw - 1) / p.upw);
    }
  }
  return p;
}

size_t mttkrp_partial_bytes(const Geom& g, const MttkrpPlan& p) {
  const size_t b = (size_t)p.nsplit * (size_t)g.In * (size_t)g.d * (size_t)p.psize;
  if (!p.prv) return b;
  // one partial row of R_2 R_0 per (row tile, t)
  const size_t bp = (size_t)p.mtiles * (size_t)p.prv_in * (size_t)(g.R[2] * g.R[0]) * p.psize;
  return b > bp ? b : bp;
}

// Index i_q (q != n, f) of outer index o of mode n, in the enumeration of
// decode_outer.
__device__ inline int outer_index(const Geom& g, int64_t o, int q) {
  int64_t t;
  int q0;
  if (g.n == 0) {
    t = o;
    q0 = 2;
  } else if (q < g.n) {
    t = o % (g.L / g.I[0]);
    q0 = 1;
  } else {
    t = o / (g.L / g.I[0]);
    q0 = g.n + 1;
  }
  for (int p = q0; p < q; ++p) t /= g.I[p];
  return (int)(t % g.I[q]);
}

// Ring product of nfac slices from mode q0 on, at the indices of outer index
// o, into the 16 x 16 LDS matrix M (zero padded); tmp is 256 doubles of
// scratch.  Every slice is staged in LDS with one load per thread (zero
// padded), so a product is a fixed 16-term sum over LDS.  Ends with a
// workgroup barrier.
template <typename TC>
__device__ inline void ring_product_lds(const Geom& g, const CoreView& cv, int64_t o, int q0,
                                        int nfac, double* M, double* tmp, int tid) {
  const int N = g.N;
  const int a = tid >> 4, b = tid & 15;
  int q = q0;
  {
    const int Ra = g.R[q], Rb = g.R[q + 1 == N ? 0 : q + 1];
    const bool ok = a < Ra && b < Rb;
    const TC* G = (const TC*)cv.ptr[q] + (int64_t)outer_index(g, o, q) * cv.si[q];
    const double v = (double)G[ok ? a * cv.sr[q] + b * cv.ss[q] : 0];
    M[tid] = ok ? v : 0.0;
  }
  for (int j = 1; j < nfac; ++j) {
    q = q + 1 == N ? 0 : q + 1;
    const int Rq = g.R[q], Rc = g.R[q + 1 == N ? 0 : q + 1];
    const bool ok = a < Rq && b < Rc;
    const TC* H = (const TC*)cv.ptr[q] + (int64_t)outer_index(g, o, q) * cv.si[q];
    const double v = (double)H[ok ? a * cv.sr[q] + b * cv.ss[q] : 0];
    tmp[tid] = ok ? v : 0.0;
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = fma(M[a * 16 + k], tmp[k * 16 + b], acc);
    __syncthreads();
    M[tid] = acc;
  }
  __syncthreads();
}

// X offset of (i_f = 0, i_n = 0) for outer index o of mode n.
__device__ inline int64_t outer_offset(const Geom& g, int64_t o) {
  if (g.n == 0) return g.I[0] * g.I[1] * o;
  const int64_t Lh = g.L / g.I[0];
  const int64_t l_hi = o % Lh, rr = o / Lh;
  return g.I[0] * l_hi + g.L * g.In * rr;
}

// ---------------------------------------------------------------------------
// MTTKRP: part[chunk][m][c] = sum over the chunk's outer indices o and all
// i_f of X_[n][m, (o, i_f)] * G^{!=n}_[2][(o, i_f), c].
// The columns of X_[n] are split as (o, i_f), f the fastest mode other than
// n, and the subchain slice factors as S(o, i_f) = U(o) G_f(i_f) V(o) (U the
// ring product of the modes n+1 .. f-1, V of f+1 .. n-1), so
//   P[m, r + R_n s] = sum_o sum_{a,b} U(o)[s,a] Y_o[m, a + R_f b] V(o)[b,r],
//   Y_o[m, :] = sum_{i_f} X[m, o, i_f] G_f(i_f)          (a GEMM, K = I_f).
// One workgroup: 16 rows m x one chunk of o.  The GEMM runs on 16x16x4
// MFMAs with both operands read straight into registers; the 4 waves split
// K in KS parts and the column tiles of R_f R_{f+1} in 4/KS parts.  Lane
// group g of K-part w handles the Q consecutive i_f from (4w + g) Q, so a
// lane's loads walk contiguous memory when i_f is the unit-stride mode.
// The K parts are summed in LDS in a fixed order, then U and V are applied
// in FP64 and the result accumulated over the chunk.
// ---------------------------------------------------------------------------
template <typename T, typename TC, int NJ, int BQ = 0, int NG = 1, bool PRV = false>
__device__ inline void mttkrp_body(const Geom& g, const MttkrpPlan& p, const T* __restrict__ X,
                                   const CoreView& cv, typename Acc<T>::type* __restrict__ part,
                                   int chunk, int mtile, char* smem) {
  typedef typename Acc<T>::type PT;
  typedef typename Acc<T>::vec V4;
  constexpr int KG = 8;                     // k-steps whose loads are issued together
  // NG groups of four waves take NG consecutive outer indices of the chunk
  // at a time, each with its own LDS region; the groups run the same phases
  // (barriers are workgroup-wide), a group past the chunk's end contributing
  // zeros
  const int grp = NG > 1 ? (int)(threadIdx.x >> 8) : 0;
  const int tid = threadIdx.x & 255, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int N = g.N, n = g.n, f = p.f;
  const int Rn = g.R[n], Rn1 = g.R[n + 1 == N ? 0 : n + 1];
  const int Rf = g.R[f], Rf1 = g.R[f + 1 == N ? 0 : f + 1];
  const int df = Rf * Rf1, nbf = p.nbf, dfp = 16 * nbf, dn = g.d;
  const int KS = p.KS, CS = 4 / KS;
  const int kslot = wave % KS, cslot = wave / KS;
  const int g4 = lane >> 4, l16 = lane & 15;
  const int If = (int)g.I[f];
  const int Q = p.Q;
  const int kbase = (kslot * 4 + g4) * Q;
  const int nU = (f - (n + 1) + N) % N;
  const int nV = (n - (f + 1) + N) % N;
  constexpr bool prv = PRV;
  const int qU = n + 1 == N ? 0 : n + 1;
  const int qV = f + 1 == N ? 0 : f + 1;
  const int wst = 16 * ((Rn1 * Rf1 + 15) / 16);

  // bytes of one group's LDS region (the launcher's per-group size)
  const size_t gbytes = (((size_t)(3 * 256 + 16 * wst) * sizeof(double) +
                          (size_t)(16 * dfp) * KS * sizeof(PT)) + 15) & ~(size_t)15;
  if constexpr (NG > 1) smem += grp * gbytes;
  double* Us = (double*)smem;               // [16][16]
  double* Vs = Us + 256;                    // [16][16]
  double* tmp = Vs + 256;                   // [256]
  double* Ws = tmp + 256;                   // [16][wst]
  PT* Ys = (PT*)(Ws + 16 * wst);            // [16][dfp]
  PT* red = Ys + 16 * dfp;                  // [KS-1][16][dfp]

  const int64_t m0 = (int64_t)mtile * 16;
  const int64_t o0 = (int64_t)chunk * p.upw;
  const int64_t o1 = o0 + p.upw < p.Kout ? o0 + p.upw : p.Kout;
  const TC* __restrict__ Gf = (const TC*)cv.ptr[f];
  // 32-bit element offsets: the launcher checks that X spans of one outer
  // index and the core G_f fit
  const int fsi = (int)cv.si[f], sf = (int)p.sf;
  int boff[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    int c = (cslot + CS * j) * 16 + l16;
    c = c < df ? c : df - 1;
    boff[j] = (int)((c % Rf) * cv.sr[f] + (c / Rf) * cv.ss[f]);
  }
  const int mrow = (int)(m0 + l16 < g.In ? m0 + l16 : g.In - 1);
  const bool mok = m0 + l16 < g.In;
  const int arow = (int)(mrow * p.sm);
  d4 pacc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) pacc[t] = d4{0, 0, 0, 0};
  // BQ > 0 (Q <= BQ, checked by the launcher): the wave's G_f operands are
  // the same for every outer index, so they are loaded once into registers
  // and only the X tile is loaded per outer index
  T bres[BQ > 0 ? BQ : 1][NJ];
  if constexpr (BQ > 0) {
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int k = kbase + q;
      const bool ok = q < Q && k < If;
      const int kcl = k < If ? k : If - 1;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const TC b = Gf[kcl * fsi + boff[j]];
        bres[q][j] = ok ? (T)b : T(0);
      }
    }
  }

  for (int64_t oo = o0; oo < o1; oo += NG) {
    const bool ovalid = oo + grp < o1;
    const int64_t o = ovalid ? oo + grp : o1 - 1;
    const bool mok_o = mok && ovalid;
    const T* __restrict__ Xo = X + outer_offset(g, o);
    if (nU > 0 && !prv) ring_product_lds<TC>(g, cv, o, qU, nU, Us, tmp, tid);
    if (nV > 0 && !prv) ring_product_lds<TC>(g, cv, o, qV, nV, Vs, tmp, tid);
    // GEMM part: acc[j] = 16 x 16 tile (rows m, columns cslot + CS j) of
    // this wave's K part; the loads of KG k-steps are issued before their
    // MFMAs, and out-of-range k contribute zeros
    V4 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = V4{0, 0, 0, 0};
    if constexpr (BQ > 0) {
      T av[BQ];
#pragma unroll
      for (int q = 0; q < BQ; ++q) {
        const int k = kbase + q;
        const bool ok = q < Q && k < If;
        const int kcl = k < If ? k : If - 1;
        const T x = Xo[arow + kcl * sf];
        av[q] = ok && mok_o ? x : T(0);
      }
#pragma unroll
      for (int q = 0; q < BQ; ++q) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = mfma16(av[q], bres[q][j], acc[j]);
      }
    }
#pragma unroll 1
    for (int kc = 0; kc < (BQ > 0 ? 0 : Q); kc += KG) {
      T av[KG], bv[KG][NJ];
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const int k = kbase + kc + q;
        const bool ok = kc + q < Q && k < If;
        const int kcl = k < If ? k : If - 1;
        const T x = Xo[arow + kcl * sf];
        av[q] = ok && mok_o ? x : T(0);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const TC b = Gf[kcl * fsi + boff[j]];
          bv[q][j] = ok ? (T)b : T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < KG; ++q) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = mfma16(av[q], bv[q][j], acc[j]);
      }
    }
    // sum the K parts in a fixed order into Ys
    if (kslot > 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int cb = cslot + CS * j;
        if (cb < nbf) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            red[((kslot - 1) * 16 + Acc<T>::row(lane, v)) * dfp + cb * 16 + l16] = acc[j][v];
        }
      }
    }
    __syncthreads();
    if (kslot == 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int cb = cslot + CS * j;
        if (cb < nbf) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = Acc<T>::row(lane, v);
            PT s = acc[j][v];
            for (int ks = 1; ks < KS; ++ks) s += red[((ks - 1) * 16 + r) * dfp + cb * 16 + l16];
            Ys[r * dfp + cb * 16 + l16] = s;
          }
        }
      }
    }
    __syncthreads();
    if constexpr (prv) {
      // order-3 temporal mode in mode 1's geometry: rows are i_1 and the
      // outer index is t, so P_2[t][r + R_2 s] gets
      //   sum_m sum_b Y[m][s + R_0 b] G_1(i_1 = m0 + m)[b][r]
      // over this tile's 16 rows: the slices staged in Ws, one output
      // column per lane, the four row groups of the workgroup's waves
      // summed in LDS in a fixed order; one partial row per (row tile, t)
      const int R0 = g.R[0], R1 = g.R[1], R2 = g.R[2], d12 = R1 * R2, dout = R2 * R0;
      const TC* __restrict__ G1 = (const TC*)cv.ptr[1];
      for (int e = tid; e < 16 * d12; e += 256) {
        const int m = e / d12, k = e - m * d12;
        const int64_t i = m0 + m < g.In ? m0 + m : g.In - 1;
        Ws[m * wst + k] = (double)G1[i * cv.si[1] + (k % R1) * cv.sr[1] + (k / R1) * cv.ss[1]];
      }
      __syncthreads();
      const int out = tid & 63, rg = tid >> 6, r = out % R2, sx = out / R2;
      double acc = 0.0;
      if (out < dout) {
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          const int m = 4 * rg + mm;
          for (int b = 0; b < R1; ++b)
            acc = fma((double)Ys[m * dfp + sx + R0 * b], Ws[m * wst + b + R1 * r], acc);
        }
      }
      Us[rg * 64 + out] = acc;
      __syncthreads();
      if (tid < dout && ovalid) {
        const double v = ((Us[tid] + Us[64 + tid]) + Us[128 + tid]) + Us[192 + tid];
        part[((size_t)mtile * p.prv_in + o) * dout + tid] = (PT)v;
      }
      __syncthreads();
      continue;
    }
    // Contraction with U and V on FP64 MFMAs (16x16x4; the K index a or b
    // padded to 16 with zeros, U and V are zero-padded 16 x 16 in LDS):
    //   W_b = Y_b U^T       (W[m][s + Rn1 b] = sum_a U[s][a] Y[m][a + Rf b]),
    //   P_s += W_s V        (P[m][r + Rn s] += sum_b W[m][s + Rn1 b] V[b][r]),
    // tile b and tile s owned by wave b % 4 and s % 4; P_s stays in
    // registers across the chunk's outer indices.
    if (nU > 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int bb = wave + 4 * t;
        if (bb < Rf1) {
          d4 wt = {0, 0, 0, 0};
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4) {
            const int ka = k0 + g4;
            const double av = ka < Rf ? (double)Ys[l16 * dfp + ka + Rf * bb] : 0.0;
            wt = mfma16(av, Us[l16 * 16 + ka], wt);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (l16 < Rn1) Ws[Acc<double>::row(lane, v) * wst + l16 + Rn1 * bb] = wt[v];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ss = wave + 4 * t;
      if (ss < Rn1) {
        if (nV > 0) {
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4) {
            const int kb = k0 + g4;
            double av = 0.0;
            if (kb < Rf1)
              av = nU > 0 ? Ws[l16 * wst + ss + Rn1 * kb] : (double)Ys[l16 * dfp + ss + Rn1 * kb];
            pacc[t] = mfma16(av, Vs[kb * 16 + l16], pacc[t]);
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = Acc<double>::row(lane, v);
            double wv = 0.0;
            if (l16 < Rn)
              wv = nU > 0 ? Ws[m * wst + ss + Rn1 * l16] : (double)Ys[m * dfp + ss + Rn1 * l16];
            pacc[t][v] += wv;
          }
        }
      }
    }
    __syncthreads();
  }
  if constexpr (prv) return;
  if constexpr (NG > 1) {
    // the groups' sums added in group order through the LDS region of
    // group 1 (free after the loop's last barrier)
    if (grp == 1) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) ((double*)smem)[(t * 4 + v) * 256 + tid] = pacc[t][v];
    }
    __syncthreads();
    if (grp != 0) return;
    const double* o1s = (const double*)(smem + gbytes);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) pacc[t][v] += o1s[(t * 4 + v) * 256 + tid];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ss = wave + 4 * t;
    if (ss < Rn1 && l16 < Rn) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = Acc<double>::row(lane, v);
        if (m0 + m < g.In)
          part[((size_t)chunk * g.In + m0 + m) * dn + l16 + Rn * ss] = (PT)pacc[t][v];
      }
    }
  }
}

template <typename T, typename TC, int NJ, int BQ>
__global__ __launch_bounds__(256, 2) void k_mttkrp(Geom g, MttkrpPlan p, const T* __restrict__ X,
                                                   CoreView cv,
                                                   typename Acc<T>::type* __restrict__ part) {
  extern __shared__ __align__(16) char smem[];
  mttkrp_body<T, TC, NJ, BQ>(g, p, X, cv, part, blockIdx.x, blockIdx.y, smem);
}

template <typename T, typename TC, int NJ>
static hipError_t launch_mttkrp_t(const Geom& g, const MttkrpPlan& p, const void* X,
                                  const CoreView& cv, void* part, hipStream_t st) {
  typedef typename Acc<T>::type PT;
  const int dfp = 16 * p.nbf;
  const int Rn1 = g.R[(g.n + 1) % g.N], Rf1 = g.R[(p.f + 1) % g.N];
  const int wst = 16 * ((Rn1 * Rf1 + 15) / 16);
  const size_t lds = (size_t)(3 * 256 + 16 * wst) * sizeof(double) +
                     (size_t)(16 * dfp) * p.KS * sizeof(PT);
  // FP32 operands with at most 16 k-steps per lane group: the G_f operands
  // stay in registers across the outer indices (64 VGPRs at NJ = 4)
  auto fn = k_mttkrp<T, TC, NJ, 0>;
  if constexpr (sizeof(T) == 4) {
    if (p.Q <= 16) fn = k_mttkrp<T, TC, NJ, 16>;
  }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid(p.nsplit, p.mtiles);
  hipLaunchKernelGGL(fn, grid, dim3(256), lds, st, g, p, (const T*)X, cv,
                     (typename Acc<T>::type*)part);
  return hipGetLastError();
}

template <typename T, typename TC>
static hipError_t launch_mttkrp_j(const Geom& g, const MttkrpPlan& p, const void* X,
                                  const CoreView& cv, void* part, hipStream_t st) {
  const int nj = (p.nbf + 4 / p.KS - 1) / (4 / p.KS);
  switch (nj) {
    case 1: return launch_mttkrp_t<T, TC, 1>(g, p, X, cv, part, st);
    case 2: return launch_mttkrp_t<T, TC, 2>(g, p, X, cv, part, st);
    case 3: return launch_mttkrp_t<T, TC, 3>(g, p, X, cv, part, st);
    default: return launch_mttkrp_t<T, TC, 4>(g, p, X, cv, part, st);
  }
}

static hipError_t launch_mttkrp_z(const Geom& g, const MttkrpPlan& p, const float* X,
                                  const CoreView& cv, float* part, hipStream_t st);

hipError_t launch_mttkrp(const Geom& g, const MttkrpPlan& p, const void* X, int xdt,
                         const CoreView& cv, int cdt, void* part, hipStream_t st) {
  if (g.d > 256 || p.nbf > 16) return hipErrorInvalidValue;
  // the kernel's per-outer-index offsets are 32-bit
  const int f = p.f;
  const int64_t xspan = (g.In - 1) * p.sm + (g.I[f] - 1) * p.sf + 1;
  const int64_t gspan = (g.I[f] - 1) * cv.si[f] + (g.R[f] - 1) * cv.sr[f] +
                        (g.R[(f + 1) % g.N] - 1) * cv.ss[f] + 1;
  if (xspan >= ((int64_t)1 << 31) || gspan >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (xdt == F64 && cdt == F64) return launch_mttkrp_j<double, double>(g, p, X, cv, part, st);
  if (xdt == F32 && cdt == F64) return launch_mttkrp_j<float, double>(g, p, X, cv, part, st);
  if (xdt == F32 && cdt == F32) {
    if (p.zform) return launch_mttkrp_z(g, p, (const float*)X, cv, (float*)part, st);
    return launch_mttkrp_j<float, float>(g, p, X, cv, part, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// MTTKRP over many outer indices with every TR-rank <= 16 and I_f <= 64, FP32
// operands and FP32 accumulation over the chunk (the fit-loss gradients).
// For each outer index o the subchain block of all i_f,
//   Z_o[i_f][s][r] = (U(o) G_f(i_f) V(o))[s][r],
// is formed once for the workgroup's 64 rows (per i_f two 16x16x16 MFMA
// products; U^T and V are MFMA chains of the core slices) into LDS, and the
// rows accumulate P[m, r + R_n s] += sum_{i_f} X[m, o, i_f] Z_o[i_f][s][r] in
// MFMA accumulators across the chunk.  Z of the next outer index is formed
// while the current one is used (two LDS buffers, one barrier per outer
// index); the X operands and core slices are loaded one outer index ahead.
// Workgroup: 8 waves over the 16 MT4 rows [16 MT4 y, 16 MT4 (y + 1)) (MT4 =
// 4, 2 or 1 row tiles by I_n: the Z blocks cost the same for any number of
// rows); wave w owns row tile w % MT4 and the 2 MT4 column tiles from
// 2 MT4 (w / MT4), and forms Z for i_f in [8 w, 8 w + 8).  K order of the main product: lane group g of
// k-step q takes i_f = 16 g + q, so the 16 Z operands of a lane in one
// column tile are one contiguous LDS row.
// Layout facts used (16x16x4 FP32 MFMA): the accumulator register v of lane
// (c, g) holds row 4 g + v, column c, which is also the B operand of k-step
// v with k = 4 g + v; the A operand of that k-step at lane (m, g) is then
// A[m][4 g + v], i.e. the accumulator layout of A^T.  So V = F_1 .. F_k is
// built right to left (C <- F_j C) and U^T = F_k^T .. F_1^T likewise.
// ---------------------------------------------------------------------------
constexpr int ZKP = 68;            // LDS pitch (floats) of one Z row (s, r): 64 i_f + 4
constexpr int ZMAXF = 2;          // most slices in U and V together (orders 2 to 4)

// Everything the formed-subchain kernels read besides X, resolved on the
// host: slot j < nU + nV is the j-th chain factor (U's modes n+1 .. f-1, then
// V's modes f+1 .. n-1), slot ZMAXF is G_f, slot ZMAXF + 1 is G_n.  Factor j
// of outer index o is the slice at index (o / div[j]) % mod[j] of its mode;
// the X offset of (i_n = 0, i_f = 0, o) is mlo (o % Lh) + mhi (o / Lh).
struct ZArgs {
  const float* ptr[ZMAXF + 2];
  int si[ZMAXF + 2], sr[ZMAXF + 2], ss[ZMAXF + 2], ra[ZMAXF + 2], rb[ZMAXF + 2];
  unsigned div[ZMAXF], mod[ZMAXF];
  int nU, nV;
  int In, If, Rn, Rn1, d;
  int sm, sf;        // X strides (elements) of the row index and of i_f
  unsigned Lh;
  long long mlo, mhi;
  int upw, Kout;
};

// Slice F (R_a x R_b, zero padded to 16 x 16) of slot j at index i, in one of
// two register patterns of lane (l16, g4):
//   acc pattern: reg v = F[4 g4 + v][l16]   (accumulator layout of F)
//   A pattern:   reg v = F[l16][4 g4 + v]   (A operand of F = acc layout of F^T)
__device__ inline bool slice16_ok(const ZArgs& z, int j, bool acc_pattern, int l16, int g4,
                                  int v) {
  const int a = acc_pattern ? 4 * g4 + v : l16, b = acc_pattern ? l16 : 4 * g4 + v;
  return a < z.ra[j] && b < z.rb[j];
}
// raw: the padding positions hold some in-range element, zeroed by the caller
__device__ inline f4 load_slice16_raw(const ZArgs& z, int j, int i, bool acc_pattern, int l16,
                                      int g4) {
  const float* F = z.ptr[j] + i * z.si[j];
  f4 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = acc_pattern ? 4 * g4 + v : l16, b = acc_pattern ? l16 : 4 * g4 + v;
    r[v] = F[slice16_ok(z, j, acc_pattern, l16, g4, v) ? a * z.sr[j] + b * z.ss[j] : 0];
  }
  return r;
}
__device__ inline f4 load_slice16(const ZArgs& z, int j, int i, bool acc_pattern, int l16,
                                  int g4) {
  f4 r = load_slice16_raw(z, j, i, acc_pattern, l16, g4);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (!slice16_ok(z, j, acc_pattern, l16, g4, v)) r[v] = 0.0f;
  return r;
}

__device__ inline f4 mfma_chain4(f4 a, f4 b) {
  f4 c = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) c = mfma16(a[q], b[q], c);
  return c;
}

// The subchain pieces of one lane: the wave's 8 slices G_f(i_f), kept for
// every outer index (the A pattern when a V follows, else the acc pattern,
// then T = G_f(i_f)); the chain slices of an outer index, loaded raw (U's
// first factor in the A pattern, its others in the acc pattern; V's last
// factor in the acc pattern, its others in the A pattern) with their padding
// zeroed where used; U^T = F_k^T .. F_1^T and V = F_1 .. F_k in the
// accumulator layout, each built right to left; and the 16 x 16 block
// Z(i_f) = U G_f(i_f) V.
template <int NU, int NV>
struct ZLane {
  static constexpr int NF = NU + NV;
  static constexpr int NS = NF > 0 ? NF : 1;
  f4 gf[8];
  unsigned okb;
  int l16, g4;

  __device__ void init(const ZArgs& z, int wave, int lane) {
    l16 = lane & 15;
    g4 = lane >> 4;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i_f = 8 * wave + u;
      gf[u] = load_slice16(z, ZMAXF, i_f < z.If ? i_f : z.If - 1, NV == 0, l16, g4);
      if (i_f >= z.If) gf[u] = f4{0, 0, 0, 0};
    }
    okb = 0;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const bool accp = j < NU ? j > 0 : j == NF - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (slice16_ok(z, j, accp, l16, g4, v)) okb |= 1u << (4 * j + v);
    }
  }
  __device__ void load(const ZArgs& z, int o, f4 (&sl)[NS]) const {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int i = (int)(((unsigned)o / z.div[j]) % z.mod[j]);
      const bool accp = j < NU ? j > 0 : j == NF - 1;
      sl[j] = load_slice16_raw(z, j, i, accp, l16, g4);
    }
  }
  __device__ void chains(const f4 (&raw)[NS], f4& ut, f4& vv) const {
    f4 sl[NS];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sl[j][v] = (okb >> (4 * j + v)) & 1u ? raw[j][v] : 0.0f;
    }
    if constexpr (NU > 0) {
      ut = sl[0];
#pragma unroll
      for (int j = 1; j < NU; ++j) ut = mfma_chain4(sl[j], ut);
    }
    if constexpr (NV > 0) {
      vv = sl[NF - 1];
#pragma unroll
      for (int j = NF - 2; j >= NU; --j) vv = mfma_chain4(sl[j], vv);
    }
  }
  // Z(i_f) for the wave's u-th i_f, accumulator layout: reg v of lane (r, g)
  // = Z[4 g + v][r]
  __device__ f4 block(int u, f4 ut, f4 vv) const {
    f4 t = gf[u];
    if constexpr (NV > 0) t = mfma_chain4(t, vv);
    if constexpr (NU > 0) t = mfma_chain4(ut, t);
    return t;
  }
};

template <int NU, int NV, int MT4>
__global__ __launch_bounds__(512, 1) void k_mttkrp_z(ZArgs z, const float* __restrict__ X,
                                                     float* __restrict__ part) {
  typedef ZLane<NU, NV> ZL;
  constexpr int NT = 2 * MT4;             // column tiles per wave
  extern __shared__ __align__(16) float zl[];            // [2][256][ZKP]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int mt = wave % MT4, tb = (wave / MT4) * NT;
  const int row = blockIdx.y * 16 * MT4 + mt * 16 + l16;
  const int arow = (row < z.In ? row : z.In - 1) * z.sm;
  const int o0 = blockIdx.x * z.upw;
  const int o1 = o0 + z.upw < z.Kout ? o0 + z.upw : z.Kout;
  const int cnt = o1 - o0;
  ZL zc;
  zc.init(z, wave, lane);

  // Z_o of the wave's 8 i_f into LDS buffer b, rows (s, r), i_f contiguous
  auto zform = [&](int b, f4 ut, f4 vv) {
    float* zb = zl + b * (256 * ZKP);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f4 zz[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) zz[u] = zc.block(4 * h + u, ut, vv);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const f4 w = {zz[0][v], zz[1][v], zz[2][v], zz[3][v]};
        *(f4*)(zb + ((4 * g4 + v) * 16 + l16) * ZKP + 8 * wave + 4 * h) = w;
      }
    }
  };
  // X operands of outer index o, unmasked: a row beyond I_n only feeds its
  // own (unwritten) accumulator row, and an i_f beyond I_f meets a zero Z row
  auto load_x = [&](int o, float (&x)[16]) {
    const unsigned ou = (unsigned)o;
    const float* Xo = X + z.mlo * (long long)(ou % z.Lh) + z.mhi * (long long)(ou / z.Lh) + arow;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i_f = 16 * g4 + q;
      x[q] = Xo[(i_f < z.If ? i_f : z.If - 1) * z.sf];
    }
  };

  f4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f4{0, 0, 0, 0};
  f4 slr[ZL::NS];
  f4 ut = {0, 0, 0, 0}, vv = {0, 0, 0, 0};
  float xa[16], xb[16];
  zc.load(z, o0, slr);
  zc.chains(slr, ut, vv);
  zform(0, ut, vv);
  load_x(o0, xa);
  zc.load(z, o0 + 1 < o1 ? o0 + 1 : o1 - 1, slr);
  __syncthreads();
  // one outer index: form Z of the next one (the last step forms an unused
  // copy), load the X operands and chain slices of the next ones, multiply
  // the current X tile by the current Z.  No branches inside, so the loads
  // stay in flight until the next step.
  auto step = [&](int j, const float (&xu)[16], float (&xl)[16]) {
    const int on = o0 + j + 1 < o1 ? o0 + j + 1 : o1 - 1;
    const int on2 = o0 + j + 2 < o1 ? o0 + j + 2 : o1 - 1;
    zc.chains(slr, ut, vv);
    load_x(on, xl);
    zc.load(z, on2, slr);
    zform((j + 1) & 1, ut, vv);
    const float* zb = zl + (j & 1) * (256 * ZKP) + (tb * 16 + l16) * ZKP + 16 * g4;
    // every column tile, valid or not (Z is zero beyond R_{n+1}); the
    // accumulators take turns so consecutive MFMAs are independent
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
      f4 b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = *(const f4*)(zb + t * 16 * ZKP + 4 * qb);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma16(xu[4 * qb + u], b[t][u], acc[t]);
      }
    }
    __syncthreads();
  };
  for (int j = 0; j < cnt; j += 2) {
    step(j, xa, xb);
    if (j + 1 < cnt) step(j + 1, xb, xa);
  }
  // this chunk's partial: acc[t] register v of lane (r, g) = row 4 g + v of
  // the row tile, column r of column tile s = tb + t
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int sc = tb + t;
    if (sc < z.Rn1 && l16 < z.Rn) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = blockIdx.y * 16 * MT4 + mt * 16 + 4 * g4 + v;
        if (m < z.In)
          part[((size_t)blockIdx.x * z.In + m) * z.d + l16 + z.Rn * sc] = acc[t][v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Squared residual of the TR model (fit-loss forward) with the same formed
// subchain blocks, for mode n:
//   Xhat[m, o, i_f] = sum_{s,r} G_n(m)[r][s] Z_o[i_f][s][r],
// a 64 x 64 x 256 MFMA product per outer index against the G_n rows held in
// registers, with Z_o stored i_f-major (one row of 256 (s, r) per i_f) so a
// lane's B operands are contiguous.  Each workgroup writes its sums of
// (X - Xhat)^2 and X^2 (FP64 per lane) as one pair.  Waves as in
// k_mttkrp_z, except that wave w takes the i_f tiles 2 (w / 4) and
// 2 (w / 4) + 1; K order: lane group g of k-step q takes (s, r) = 64 g + q.
// ---------------------------------------------------------------------------
constexpr int ZTP = 260;           // LDS pitch (floats) of one Z row i_f: 256 (s, r) + 4

template <int NU, int NV>
__global__ __launch_bounds__(512, 1) void k_recon_z(ZArgs z, const float* __restrict__ X,
                                                    double* __restrict__ wg_out) {
  typedef ZLane<NU, NV> ZL;
  extern __shared__ __align__(16) float zt[];            // [2][64][ZTP]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int mt = wave & 3, sh = wave >> 2;
  const int o0 = blockIdx.x * z.upw;
  const int o1 = o0 + z.upw < z.Kout ? o0 + z.upw : z.Kout;
  const int cnt = o1 - o0;
  ZL zc;
  zc.init(z, wave, lane);
  // A operands: G_n(m)[r][s] for (s, r) = 64 g4 + q, zero outside the ranks
  float ga[64];
  {
    const int m = blockIdx.y * 64 + mt * 16 + l16;
    const int j = ZMAXF + 1;
    const float* Gn = z.ptr[j] + (m < z.In ? m : z.In - 1) * z.si[j];
#pragma unroll
    for (int q = 0; q < 64; ++q) {
      const int sc = 4 * g4 + (q >> 4), r = q & 15;
      const bool ok = m < z.In && r < z.Rn && sc < z.Rn1;
      const float v = Gn[ok ? r * z.sr[j] + sc * z.ss[j] : 0];
      ga[q] = ok ? v : 0.0f;
    }
  }
  // Z_o of the wave's 8 i_f into LDS buffer b, one row of (s, r) per i_f
  auto zform = [&](int b, f4 ut, f4 vv) {
    float* zb = zt + b * (64 * ZTP);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const f4 w = zc.block(u, ut, vv);
#pragma unroll
      for (int v = 0; v < 4; ++v) zb[(8 * wave + u) * ZTP + (4 * g4 + v) * 16 + l16] = w[v];
    }
  };
  // X at the accumulator positions of the wave's two i_f tiles: reg v of
  // lane (c, g) is row 16 mt + 4 g + v, i_f = 16 (2 sh + h) + c
  const int mrow0 = blockIdx.y * 64 + mt * 16 + 4 * g4;
  auto load_x = [&](int o, float (&x)[8]) {
    const unsigned ou = (unsigned)o;
    const float* Xo = X + z.mlo * (long long)(ou % z.Lh) + z.mhi * (long long)(ou / z.Lh);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i_f = 16 * (2 * sh + h) + l16;
      const int ic = i_f < z.If ? i_f : z.If - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mrow0 + v < z.In ? mrow0 + v : z.In - 1;
        x[4 * h + v] = Xo[m * z.sm + ic * z.sf];
      }
    }
  };
  double err = 0.0, nrm = 0.0;
  f4 slr[ZL::NS];
  f4 ut = {0, 0, 0, 0}, vv = {0, 0, 0, 0};
  float xa[8], xb[8];
  zc.load(z, o0, slr);
  zc.chains(slr, ut, vv);
  zform(0, ut, vv);
  load_x(o0, xa);
  zc.load(z, o0 + 1 < o1 ? o0 + 1 : o1 - 1, slr);
  __syncthreads();
  auto step = [&](int j, const float (&xu)[8], float (&xl)[8]) {
    const int on = o0 + j + 1 < o1 ? o0 + j + 1 : o1 - 1;
    const int on2 = o0 + j + 2 < o1 ? o0 + j + 2 : o1 - 1;
    zc.chains(slr, ut, vv);
    load_x(on, xl);
    zc.load(z, on2, slr);
    zform((j + 1) & 1, ut, vv);
    const float* zb = zt + (j & 1) * (64 * ZTP) + (32 * sh + l16) * ZTP + 64 * g4;
    // two i_f tiles x two halves of K: four independent accumulators
    f4 acc[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[h][0] = acc[h][1] = f4{0, 0, 0, 0};
#pragma unroll
    for (int qb = 0; qb < 8; ++qb) {
      f4 b[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        b[h][0] = *(const f4*)(zb + h * 16 * ZTP + 4 * qb);
        b[h][1] = *(const f4*)(zb + h * 16 * ZTP + 32 + 4 * qb);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[h][0] = mfma16(ga[4 * qb + u], b[h][0][u], acc[h][0]);
          acc[h][1] = mfma16(ga[32 + 4 * qb + u], b[h][1][u], acc[h][1]);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i_f = 16 * (2 * sh + h) + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (i_f < z.If && mrow0 + v < z.In) {
          const double x = (double)xu[4 * h + v];
          const double e = x - (double)(acc[h][0][v] + acc[h][1][v]);
          err += e * e;
          nrm += x * x;
        }
      }
    }
    __syncthreads();
  };
  for (int j = 0; j < cnt; j += 2) {
    step(j, xa, xb);
    if (j + 1 < cnt) step(j + 1, xb, xa);
  }
  // workgroup sums in a fixed order: wave shuffles, then the 8 wave sums
  for (int off = 32; off > 0; off >>= 1) {
    err += __shfl_xor(err, off);
    nrm += __shfl_xor(nrm, off);
  }
  double* red = (double*)zt;
  if (lane == 0) {
    red[wave] = err;
    red[8 + wave] = nrm;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 8; ++w) {
      a += red[w];
      b += red[8 + w];
    }
    const int blk = blockIdx.x + gridDim.x * blockIdx.y;
    wg_out[2 * blk] = a;
    wg_out[2 * blk + 1] = b;
  }
}

// The chain, fast-mode and row cores and the outer-index decoding of a
// formed-subchain plan (false if an offset would leave 32 bits).
static bool make_zargs(const Geom& g, const MttkrpPlan& p, const CoreView& cv, ZArgs* zp) {
  const int N = g.N, n = g.n, f = p.f;
  ZArgs& z = *zp;
  z = ZArgs{};
  z.nU = (f - (n + 1) + N) % N;
  z.nV = (n - (f + 1) + N) % N;
  if (z.nU + z.nV > ZMAXF) return false;
  // index divisor of mode q in the enumeration of the outer indices (the
  // multi-index of the modes other than n and f, fastest first)
  auto divisor = [&](int q) -> int64_t {
    int64_t dv = 1;
    for (int p2 = 0; p2 < q; ++p2)
      if (p2 != n && p2 != f) dv *= g.I[p2];
    return dv;
  };
  bool ok = true;
  auto set_slot = [&](int j, int k) {
    z.ptr[j] = (const float*)cv.ptr[k];
    z.si[j] = (int)cv.si[k];
    z.sr[j] = (int)cv.sr[k];
    z.ss[j] = (int)cv.ss[k];
    z.ra[j] = g.R[k];
    z.rb[j] = g.R[(k + 1) % N];
    const int64_t span = (g.I[k] - 1) * cv.si[k] + (g.R[k] - 1) * cv.sr[k] +
                         (g.R[(k + 1) % N] - 1) * cv.ss[k] + 1;
    ok = ok && span < ((int64_t)1 << 31);
  };
  for (int j = 0; j < z.nU + z.nV; ++j) {
    const int k = j < z.nU ? (n + 1 + j) % N : (f + 1 + (j - z.nU)) % N;
    set_slot(j, k);
    z.div[j] = (unsigned)divisor(k);
    z.mod[j] = (unsigned)g.I[k];
  }
  set_slot(ZMAXF, f);
  set_slot(ZMAXF + 1, n);
  z.In = (int)g.In;
  z.If = (int)g.I[f];
  z.Rn = g.R[n];
  z.Rn1 = g.R[(n + 1) % N];
  z.d = g.d;
  z.sm = (int)p.sm;
  z.sf = (int)p.sf;
  if (n == 0) {
    z.Lh = 1u;
    z.mlo = 0;
    z.mhi = g.I[0] * g.I[1];
  } else {
    z.Lh = (unsigned)(g.L / g.I[0]);
    z.mlo = g.I[0];
    z.mhi = g.L * g.In;
  }
  z.upw = (int)p.upw;
  z.Kout = (int)p.Kout;
  // 32-bit index arithmetic inside the kernels
  if (p.Kout >= ((int64_t)1 << 31) || (g.In - 1) * p.sm + (g.I[f] - 1) * p.sf >= ((int64_t)1 << 31))
    ok = false;
  return ok;
}

template <template <int, int> class K, typename... A>
static hipError_t launch_z(const ZArgs& z, dim3 grid, size_t lds, hipStream_t st, A... args) {
  void (*fn)(ZArgs, A...) = nullptr;
  switch (z.nU * 3 + z.nV) {
    case 0: fn = K<0, 0>::fn; break;
    case 1: fn = K<0, 1>::fn; break;
    case 2: fn = K<0, 2>::fn; break;
    case 3: fn = K<1, 0>::fn; break;
    case 4: fn = K<1, 1>::fn; break;
    case 6: fn = K<2, 0>::fn; break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e =
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, dim3(512), lds, st, z, args...);
  return hipGetLastError();
}
template <int MT4> struct MttkrpZT {
  template <int NU, int NV> struct K {
    static constexpr auto fn = k_mttkrp_z<NU, NV, MT4>;
  };
};
template <int NU, int NV> struct ReconZ {
  static constexpr auto fn = k_recon_z<NU, NV>;
};

hipError_t launch_recon_z(const Geom& g, const float* X, const CoreView& cv, double* wg_out,
                          int max_wg, int* nwg, hipStream_t st) {
  *nwg = 0;
  const MttkrpPlan p = plan_mttkrp(g, F32, 0, true);
  ZArgs z;
  const int64_t mg = (g.In + 63) / 64;
  if (!p.zform || p.MT != 64 || (int64_t)p.nsplit * mg > max_wg || !make_zargs(g, p, cv, &z))
    return hipErrorNotSupported;
  const dim3 grid(p.nsplit, (unsigned)mg);
  *nwg = (int)(p.nsplit * mg);
  return launch_z<ReconZ>(z, grid, (size_t)2 * 64 * ZTP * sizeof(float), st, X, wg_out);
}

static hipError_t launch_mttkrp_z(const Geom& g, const MttkrpPlan& p, const float* X,
                                  const CoreView& cv, float* part, hipStream_t st) {
  ZArgs z;
  if (!make_zargs(g, p, cv, &z)) return hipErrorInvalidValue;
  const dim3 grid(p.nsplit, (unsigned)((g.In + p.MT - 1) / p.MT));
  const size_t lds = (size_t)2 * 256 * ZKP * sizeof(float);
  switch (p.MT) {
    case 16: return launch_z<MttkrpZT<1>::K>(z, grid, lds, st, X, part);
    case 32: return launch_z<MttkrpZT<2>::K>(z, grid, lds, st, X, part);
    case 64: return launch_z<MttkrpZT<4>::K>(z, grid, lds, st, X, part);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Split reduction (fixed order), P accumulation and the right-multiply by
// Q_n^{-1}: G_{n(2)} = P_n Q_n^dagger (Alg. 4).  One row per workgroup (the
// work is latency-bound: a few loads per thread, all in flight at once).
// Wave q sums the splits q, q+4, q+8, ... of every column (a wave reads 64
// consecutive columns of one split), the four wave sums are added in a fixed
// order; the product with Q_n^{-1} splits the inner index over the waves the
// same way.
// ---------------------------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void k_reduce_solve(const PT* __restrict__ part, int nsplit,
                                                      int64_t In, int d, double* P,
                                                      int accumulate,
                                                      const double* __restrict__ Minv,
                                                      double* __restrict__ out,
                                                      float* __restrict__ out32) {
  extern __shared__ double sh[];                        // [4][d] wave sums, [d] row
  double* red = sh;
  double* prow = sh + 4 * d;
  const int q = threadIdx.x >> 6, c0 = threadIdx.x & 63;
  const int64_t row = blockIdx.x;
  const size_t stride = (size_t)In * d;
  const PT* __restrict__ src = part + (size_t)row * d;
  // without the solve the row's columns are split over blockIdx.y in blocks
  // of 64 (the solve needs the whole row in one workgroup)
  const int cbeg = Minv ? 0 : blockIdx.y * 64, cend = Minv ? d : min(d, cbeg + 64);
  for (int c = cbeg + c0; c < cend; c += 64) {
    double sum = 0.0;
    int sp = q;
    for (; sp + 28 < nsplit; sp += 32) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = (double)src[(size_t)(sp + 4 * u) * stride + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += x[u];
    }
    for (; sp < nsplit; sp += 4) sum += (double)src[(size_t)sp * stride + c];
    red[q * d + c] = sum;
  }
  __syncthreads();
  for (int c = cbeg + threadIdx.x; c < cend; c += 256) {
    double sum = ((red[c] + red[d + c]) + red[2 * d + c]) + red[3 * d + c];
    if (P) {
      const size_t pi = (size_t)row * d + c;
      if (accumulate) sum += P[pi];
      P[pi] = sum;
    }
    prow[c] = sum;
  }
  if (!Minv) return;
  __syncthreads();
  const int cq = (d + 3) >> 2, cb = q * cq, ce = min(d, cb + cq);
  for (int c2 = c0; c2 < d; c2 += 64) {
    double g0 = 0.0, g1 = 0.0;
    int c = cb;
#pragma unroll 4
    for (; c + 1 < ce; c += 2) {
      g0 += prow[c] * Minv[(size_t)c * d + c2];
      g1 += prow[c + 1] * Minv[(size_t)(c + 1) * d + c2];
    }
    if (c < ce) g0 += prow[c] * Minv[(size_t)c * d + c2];
    red[q * d + c2] = g0 + g1;
  }
  __syncthreads();
  for (int c2 = threadIdx.x; c2 < d; c2 += 256) {
    const double g = ((red[c2] + red[d + c2]) + red[2 * d + c2]) + red[3 * d + c2];
    out[(size_t)row * d + c2] = g;
    if (out32) out32[(size_t)row * d + c2] = (float)g;
  }
}

hipError_t launch_reduce_solve(const void* part, int psize, int nsplit, int64_t In, int d,
                               double* P, int accumulate, const double* Minv, double* out,
                               hipStream_t st, float* out32) {
  if (In <= 0) return hipSuccess;
  if (In > 0x7fffffff || d <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)In, Minv ? 1u : (unsigned)((d + 63) / 64));
  const size_t lds = (size_t)5 * d * sizeof(double);
  if (lds > 65536) return hipErrorInvalidValue;
  if (psize == 8)
    hipLaunchKernelGGL(k_reduce_solve<double>, grid, dim3(256), lds, st, (const double*)part,
                       nsplit, In, d, P, accumulate, Minv, out, out32);
  else
    hipLaunchKernelGGL(k_reduce_solve<float>, grid, dim3(256), lds, st, (const float*)part,
                       nsplit, In, d, P, accumulate, Minv, out, out32);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram matrices of core slices in the "transfer" layout:
//   E[(a + Ra*a'), (b + Rb*b')] = sum_i G(i)[a,b] G(i)[a',b'].
// E_k holds the same numbers as the paper's Gram tensor Z_k (Alg. 2),
// Z_k[b, a, b', a'] = E_k[(a, a'), (b, b')]; products of E's in ring order
// give the Gram chain of Prop. subchain Gram.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_E(const double* __restrict__ G, int64_t rows,
                                                int Ra, int Rb, double* __restrict__ E) {
  // Gram[c1][c2] = sum_i G_(2)[i][c1] G_(2)[i][c2] on one 16x16 tile, rows
  // staged 64 at a time; c = a + Ra*b, written to the transfer layout.
  __shared__ double A1[64][17], A2[64][17];
  const int dd = Ra * Rb;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int c1 = blockIdx.y * 16 + ty, c2 = blockIdx.x * 16 + tx;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i0 = 0; i0 < rows; i0 += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e >> 4, c = e & 15;
      const int64_t i = i0 + r;
      const int ca = blockIdx.y * 16 + c, cb = blockIdx.x * 16 + c;
      A1[r][c] = (i < rows && ca < dd) ? G[i * dd + ca] : 0.0;
      A2[r][c] = (i < rows && cb < dd) ? G[i * dd + cb] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 64; r += 2) {
      s0 += A1[r][ty] * A2[r][tx];
      s1 += A1[r + 1][ty] * A2[r + 1][tx];
    }
    __syncthreads();
  }
  if (c1 < dd && c2 < dd) {
    const int a1 = c1 % Ra, b1 = c1 / Ra, a2 = c2 % Ra, b2 = c2 / Ra;
    E[(size_t)(a1 + Ra * a2) * (Rb * Rb) + (b1 + Rb * b2)] = s0 + s1;
  }
}

hipError_t launch_gram_E(const double* G, int64_t rows, int Ra, int Rb, double* E,
                         hipStream_t st) {
  const int dd = Ra * Rb, tiles = (dd + 15) / 16;
  hipLaunchKernelGGL(k_gram_E, dim3(tiles, tiles), dim3(256), 0, st, G, rows, Ra, Rb, E);
  return hipGetLastError();
}

// C = A * B (row-major FP64) on FP64 MFMAs: one 16x16 output tile per
// workgroup; wave w takes the w-th quarter of K (lane group g the k = 4j + g
// of it), with its loads issued 8 k-steps at a time into two alternating
// accumulators; the four wave sums are added in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_matmul(const double* __restrict__ A,
                                                const double* __restrict__ B,
                                                double* __restrict__ C, int d1, int d2, int d3) {
  __shared__ double red[3][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  const int kw = ((d2 + 15) / 16) * 4;      // k per wave, a multiple of 4
  const int kb = wave * kw;
  const int arow = r0 + l16 < d1 ? r0 + l16 : d1 - 1;
  const int bcol = c0 + l16 < d3 ? c0 + l16 : d3 - 1;
  const bool rok = r0 + l16 < d1, cok = c0 + l16 < d3;
  d4 acc[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
  for (int j0 = 0; j0 < kw / 4; j0 += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + 4 * (j0 + u) + g4;
      const bool ok = j0 + u < kw / 4 && k < d2;
      const int kc = k < d2 ? k : d2 - 1;
      const double a = A[(size_t)arow * d2 + kc], b = B[(size_t)kc * d3 + bcol];
      av[u] = ok && rok ? a : 0.0;
      bv[u] = ok && cok ? b : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u & 1] = mfma16(av[u], bv[u], acc[u & 1]);
  }
  d4 s = acc[0] + acc[1];
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave - 1][v * 64 + lane] = s[v];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double t = ((s[v] + red[0][v * 64 + lane]) + red[1][v * 64 + lane]) +
                       red[2][v * 64 + lane];
      const int row = r0 + Acc<double>::row(lane, v), col = c0 + l16;
      if (row < d1 && col < d3) C[(size_t)row * d3 + col] = t;
    }
  }
}

// Transfer layout of a Gram tensor given in the paper's layout: Z of size
// R' x R x R' x R (R = R_k, R' = R_{k+1}, column-major, the Gram tensor
// Z[b, a, b2, a2] = sum_i G(i)[a, b] G(i)[a2, b2] of Alg. 2) to
// E[(a + R a2), (b + R' b2)] (row-major), one thread per element.
__global__ void k_z_to_E(const double* __restrict__ Z, int R, int R1, double* __restrict__ E) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int n = R * R * R1 * R1;
  if (e >= n) return;
  const int row = e / (R1 * R1), col = e - row * (R1 * R1);
  const int a = row % R, a2 = row / R, b = col % R1, b2 = col / R1;
  E[e] = Z[b + R1 * (a + R * (b2 + R1 * a2))];
}

hipError_t launch_z_to_E(const double* Z, int R, int R1, double* E, hipStream_t st) {
  const int n = R * R * R1 * R1;
  hipLaunchKernelGGL(k_z_to_E, dim3((n + 255) / 256), dim3(256), 0, st, Z, R, R1, E);
  return hipGetLastError();
}

hipError_t launch_matmul(const double* A, const double* B, double* C, int d1, int d2, int d3,
                         hipStream_t st) {
  dim3 grid((d3 + 15) / 16, (d1 + 15) / 16);
  hipLaunchKernelGGL(k_matmul, grid, dim3(256), 0, st, A, B, C, d1, d2, d3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pseudo-inverse fallback of the normal-equation solves (the dagger in
// G_{n(2)} = P_n Q_n^dagger of Alg. 4, and in Algs. 7-9).  The eliminations
// below invert Q assuming it is positive definite; when one of their pivots
// fails the positivity test the whole workgroup comes here instead and
// replaces the result by the pseudo-inverse of the symmetric d x d matrix H.
//
// One-sided Jacobi (Hestenes): rotate pairs of columns of W (= H at the
// start), accumulating the rotations in V, until every pair is orthogonal
// to working precision.  Then H V = W, the column norms sigma_j = ||w_j||
// are the singular values of H, and
//   H^dagger = sum over sigma_j > tol of v_j w_j^T / sigma_j^2,
//   tol = d * eps * max_j sigma_j
// (singular values at or below tol are taken as zero, the cut-off of an
// SVD pseudo-inverse).  The pairs of one round of a round-robin schedule
// are disjoint, so groups of 16 lanes rotate them in parallel between
// workgroup barriers.  W, V and the norms live in `work` (2 d^2 + d
// doubles of global scratch).  status[2] counts the fallbacks, status[3] is
// set for the solve that took one (the leverage scores read it), status[0]
// is set to 2 if H holds NaN or Inf.  Called by every thread of the
// workgroup (nthr threads), or by one whole wave (nthr = 64).
// ---------------------------------------------------------------------------
__device__ inline void fb_sync(int nthr) {
  if (nthr > 64) {
    __syncthreads();
  } else {
    // one wave: its own global stores complete before its next loads
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ inline bool fb_any(int x, int nthr) {
  if (nthr > 64) return __syncthreads_or(x) != 0;
  fb_sync(nthr);
  return __ballot(x) != 0;
}

__device__ __forceinline__ void pinv_fallback(const double* H, int d, double* Hinv, double* work,
                                           int* status, int tid, int nthr) {
  double* W = work;                       // column j at W + j d
  double* V = work + (size_t)d * d;
  double* sg = V + (size_t)d * d;
  for (int e = tid; e < d * d; e += nthr) {
    const int j = e / d, i = e - j * d;
    W[e] = H[e];                          // H is symmetric: column j = row j
    V[e] = i == j ? 1.0 : 0.0;
  }
  fb_sync(nthr);
  const int grp = tid >> 4, ngrp = nthr >> 4, l = tid & 15;
  const int D = d + (d & 1);              // an even count of columns: index d sits out
  for (int sweep = 0; sweep < 48; ++sweep) {
    int rot = 0;
    for (int r = 0; r < D - 1; ++r) {
      for (int k = grp; k < D / 2; k += ngrp) {
        const int p = k == 0 ? r : (r + k) % (D - 1);
        const int q = k == 0 ? D - 1 : (r + D - 1 - k) % (D - 1);
        if (p >= d || q >= d) continue;   // the same for the 16 lanes of a group
        double* wp = W + (size_t)p * d;
        double* wq = W + (size_t)q * d;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = l; i < d; i += 16) {
          const double x = wp[i], y = wq[i];
          a = fma(x, x, a);
          b = fma(y, y, b);
          c = fma(x, y, c);
        }
        for (int off = 8; off > 0; off >>= 1) {
          a += __shfl_xor(a, off, 16);
          b += __shfl_xor(b, off, 16);
          c += __shfl_xor(c, off, 16);
        }
        if (c != 0.0 && fabs(c) > 1e-15 * sqrt(a * b)) {
          // tan of the angle that makes the pair orthogonal (the smaller root
          // of t^2 + 2 z t - 1 = 0, z = (b - a) / 2c)
          const double z = (b - a) / (2.0 * c);
          const double t = fabs(z) > 1e150 ? 0.5 / z
                                           : (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          double* vp = V + (size_t)p * d;
          double* vq = V + (size_t)q * d;
          for (int i = l; i < d; i += 16) {
            const double x = wp[i], y = wq[i];
            wp[i] = cs * x - sn * y;
            wq[i] = sn * x + cs * y;
            const double u = vp[i], v = vq[i];
            vp[i] = cs * u - sn * v;
            vq[i] = sn * u + cs * v;
          }
          rot = 1;
        }
      }
      fb_sync(nthr);
    }
    if (!fb_any(rot, nthr)) break;
  }
  for (int j = grp; j < d; j += ngrp) {
    double a = 0.0;
    for (int i = l; i < d; i += 16) a = fma(W[(size_t)j * d + i], W[(size_t)j * d + i], a);
    for (int off = 8; off > 0; off >>= 1) a += __shfl_xor(a, off, 16);
    if (l == 0) sg[j] = sqrt(a);
  }
  fb_sync(nthr);
  double smax = 0.0;
  bool finite = true;
  for (int j = 0; j < d; ++j) {
    const double x = sg[j];
    finite = finite && isfinite(x);
    smax = fmax(smax, x);
  }
  const double tol = (double)d * 2.220446049250313e-16 * smax;
  fb_sync(nthr);
  for (int j = tid; j < d; j += nthr) {
    const double x = sg[j];
    sg[j] = x > tol ? 1.0 / (x * x) : 0.0;
  }
  fb_sync(nthr);
  // upper triangle, mirrored: the result is exactly symmetric
  for (int e = tid; e < d * d; e += nthr) {
    const int i = e / d, k = e - i * d;
    if (k < i) continue;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) acc = fma(V[(size_t)j * d + i] * sg[j], W[(size_t)j * d + k], acc);
    Hinv[(size_t)i * d + k] = acc;
    Hinv[(size_t)k * d + i] = acc;
  }
  if (tid == 0 && status) {
    if (!finite) status[0] = 2;
    atomicAdd(status + 2, 1);
    status[3] = 1;
  }
}

// End of an elimination, once `any` (some pivot test of the workgroup
// failed) is known: the pseudo-inverse fallback from the stored matrix H
// (the Q the elimination started from), or, without a stored matrix or
// scratch, the failure flagged in status[0] (value 1).  Called by the
// nthr threads the fallback is to use (the workgroup, or one wave).
__device__ inline void finish_inverse(bool any, const double* H, int d, double* Hinv,
                                      double* work, int* status, int tid, int nthr) {
  if (any && H && work) {
    pinv_fallback(H, d, Hinv, work, status, tid, nthr);
    return;
  }
  if (tid == 0 && status) {
    if (any) status[0] = 1;
    status[3] = 0;
  }
}

// ---------------------------------------------------------------------------
// Q-layout assembly and in-place Gauss-Jordan inverse (no pivoting: the
// normal-equation matrices are symmetric positive definite).  A TG x TG grid
// of threads keeps the d x d matrix in registers, thread (ty, tx) owning the
// B x B block at rows ty*B.., columns tx*B...  Pivot k: the owners publish
// row k and column k to LDS (alternating buffers: one barrier per pivot);
// every element takes a -= f_i r_j with f, r zeroed on the pivot row /
// column, then the pivot row becomes a_kj / p, the pivot column -a_ik / p
// and the pivot 1 / p.  M is Rb^2 x Ra^2 (row-major) and
//   Q[r + Ra*s, r' + Ra*s'] = M[s + Rb*s', r + Ra*r']
// unless m_plain says M is already d x d in the Q layout.
// ---------------------------------------------------------------------------
template <int TG, int B>
__global__ __launch_bounds__(TG* TG) void k_invert_spd(const double* __restrict__ M, int Ra,
                                                       int Rb, double* Q, int accumulate,
                                                       int store_Q, double* __restrict__ Qinv,
                                                       int* status, int m_plain, double* work) {
  __shared__ double rowk[2][TG * B], colk[2][TG * B];
  __shared__ double sh_tol;
  const int tid = threadIdx.x;
  const int ty = tid / TG, tx = tid - (tid / TG) * TG;
  const int d = Ra * Rb;
  double a[B][B];
#pragma unroll
  for (int i = 0; i < B; ++i) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int gi = ty * B + i, gj = tx * B + j;
      double v = 0.0;
      if (gi < d && gj < d) {
        const int e = gi * d + gj;
        if (M && m_plain) {
          v = M[e];
        } else if (M) {
          const int r = gi % Ra, s1 = gi / Ra, r2 = gj % Ra, s2 = gj / Ra;
          v = M[(size_t)(s1 + Rb * s2) * (Ra * Ra) + (r + Ra * r2)];
        }
        if (Q && accumulate) v += Q[e];
        if (Q && store_Q) Q[e] = v;
      }
      a[i][j] = v;
    }
  }
  if (!Qinv) return;
  // tolerance d * eps * max diagonal
  if (ty == tx) {
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (ty * B + i < d) colk[1][ty * B + i] = a[i][i];
  }
  __syncthreads();
  if (tid < 64) {
    double mx = 0.0;
    for (int i = tid; i < d; i += 64) mx = fmax(mx, colk[1][i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (tid == 0) sh_tol = (double)d * 2.220446049250313e-16 * mx;
  }
  __syncthreads();
  const double tol = sh_tol;
  bool bad = false;
  for (int k = 0; k < d; ++k) {
    const int bs = k & 1;
    const int kb = k / B, kr = k - (k / B) * B;
    if (ty == kb) {
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i == kr) {
#pragma unroll
          for (int j = 0; j < B; ++j) rowk[bs][tx * B + j] = a[i][j];
        }
    }
    if (tx == kb) {
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j == kr) {
#pragma unroll
          for (int i = 0; i < B; ++i) colk[bs][ty * B + i] = a[i][j];
        }
    }
    __syncthreads();
    const double pv = colk[bs][k];
    if (!(pv > tol)) bad = true;
    const double ip = 1.0 / pv;
    // unconditional LDS loads (clamped index), then selects
    double cf[B], fr[B], rr[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int gi = ty * B + i;
      cf[i] = colk[bs][gi < d ? gi : d - 1];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int gj = tx * B + j;
      rr[j] = rowk[bs][gj < d ? gj : d - 1];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) fr[i] = (ty * B + i == k) ? 0.0 : cf[i];
#pragma unroll
    for (int j = 0; j < B; ++j) rr[j] = (tx * B + j == k) ? 0.0 : rr[j] * ip;
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
      for (int j = 0; j < B; ++j) a[i][j] -= fr[i] * rr[j];
    }
    if (ty == kb) {
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i == kr) {
#pragma unroll
          for (int j = 0; j < B; ++j) a[i][j] = (tx * B + j == k) ? ip : a[i][j] * ip;
        }
    }
    if (tx == kb) {
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j == kr) {
#pragma unroll
          for (int i = 0; i < B; ++i) a[i][j] = (ty * B + i != k) ? -cf[i] * ip : a[i][j];
        }
    }
  }
  const bool any = __syncthreads_or(bad) != 0;
  if (!any) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int gi = ty * B + i, gj = tx * B + j;
        if (gi < d && gj < d) Qinv[gi * d + gj] = a[i][j];
      }
    }
  }
  finish_inverse(any, Q && store_Q ? Q : nullptr, d, Qinv, work, status, tid, TG * TG);
}

// Q-layout assembly alone (no inverse), one thread per element:
//   Q[r + Ra s, r' + Ra s'] (+)= M[s + Rb s', r + Ra r']
// with M the Rb^2 x Ra^2 Gram-chain product (row-major).
__global__ __launch_bounds__(256) void k_assemble_q(const double* __restrict__ M, int Ra, int Rb,
                                                    double* __restrict__ Q, int accumulate) {
  const int d = Ra * Rb;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d * d) return;
  const int gi = e / d, gj = e - gi * d;
  const int r = gi % Ra, s1 = gi / Ra, r2 = gj % Ra, s2 = gj / Ra;
  double v = M[(size_t)(s1 + Rb * s2) * (Ra * Ra) + (r + Ra * r2)];
  if (accumulate) v += Q[e];
  Q[e] = v;
}

hipError_t launch_assemble_q(const double* M, int Ra, int Rb, double* Q, int accumulate,
                             hipStream_t st) {
  const int d = Ra * Rb;
  if (d <= 0 || d > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_assemble_q, dim3((d * d + 255) / 256), dim3(256), 0, st, M, Ra, Rb, Q,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_invert_spd(const double* M, int Ra, int Rb, double* Q, int accumulate,
                             int store_Q, double* Qinv, int* status, hipStream_t st,
                             int m_plain, double* work) {
  const int d = Ra * Rb;
  if (d > 256) return hipErrorInvalidValue;
#define TRK_INV(TG, B)                                                                    \
  hipLaunchKernelGGL((k_invert_spd<TG, B>), dim3(1), dim3(TG * TG), 0, st, M, Ra, Rb, Q, \
                     accumulate, store_Q, Qinv, status, m_plain, work)
  const int B16 = (d + 15) / 16;
  switch (B16) {
    case 1: TRK_INV(16, 1); break;
    case 2: TRK_INV(16, 2); break;
    case 3: TRK_INV(16, 3); break;
    case 4: TRK_INV(16, 4); break;
    case 5: TRK_INV(16, 5); break;
    case 6: TRK_INV(16, 6); break;
    case 7: TRK_INV(16, 7); break;
    case 8: TRK_INV(16, 8); break;
    case 9: TRK_INV(16, 9); break;
    case 10: TRK_INV(16, 10); break;
    default: TRK_INV(32, 8); break;
  }
#undef TRK_INV
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused side step of one mode (Alg. 4): Gram refresh of the core updated by
// the previous mode, Gram-chain product (Prop. subchain Gram), Q assembly
// and Gauss-Jordan inverse, in one workgroup of 1024 threads (16 waves).
// The Gram and the chain products use 16x16x4 FP64 MFMAs with operands
// read through the cache; stages are separated by workgroup barriers.
// ---------------------------------------------------------------------------
__device__ inline void side_matmul(const double* __restrict__ A, const double* __restrict__ Bm,
                                   double* __restrict__ C, int d1, int d2, int d3, int wave,
                                   int lane) {
  const int nb1 = (d1 + 15) >> 4, nb3 = (d3 + 15) >> 4;
  const int ar = lane & 15, ak = lane >> 4;
  for (int b = wave; b < nb1 * nb3; b += 16) {
    const int rb = b / nb3, cb = b - rb * nb3;
    d4 acc = {0, 0, 0, 0};
    const int arow = rb * 16 + ar, bcol = cb * 16 + ar;
    for (int k0 = 0; k0 < d2; k0 += 4) {
      const int k = k0 + ak;
      const double av = (arow < d1 && k < d2) ? A[(size_t)arow * d2 + k] : 0.0;
      const double bv = (k < d2 && bcol < d3) ? Bm[(size_t)k * d3 + bcol] : 0.0;
      acc = mfma16(av, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rb * 16 + Acc<double>::row(lane, v), c = cb * 16 + (lane & 15);
      if (r < d1 && c < d3) C[(size_t)r * d3 + c] = acc[v];
    }
  }
}

template <int B>
__global__ __launch_bounds__(1024) void k_side(SideArgs sa) {
  constexpr int TG = 32;
  __shared__ double rowk[2][TG * B], colk[2][TG * B];
  __shared__ double sh_tol;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  // 1. Gram of the previous core, written in the transfer layout
  if (sa.Gp) {
    const int Ra = sa.Rpa, Rb = sa.Rpb, dp = Ra * Rb;
    const int nb = (dp + 15) >> 4;
    const int ar = lane & 15, ak = lane >> 4;
    for (int b = wave; b < nb * nb; b += 16) {
      const int rb = b / nb, cb = b - rb * nb;
      const int c1 = rb * 16 + ar, c2 = cb * 16 + ar;
      d4 acc = {0, 0, 0, 0};
      for (int64_t k0 = 0; k0 < sa.rows_p; k0 += 4) {
        const int64_t i = k0 + ak;
        const double av = (i < sa.rows_p && c1 < dp) ? sa.Gp[i * dp + c1] : 0.0;
        const double bv = (i < sa.rows_p && c2 < dp) ? sa.Gp[i * dp + c2] : 0.0;
        acc = mfma16(av, bv, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb * 16 + Acc<double>::row(lane, v), c = cb * 16 + (lane & 15);
        if (r < dp && c < dp) {
          const int a1 = r % Ra, b1 = r / Ra, a2 = c % Ra, b2 = c / Ra;
          sa.Ep[(size_t)(a1 + Ra * a2) * (Rb * Rb) + (b1 + Rb * b2)] = acc[v];
        }
      }
    }
    __syncthreads();
  }
  // 2. ring product of the transfer-layout factors
  const double* M = sa.fac[0] ? sa.fac[0] : sa.Ep;
  for (int j = 1; j < sa.nfac; ++j) {
    const double* F = sa.fac[j] ? sa.fac[j] : sa.Ep;
    double* out = sa.cbuf[(j - 1) & 1];
    side_matmul(M, F, out, sa.fr[0], sa.fc[j - 1], sa.fc[j], wave, lane);
    __syncthreads();
    M = out;
  }
  // 3. Q assembly and Gauss-Jordan inverse (32 x 32 thread grid, B x B blocks)
  const int Ra = sa.Ra, Rb = sa.Rb, d = Ra * Rb;
  const int ty = tid / TG, tx = tid - (tid / TG) * TG;
  double a[B][B];
#pragma unroll
  for (int i = 0; i < B; ++i) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int gi = ty * B + i, gj = tx * B + j;
      double v = 0.0;
      if (gi < d && gj < d) {
        const int e = gi * d + gj;
        const int r = gi % Ra, s1 = gi / Ra, r2 = gj % Ra, s2 = gj / Ra;
        v = M[(size_t)(s1 + Rb * s2) * (Ra * Ra) + (r + Ra * r2)];
        if (sa.Q && sa.accumulate) v += sa.Q[e];
        if (sa.Q && sa.store_Q) sa.Q[e] = v;
      }
      a[i][j] = v;
    }
  }
  if (!sa.Qinv) return;
  if (ty == tx) {
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (ty * B + i < d) colk[1][ty * B + i] = a[i][i];
  }
  __syncthreads();
  if (tid < 64) {
    double mx = 0.0;
    for (int i = tid; i < d; i += 64) mx = fmax(mx, colk[1][i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (tid == 0) sh_tol = (double)d * 2.220446049250313e-16 * mx;
  }
  __syncthreads();
  const double tol = sh_tol;
  bool bad = false;
  for (int k = 0; k < d; ++k) {
    const int bs = k & 1;
    const int kb = k / B, kr = k - (k / B) * B;
    if (ty == kb) {
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i == kr) {
#pragma unroll
          for (int j = 0; j < B; ++j) rowk[bs][tx * B + j] = a[i][j];
        }
    }
    if (tx == kb) {
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j == kr) {
#pragma unroll
          for (int i = 0; i < B; ++i) colk[bs][ty * B + i] = a[i][j];
        }
    }
    __syncthreads();
    const double pv = colk[bs][k];
    if (!(pv > tol)) bad = true;
    const double ip = 1.0 / pv;
    double cf[B], fr[B], rr[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int gi = ty * B + i;
      cf[i] = colk[bs][gi < d ? gi : d - 1];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int gj = tx * B + j;
      rr[j] = rowk[bs][gj < d ? gj : d - 1];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) fr[i] = (ty * B + i == k) ? 0.0 : cf[i];
#pragma unroll
    for (int j = 0; j < B; ++j) rr[j] = (tx * B + j == k) ? 0.0 : rr[j] * ip;
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
      for (int j = 0; j < B; ++j) a[i][j] -= fr[i] * rr[j];
    }
    if (ty == kb) {
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i == kr) {
#pragma unroll
          for (int j = 0; j < B; ++j) a[i][j] = (tx * B + j == k) ? ip : a[i][j] * ip;
        }
    }
    if (tx == kb) {
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j == kr) {
#pragma unroll
          for (int i = 0; i < B; ++i) a[i][j] = (ty * B + i != k) ? -cf[i] * ip : a[i][j];
        }
    }
  }
  const bool any = __syncthreads_or(bad) != 0;
  if (!any) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int gi = ty * B + i, gj = tx * B + j;
        if (gi < d && gj < d) sa.Qinv[gi * d + gj] = a[i][j];
      }
    }
  }
  finish_inverse(any, sa.Q && sa.store_Q ? sa.Q : nullptr, d, sa.Qinv, sa.pw, sa.status, tid,
                 1024);
}

// ---------------------------------------------------------------------------
// MFMA form of the side step for d <= 192.  Q is padded to D = 16*nb with an
// identity block and held in 16x16 tiles in the FP64 MFMA accumulator layout
// (lane l, register v: row l/16 + 4v, column l%16); tile t = ti*nb + tj
// belongs to wave t % 16.  The inverse is the in-place Gauss-Jordan
// elimination taken over 16x16 pivot blocks K:
//   P = A_KK^{-1};  A_Kj <- P A_Kj;  A_iK <- -A_iK P;
//   A_ij <- A_ij - A_iK P A_Kj;  A_KK <- P,
// which leaves A^{-1} after the last block.  The pivot block is inverted by
// its owning wave with cross-lane shuffles; the block updates run on MFMAs.
// The scalar pivots met inside the pivot blocks are the Schur-complement
// diagonals of the unblocked elimination, so the positivity test is the
// same.  One workgroup barrier per pivot block.
// ---------------------------------------------------------------------------

// floor(a / b) for 0 <= a < 2^22 and b > 0, given rb = 1.0f / b: the float
// product is within a relative 2^-23 of (a + 0.5) / b, which lies at least
// 0.5 / b from the nearest integer, so the truncation is exact.  It replaces
// the integer division sequence on the latency-bound side path.
__device__ inline int small_div(int a, float rb) { return (int)(((float)a + 0.5f) * rb); }

// Device-coherent access to data that other workgroups of the same launch
// write: agent-scope relaxed atomic stores and loads are coherent across the
// whole device (every XCD's L2) by themselves, so the Gram tiles handed from
// the Gram workgroups to the side step need no cache write-back or
// invalidation fences.
__device__ inline void coherent_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane moves of the pivot step, all on the VALU (no LDS round trip).
// pair_bcast<G> (G even) gives every lane the values held by the lanes of
// its column in row groups G and G + 1 (lanes 16G.. and 16(G+1)..): an
// exchange of 32-lane halves keeps half G/2 in both, an exchange of 16-lane
// rows then separates the two groups.  row_bcast<p> gives every lane the
// value of lane p of its own 16-lane row (DPP row broadcast; every lane is
// written, so the old value is arbitrary: passing one that is dead
// afterwards spares the copy of a constant).  lane_value<L> reads lane L
// into a wave-uniform value.
template <int G>
__device__ inline void pair_bcast(double x, double& r0, double& r1) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const unsigned lo1 = (G & 2) ? a[1] : a[0], hi1 = (G & 2) ? b[1] : b[0];
  const auto c = __builtin_amdgcn_permlane16_swap(lo1, lo1, false, false);
  const auto e = __builtin_amdgcn_permlane16_swap(hi1, hi1, false, false);
  r0 = __builtin_bit_cast(double, ((unsigned long long)e[0] << 32) | c[0]);
  r1 = __builtin_bit_cast(double, ((unsigned long long)e[1] << 32) | c[1]);
}
template <int P>
__device__ inline double row_bcast(double old, double x) {
  return __builtin_amdgcn_update_dpp(old, x, 0x150 + P, 0xf, 0xf, false);
}
template <int L>
__device__ inline double lane_value(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, L);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), L);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Two pivot steps p, p + 1 (p even) of the in-wave Gauss-Jordan elimination
// at once, as one step with the 2 x 2 pivot block B = {p, p + 1} (tile
// layout: lane l, register v holds T[l/16 + 4v][l%16]; rows p and p + 1
// share register p/4).  With P = T[B][B] = [[a, b], [c, e]]:
//   T'[B][j] = P^-1 T[B][j],  T'[i][B] = -T[i][B] P^-1,  T'[B][B] = P^-1,
//   T'[i][j] = T[i][j] - T[i][B] P^-1 T[B][j]          (i, j not in B),
// which is the result of the two scalar steps.  The cross-lane moves (the
// latency of the step) are shared by the two pivots: both pivot rows come
// from one row-pair exchange, the columns from row broadcasts.  In lanes
// j in B the pivot-row values are replaced by the identity columns, so the
// same expressions give P^-1 in the pivot rows and -T[i][B] P^-1 in the
// pivot columns (where x is masked to zero).  The scalar pivots of the
// unblocked elimination are a and det(P) / a, and are tested as such.
template <int p>
__device__ inline void gj16_step2(d4& c, int r0, int j, double tol, int nvalid, bool& bad,
                                  d4 C0, d4 C1) {
  constexpr int vp = p >> 2, gp = p & 3, gq = gp + 1;
  double R0, R1;                                                // T[p][j], T[p+1][j]
  pair_bcast<gp>(c[vp], R0, R1);
  const double a = lane_value<(gp << 4) | p>(c[vp]);
  const double b = lane_value<(gp << 4) | (p + 1)>(c[vp]);
  const double cc = lane_value<(gq << 4) | p>(c[vp]);
  const double e = lane_value<(gq << 4) | (p + 1)>(c[vp]);
  // C0, C1 (the previous step's, dead now) serve as the old values
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    C0[v] = row_bcast<p>(C0[v], c[v]);                           // T[r0 + 4v][p]
    C1[v] = row_bcast<p + 1>(C1[v], c[v]);                       // T[r0 + 4v][p+1]
  }
  const double det = fma(a, e, -(b * cc));
  if (p < nvalid && !(a > tol)) bad = true;
  if (p + 1 < nvalid && !(det > tol * a)) bad = true;
  // 1/det: hardware reciprocal refined by two Newton steps
  double ip = __builtin_amdgcn_rcp(det);
  ip = fma(fma(-det, ip, 1.0), ip, ip);
  ip = fma(fma(-det, ip, 1.0), ip, ip);
  const bool jb = j == p || j == p + 1;
  const double S0 = jb ? (j == p ? 1.0 : 0.0) : R0;
  const double S1 = jb ? (j == p ? 0.0 : 1.0) : R1;
  const double M0 = fma(e, S0, -(b * S1)) * ip;                 // (P^-1 T[B][j])_0
  const double M1 = fma(a, S1, -(cc * S0)) * ip;                // (P^-1 T[B][j])_1
  const double mb = jb ? 0.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double y = fma(-C0[v], M0, fma(-C1[v], M1, c[v] * mb));
    if (v == vp)
      c[v] = r0 == gp ? M0 : (r0 == gq ? M1 : y);
    else
      c[v] = y;
  }
  if constexpr (p < 14) gj16_step2<p + 2>(c, r0, j, tol, nvalid, bad, C0, C1);
}

// In-place Gauss-Jordan inverse of a 16x16 tile held by one wave in the
// accumulator layout; rows / columns >= nvalid are identity padding and are
// not tested.  Returns true if a tested pivot is not above tol.
__device__ inline bool wave_gj16(d4& c, int lane, double tol, int nvalid) {
  bool bad = false;
  gj16_step2<0>(c, lane >> 4, lane & 15, tol, nvalid, bad, d4{0, 0, 0, 0}, d4{0, 0, 0, 0});
  return bad;
}

// ---------------------------------------------------------------------------
// Column-owner Gauss-Jordan inverse over 16x16 pivot blocks of a symmetric
// positive definite matrix of at most 64 x 64 (nb <= 4 tiles a side) on four
// waves: wave w holds tile column w (A[i] = tile (i, w)) in the MFMA
// accumulator layout.  Step K (pivot block K, P = A_KK^{-1}):
//   A_Kj <- P A_Kj,  A_ij <- A_ij - A_iK (P A_Kj),  A_iK <- -A_iK P,  A_KK <- P.
// The pivot-block inverse is the owner wave's 16 in-register scalar pivots
// (wave_gj16).  Only the pivot row strip (K, i) and P are exchanged, through
// LDS (two buffers, one barrier per step): in-place elimination of a
// symmetric matrix keeps A_iK = (A_Ki)^T while neither block is pivoted and
// A_iK = -(A_Ki)^T once block i is, so the pivot column comes from the
// pivot row, and register q of an accumulator tile is the A operand of
// k-step q of its transpose (P is symmetric, so it serves as its own A
// operand).  Look-ahead: every wave updates its tile of the next pivot row
// first and publishes it; the next owner inverts its updated diagonal tile
// at once, before its other updates.  The scalar pivots are those of the
// unblocked elimination, so the positivity test is the same.
// ---------------------------------------------------------------------------
__device__ inline void gj_cols16(d4 (&A)[4], double* lds, int lane, int wave, int nb, int d,
                                 double tol, bool& bad) {
  // slot i of buffer b: lds + 1024 b + 256 i (tile (K, i), or P in slot K)
  if (wave < nb) {
    if (wave == 0) bad |= wave_gj16(A[0], lane, tol, d);
#pragma unroll
    for (int v = 0; v < 4; ++v) lds[wave * 256 + v * 64 + lane] = A[0][v];
  }
  __syncthreads();
#pragma unroll
  for (int K = 0; K < 4; ++K) {
    if (K >= nb) break;
    const double* Sc = lds + (K & 1) * 1024;
    double* Sn = lds + ((K & 1) ^ 1) * 1024;
    const bool nextp = K + 1 < nb;
    if (wave < nb) {
      if (wave != K) {
        // two accumulators per product (k-steps 0, 1 and 2, 3): a dependent
        // FP64 MFMA chain costs its full latency per step
        d4 U0 = {0, 0, 0, 0}, U1 = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; q += 2) {
          U0 = mfma16(Sc[K * 256 + q * 64 + lane], A[K][q], U0);
          U1 = mfma16(Sc[K * 256 + (q + 1) * 64 + lane], A[K][q + 1], U1);
        }
        const d4 U = U0 + U1;
#pragma unroll
        for (int t = 1; t < 4; ++t) {
          const int i = (K + t) & 3;
          if (i < nb) {
            const double sg = i < K ? 1.0 : -1.0;
            d4 acc = A[i], acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; q += 2) {
              acc = mfma16(sg * Sc[i * 256 + q * 64 + lane], U[q], acc);
              acc1 = mfma16(sg * Sc[i * 256 + (q + 1) * 64 + lane], U[q + 1], acc1);
            }
            A[i] = acc + acc1;
            if (t == 1 && nextp) {
              if (wave == K + 1) bad |= wave_gj16(A[i], lane, tol, d - 16 * (K + 1));
#pragma unroll
              for (int v = 0; v < 4; ++v) Sn[wave * 256 + v * 64 + lane] = A[i][v];
            }
          }
        }
        A[K] = U;
      } else {
#pragma unroll
        for (int t = 1; t < 4; ++t) {
          const int i = (K + t) & 3;
          if (i < nb) {
            const double sg = i < K ? 1.0 : -1.0;
            d4 acc = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; q += 2) {
              acc = mfma16(sg * Sc[i * 256 + q * 64 + lane], A[K][q], acc);
              acc1 = mfma16(sg * Sc[i * 256 + (q + 1) * 64 + lane], A[K][q + 1], acc1);
            }
            A[i] = acc + acc1;
            if (t == 1 && nextp) {
#pragma unroll
              for (int v = 0; v < 4; ++v) Sn[wave * 256 + v * 64 + lane] = A[i][v];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// LDS budget of the side step, in doubles (66 KiB: two 64 x 64 chain operands,
// one of them with padded rows; room is left on the CU for an MTTKRP
// workgroup beside it).
constexpr int SIDE_LDS = 8448;
// allocation: SIDE_LDS plus the spare slot that takes the staging copy's
// out-of-range stores
constexpr int SIDE_LDS_ALLOC = SIDE_LDS + 2;
// The 16-wave side kernel has its compute unit to itself: its budget holds
// both operands of a 100 x 100 x 100 chain product (order-4 streams with
// TR-ranks 10), 158 KiB of the 160.
constexpr int SIDE_LDS_MF = 20200;
constexpr int SIDE_LDS_MF_ALLOC = SIDE_LDS_MF + 2;

// Serial part of the side step, for a workgroup of NW waves: the ring
// product of the transfer-layout factors, the Q tiles (assembly,
// accumulation, store) and the blocked Gauss-Jordan inverse.  MAXT >=
// ceil(nb (nb + 1) / 2 / NW) upper-triangle tiles per wave (four tiles of
// a tile column for the four-wave column-owner form).
template <int NW, int MAXT>
__device__ inline void side_serial(const SideArgs& sa, double* lds, double* dmax, int tid,
                                   bool pre = false, bool mpre = false) {
  // LDS budget in doubles (the allocation has one spare slot past it)
  constexpr int CAP = NW == 16 ? SIDE_LDS_MF : SIDE_LDS;
  // [0] some pivot test failed, [1] waves done (zeroed here; the barriers of
  // the chain product order this before any use)
  __shared__ int fb_rec[2];
  if (tid == 0) {
    fb_rec[0] = 0;
    fb_rec[1] = 0;
  }
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int ar = lane & 15, ak = lane >> 4;
  const int Ra = sa.Ra, Rb = sa.Rb, d = Ra * Rb;
  const int nb = (d + 15) >> 4, ntri = nb * (nb + 1) / 2;
  const float rRa = 1.0f / (float)Ra;
  // tile coordinates of the (up to MAXT) Q tiles of this wave: with four
  // waves and MAXT = 4 (nb <= 4, checked by the host) wave w holds tile
  // column w, as the column-owner elimination needs; otherwise the tiles
  // of the upper triangle (ti <= tj), tile t = wave + NW*s in row-major
  // order over it (the lower triangle follows from the symmetry)
  constexpr bool COLS = NW == 4 && MAXT == 4;
  int TI[MAXT], TJ[MAXT];
  bool TV[MAXT];
  {
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
      if (COLS) {
        TI[s] = s;
        TJ[s] = wave;
        TV[s] = s < nb && wave < nb;
      } else {
        const int t = wave + NW * s;
        TV[s] = t < ntri;
        int rb = 0, cb = TV[s] ? t : 0;
        while (cb >= nb - rb) {
          cb -= nb - rb;
          ++rb;
        }
        TI[s] = rb;
        TJ[s] = cb + rb;
      }
    }
  }
  // the Q entries this lane accumulates, loaded now so that their latency
  // overlaps the chain product
  const bool qacc = sa.Q && sa.accumulate;
  double qpre[MAXT][4];
#pragma unroll
  for (int s = 0; s < MAXT; ++s) {
    const int ti = TV[s] ? TI[s] : nb - 1, tj = TV[s] ? TJ[s] : nb - 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = min(ti * 16 + Acc<double>::row(lane, v), d - 1), gj = min(tj * 16 + ar, d - 1);
      const double q = qacc ? sa.Q[gi * d + gj] : 0.0;
      qpre[s][v] = q;
    }
  }
  // 2. ring product of the transfer-layout factors: both operands staged in
  //    LDS when they fit (rows of the left factor padded by one element, so
  //    the 16 lanes of an operand read 16 different banks and the staging
  //    stores are contiguous), else read through the cache in batches of 8
  //    k-steps.  When the last product has at most 16 tiles it is kept in
  //    LDS for the assembly.
  // M is always a global pointer (a pointer that may also address LDS would
  // turn every load into a flat load with conservative waits); m_lds says
  // the last product is in LDS instead
  // mpre: the Gram workgroups formed the (two-factor) product in cbuf[0]
  const double* M = mpre ? sa.cbuf[0] : (sa.fac[0] ? sa.fac[0] : sa.Ep);
  bool m_lds = false;
  for (int j = 1; j < (mpre ? 1 : sa.nfac); ++j) {
    const double* __restrict__ F = sa.fac[j] ? sa.fac[j] : sa.Ep;
    double* out = sa.cbuf[(j - 1) & 1];
    const int d1 = sa.fr[0], d2 = sa.fc[j - 1], d3 = sa.fc[j];
    const int nb1 = (d1 + 15) >> 4, nb3 = (d3 + 15) >> 4, ntile = nb1 * nb3;
    const int d2p = d2 + 1;
    const float rd2 = 1.0f / (float)d2, rnb3 = 1.0f / (float)nb3;
    const bool staged = d1 * d2p + d2 * d3 <= CAP;
    if (staged && pre && j == 1) {
      // M is already in LDS (loaded by prestage_first_factor while the Gram
      // tile was computed): copy F only
      const int n2 = d2 * d3;
      constexpr int PER = (CAP + 64 * NW - 1) / (64 * NW);
      constexpr int BATCH = NW == 16 ? 10 : PER;   // loads in flight per thread
#pragma unroll 1
      for (int q0 = 0; q0 < PER; q0 += BATCH) {
        double x[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int q = q0 + u;
          if (q < PER && q * 64 * NW < n2) x[u] = coherent_load(F + min(tid + 64 * NW * q, n2 - 1));
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int q = q0 + u;
          const int e = tid + 64 * NW * q;
          if (q < PER && q * 64 * NW < n2) lds[e < n2 ? d1 * d2p + e : CAP] = x[u];
        }
      }
      __syncthreads();
    } else if (staged) {
      // [M (padded rows) | F] copied to LDS with all loads in flight at once:
      // one load per element (the source pointer is selected, both sources
      // clamped in range) and one unconditional LDS store (elements past the
      // end go to the spare slot CAP), so the copy has no branches
      const int n1 = d1 * d2, n2 = d2 * d3;
      constexpr int PER = (CAP + 64 * NW - 1) / (64 * NW);
      constexpr int BATCH = NW == 16 ? 10 : PER;   // loads in flight per thread
#pragma unroll 1
      for (int q0 = 0; q0 < PER; q0 += BATCH) {
        double x[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int e = tid + 64 * NW * (q0 + u);
          const double* src = e < n1 ? M + min(e, n1 - 1) : F + min(max(e - n1, 0), n2 - 1);
          if (q0 + u < PER) x[u] = coherent_load(src);
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int e = tid + 64 * NW * (q0 + u);
          const int em = min(e, n1 - 1);
          const int r = small_div(em, rd2);
          const int dst = e < n1 ? r * d2p + (em - r * d2)
                                 : (e < n1 + n2 ? d1 * d2p + (e - n1) : CAP);
          if (q0 + u < PER) lds[dst] = x[u];
        }
      }
      __syncthreads();
    }
    auto tile_mm = [&](int b) -> d4 {
      const int rb = small_div(b, rnb3), cb = b - rb * nb3;
      const int arow = min(rb * 16 + ar, d1 - 1), bcol = min(cb * 16 + ar, d3 - 1);
      d4 acc = {0, 0, 0, 0};
      const int kfull = d2 & ~3;
      if (staged) {
        const double* Ms = lds;
        const double* Fs = lds + d1 * d2p;
        // two accumulators (alternate k-steps) halve the dependent chain
        d4 acc1 = {0, 0, 0, 0};
        int k0 = 0;
#pragma unroll 4
        for (; k0 + 8 <= kfull; k0 += 8) {
          const int k = k0 + ak;
          acc = mfma16(Ms[arow * d2p + k], Fs[k * d3 + bcol], acc);
          acc1 = mfma16(Ms[arow * d2p + k + 4], Fs[(k + 4) * d3 + bcol], acc1);
        }
        if (k0 < kfull) {
          const int k = k0 + ak;
          acc = mfma16(Ms[arow * d2p + k], Fs[k * d3 + bcol], acc);
        }
        acc += acc1;
      } else {
        int k0 = 0;
        for (; k0 + 32 <= kfull; k0 += 32) {
          double av[8], bv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int k = k0 + 4 * q + ak;
            av[q] = coherent_load(M + (size_t)arow * d2 + k);
            bv[q] = coherent_load(F + (size_t)k * d3 + bcol);
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) acc = mfma16(av[q], bv[q], acc);
        }
        for (; k0 < kfull; k0 += 4) {
          const int k = k0 + ak;
          acc = mfma16(coherent_load(M + (size_t)arow * d2 + k),
                       coherent_load(F + (size_t)k * d3 + bcol), acc);
        }
      }
      if (kfull < d2) {
        // ragged last k-step: lanes past d2 contribute zeros (LDS and global
        // reads kept apart so neither becomes a generic-address load)
        const int k = kfull + ak;
        const int kc = min(k, d2 - 1);
        double av, bv;
        if (staged) {
          av = lds[arow * d2p + kc];
          bv = lds[d1 * d2p + kc * d3 + bcol];
        } else {
          av = coherent_load(M + (size_t)arow * d2 + kc);
          bv = coherent_load(F + (size_t)kc * d3 + bcol);
        }
        acc = mfma16(k < d2 ? av : 0.0, k < d2 ? bv : 0.0, acc);
      }
      return acc;
    };
    auto store_tile = [&](int b, const d4& acc, bool to_lds) {
      const int rb = small_div(b, rnb3), cb = b - rb * nb3;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb * 16 + Acc<double>::row(lane, v), c = cb * 16 + ar;
        if (r < d1 && c < d3) {
          if (to_lds)
            lds[r * d3 + c] = acc[v];
          else
            coherent_store(out + (size_t)r * d3 + c, acc[v]);
        }
      }
    };
    constexpr int RM = (16 + NW - 1) / NW;
    if (ntile <= NW * RM) {
      const bool keep = j == sa.nfac - 1 && d1 * d3 <= CAP;
      d4 res[RM];
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        const int b = wave + NW * t;
        res[t] = b < ntile ? tile_mm(b) : d4{0, 0, 0, 0};
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        const int b = wave + NW * t;
        if (b < ntile) store_tile(b, res[t], keep);
      }
      __syncthreads();
      M = out;
      m_lds = keep;
    } else {
      for (int b = wave; b < ntile; b += NW) store_tile(b, tile_mm(b), false);
      __syncthreads();
      M = out;
    }
  }
  // 3. Q tiles: assembly from the chain product, accumulation, store.  All
  //    chain-product reads first (from LDS or from global memory: two
  //    separate loops, so neither becomes a generic-address load), then the
  //    accumulation and stores.
  const bool storeQ = sa.Q && sa.store_Q;
  double mv[MAXT][4];
  auto m_index = [&](int s, int v) {
    const int tj = TJ[s], ti = TI[s];
    const int gi = ti * 16 + Acc<double>::row(lane, v), gj = tj * 16 + ar;
    const int s1 = small_div(gi, rRa), r = gi - s1 * Ra;
    const int s2 = small_div(gj, rRa), r2 = gj - s2 * Ra;
    const bool ok = TV[s] && gi < d && gj < d;
    return ok ? (s1 + Rb * s2) * (Ra * Ra) + (r + Ra * r2) : 0;
  };
  if (m_lds) {
#pragma unroll
    for (int s = 0; s < MAXT; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) mv[s][v] = lds[m_index(s, v)];
  } else {
#pragma unroll
    for (int s = 0; s < MAXT; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) mv[s][v] = coherent_load(M + m_index(s, v));
  }
  d4 A[MAXT];
  double mx = 0.0;
#pragma unroll
  for (int s = 0; s < MAXT; ++s) {
    const int ti = TI[s], tj = TJ[s];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = ti * 16 + Acc<double>::row(lane, v), gj = tj * 16 + ar;
      const bool ok = TV[s] && gi < d && gj < d;
      double val = mv[s][v];
      if (qacc) val += qpre[s][v];
      if (ok && storeQ) {
        sa.Q[gi * d + gj] = val;
        // the mirror of an upper off-diagonal tile (the upper-triangle
        // elimination keeps only those; Q stays exactly symmetric)
        if (!COLS && ti != tj) sa.Q[gj * d + gi] = val;
      }
      if (ok && gi == gj) mx = fmax(mx, val);
      A[s][v] = ok ? val : (gi == gj ? 1.0 : 0.0);
    }
  }
  if (!sa.Qinv) return;
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) dmax[wave] = mx;
  __syncthreads();
  mx = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) mx = fmax(mx, dmax[w]);
  const double tol = (double)d * 2.220446049250313e-16 * mx;
  bool bad = false;
  if constexpr (COLS) {
    // 4. column-owner elimination over 16x16 pivot blocks
    gj_cols16(A, lds, lane, wave, nb, d, tol, bad);
  } else {
  // 4. blocked Gauss-Jordan over the upper-triangle tiles, LDS
  //    double-buffered per pivot block: Pb = P (row-major), PbT = P^T,
  //    RowB[j] = A_Kj (row-major), ColT[i] = A_iK^T.  In-place elimination
  //    of a symmetric matrix keeps A_ab = A_ba^T when both or neither of the
  //    blocks a, b have been pivoted and A_ab = -A_ba^T when exactly one has,
  //    so before pivot block K (pivoted: blocks < K) the strips come from the
  //    upper tiles alone: for i > K, RowB[i] = ColT[i] = tile (K, i); for
  //    i < K, ColT[i] = tile(i, K)^T and RowB[i] = -tile(i, K)^T.  The block
  //    updates below are those of the full elimination restricted to i <= j.
  const int bstride = 2 * nb * 256 + 512;
  const bool dbuf = 2 * bstride <= CAP;
  const int kq = lane >> 4, cl = lane & 15;
  for (int K = 0; K < nb; ++K) {
    double* Pb = lds + (dbuf ? (K & 1) * bstride : 0);
    double* PbT = Pb + 256;
    double* RowB = Pb + 512;
    double* ColT = RowB + nb * 256;
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
      if (TV[s]) {
        const int ti = TI[s], tj = TJ[s];
        if (ti == K && tj == K) {
          bad |= wave_gj16(A[s], lane, tol, d - 16 * K);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = Acc<double>::row(lane, v);
            Pb[r * 16 + cl] = A[s][v];
            PbT[cl * 16 + r] = A[s][v];
          }
        } else if (ti == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int o = Acc<double>::row(lane, v) * 16 + cl;
            RowB[tj * 256 + o] = A[s][v];
            ColT[tj * 256 + o] = A[s][v];
          }
        } else if (tj == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int o = cl * 16 + Acc<double>::row(lane, v);
            ColT[ti * 256 + o] = A[s][v];
            RowB[ti * 256 + o] = -A[s][v];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
      if (TV[s]) {
        const int ti = TI[s], tj = TJ[s];
        if (ti == K && tj == K) {
          // holds P already
        } else if (ti == K) {
          // A_Kj <- P A_Kj
          d4 acc = {0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = (4 * q + kq) * 16 + cl;
            acc = mfma16(PbT[o], RowB[tj * 256 + o], acc);
          }
          A[s] = acc;
        } else if (tj == K) {
          // A_iK <- -A_iK P
          d4 acc = {0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = (4 * q + kq) * 16 + cl;
            acc = mfma16(-ColT[ti * 256 + o], Pb[o], acc);
          }
          A[s] = acc;
        } else {
          // U = -P^T A_iK^T = (-A_iK P)^T: its accumulator layout is the
          // A-operand layout of -A_iK P, so A_ij += (-A_iK P) A_Kj follows.
          d4 u = {0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = (4 * q + kq) * 16 + cl;
            u = mfma16(-Pb[o], ColT[ti * 256 + o], u);
          }
          d4 acc = A[s];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = (4 * q + kq) * 16 + cl;
            acc = mfma16(u[q], RowB[tj * 256 + o], acc);
          }
          A[s] = acc;
        }
      }
    }
    if (!dbuf) __syncthreads();
  }
  }
  const int cl = lane & 15;
#pragma unroll
  for (int s = 0; s < MAXT; ++s) {
    if (TV[s]) {
      const int ti = TI[s], tj = TJ[s];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = ti * 16 + Acc<double>::row(lane, v), gj = tj * 16 + cl;
        if (gi < d && gj < d) {
          sa.Qinv[gi * d + gj] = A[s][v];
          // all blocks pivoted: the inverse is symmetric
          if (!COLS && ti != tj) sa.Qinv[gj * d + gi] = A[s][v];
        }
      }
    }
  }
  if (!sa.status) return;
  // The waves do not wait for each other here (a workgroup barrier at this
  // point measured about 2.5 us per launch): each wave records a failed
  // pivot test in LDS, waits for its own stores, and counts itself out;
  // the last wave out reads the record and, if a test failed, replaces the
  // stored inverse by the pseudo-inverse on its own (its stores follow the
  // other waves', which completed before they counted out).
  if (bad) atomicOr(fb_rec, 1);
  __builtin_amdgcn_s_waitcnt(0);
  int prev = 0;
  if (lane == 0) prev = atomicAdd(fb_rec + 1, 1);
  prev = __shfl(prev, 0);
  if (prev != NW - 1) return;
  const bool any = atomicOr(fb_rec, 0) != 0;
  finish_inverse(any, storeQ ? sa.Q : nullptr, d, sa.Qinv, sa.pw, sa.status, lane, 64);
}

// One upper-triangle 16x16 tile (index `tile`, row-major over the upper
// triangle) of G_(2)^T G_(2) of the previous core: the rows are split over
// the NW waves (8 k-steps of loads in flight per wave), the partial tiles
// summed in LDS in a fixed order, and the tile and its mirror written in the
// transfer layout.
template <int NW, bool WEIGHTED = false>
__device__ inline void gram_tile(const SideArgs& sa, double* lds, int tid, int tile,
                                 double* keep = nullptr) {
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int ar = lane & 15, ak = lane >> 4;
  const int Ra = sa.Rpa, Rb = sa.Rpb, dp = Ra * Rb;
  const int nbp = (dp + 15) >> 4;
  int rb = 0, cb = tile;
  while (cb >= nbp - rb) {
    cb -= nbp - rb;
    ++rb;
  }
  cb += rb;
  const int64_t rows = sa.rows_p, rl = rows > 0 ? rows - 1 : 0;
  const int64_t nks = (rows + 3) / 4;
  const double* __restrict__ Gp = sa.Gp;
  const int c1 = min(rb * 16 + ar, dp - 1), c2 = min(cb * 16 + ar, dp - 1);
  // KB k-steps of loads in flight per wave (16 with four waves, 8 with the
  // 16-wave kernel's register budget); with four waves four accumulators
  // (k-steps q mod 4) shorten the dependent MFMA chains
  constexpr int KB = NW <= 4 ? 16 : 8;
  d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0}, acc3 = {0, 0, 0, 0};
  for (int64_t k0 = wave; k0 < nks; k0 += KB * NW) {
    double av[KB], bv[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int64_t ks = k0 + NW * q;
      const int64_t i = ks * 4 + ak;
      const int64_t ic = i < rows ? i : rl;
      const double xa = Gp[ic * dp + c1], xb = Gp[ic * dp + c2];
      const double wa = WEIGHTED ? sa.Gw[ic] : 1.0;
      const bool ok = i < rows && ks < nks;
      av[q] = ok ? (WEIGHTED ? xa * wa : xa) : 0.0;
      bv[q] = ok ? xb : 0.0;
    }
    if constexpr (NW <= 4) {
#pragma unroll
      for (int q = 0; q < KB; q += 4) {
        acc0 = mfma16(av[q], bv[q], acc0);
        acc1 = mfma16(av[q + 1], bv[q + 1], acc1);
        acc2 = mfma16(av[q + 2], bv[q + 2], acc2);
        acc3 = mfma16(av[q + 3], bv[q + 3], acc3);
      }
    } else {
#pragma unroll
      for (int q = 0; q < KB; ++q) acc0 = mfma16(av[q], bv[q], acc0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    lds[wave * 256 + Acc<double>::row(lane, v) * 16 + ar] = (acc0[v] + acc1[v]) + (acc2[v] + acc3[v]);
  __syncthreads();
  for (int e = tid; e < 256; e += 64 * NW) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += lds[w * 256 + e];
    const int r = rb * 16 + (e >> 4), c = cb * 16 + (e & 15);
    if (keep) keep[e] = r < dp && c < dp ? sum : 0.0;
    // weighted: (w x) y and (w y) x may differ in the last bit, so in the
    // diagonal tile only r <= c writes (both positions: exactly symmetric)
    if (r < dp && c < dp && (!WEIGHTED || r <= c)) {
      const float rRa = 1.0f / (float)Ra;
      const int b1 = small_div(r, rRa), a1 = r - b1 * Ra, b2 = small_div(c, rRa), a2 = c - b2 * Ra;
      coherent_store(sa.Ep + (size_t)(a1 + Ra * a2) * (Rb * Rb) + (b1 + Rb * b2), sum);
      coherent_store(sa.Ep + (size_t)(a2 + Ra * a1) * (Rb * Rb) + (b2 + Rb * b1), sum);
    }
  }
}

// The first factor of the side step's ring product is never the Gram matrix
// that the launch's Gram tiles refresh (that one is always the last factor),
// so every Gram workgroup loads it while its tile is computed and leaves it
// in LDS in the padded-row layout of the staged product; the workgroup that
// goes on with the side step then copies only the second factor.  Not done
// when the first product is not staged or the factor exceeds one register
// batch (FirstFactor::ok false).
struct FirstFactor {
  static constexpr int PER = 16;            // 4096 doubles over 256 threads
  double x[PER];
  bool ok;
};

__device__ inline void prestage_first_factor_load(const SideArgs& sa, FirstFactor& ff, int tid) {
  ff.ok = false;
  if (sa.nfac < 2 || !sa.fac[0] || sa.fac[0] == sa.Ep) return;
  const int d1 = sa.fr[0], d2 = sa.fc[0], d3 = sa.fc[1];
  ff.ok = d1 * d2 <= 256 * FirstFactor::PER && d1 * (d2 + 1) + d2 * d3 <= SIDE_LDS;
  if (!ff.ok) return;
  const double* __restrict__ M = sa.fac[0];
  const int n1 = d1 * d2;
#pragma unroll
  for (int q = 0; q < FirstFactor::PER; ++q) ff.x[q] = M[min(tid + 256 * q, n1 - 1)];
}

// After the Gram tile (its LDS use must be over): the loaded factor to LDS.
__device__ inline void prestage_first_factor_store(const SideArgs& sa, const FirstFactor& ff,
                                                   double* lds, int tid) {
  if (!ff.ok) return;
  const int d2 = sa.fc[0], d2p = d2 + 1, n1 = sa.fr[0] * d2;
  const float rd2 = 1.0f / (float)d2;
#pragma unroll
  for (int q = 0; q < FirstFactor::PER; ++q) {
    const int e = tid + 256 * q;
    const int em = min(e, n1 - 1);
    const int r = small_div(em, rd2);
    lds[e < n1 ? r * d2p + (em - r * d2) : SIDE_LDS] = ff.x[q];
  }
}

// Arrival of a Gram workgroup: count it in once its tile is stored; true for
// the last of `total` to arrive (which also resets the counter).  The tile
// stores are device-coherent atomic stores: each thread waits for its own to
// complete (vmcnt covers stores on gfx9) before the barrier, so every tile is
// in place before its workgroup's count, and the last workgroup, which reads
// the tiles with device-coherent loads issued after it has seen the full
// count, needs no fence on either side (a __threadfence here writes back and
// invalidates the L2 of the workgroup's XCD, several microseconds).
__device__ inline bool gram_arrive(unsigned* counter, unsigned total, int tid) {
  __shared__ int sh_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0)
    sh_last = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
              total - 1;
  __syncthreads();
  if (!sh_last) return false;
  if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// One 16 x 16 tile of the sketched product (SideArgs::Pout) on a 16-wave
// workgroup: wave w takes the k-steps w, w + 16, .. (4 samples each), 8 of
// them with their loads in flight, on FP64 MFMAs; the wave sums are added in
// LDS in a fixed order.
__device__ inline void sketch_ptile(const SideArgs& sa, double* lds, int tid, int pt) {
  constexpr int NW = 16, KB = 8;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int ar = lane & 15, ak = lane >> 4;
  const int dp = sa.Rpa * sa.Rpb, nbp = (dp + 15) >> 4;
  const int rb = pt / nbp, cb = pt - rb * nbp;
  const int64_t rows = sa.rows_p, rl = rows > 0 ? rows - 1 : 0;
  const int64_t nks = (rows + 3) / 4;
  const bool rok = rb * 16 + ar < sa.pIn;
  const int64_t irow = rok ? rb * 16 + ar : sa.pIn - 1;
  const int col = min(cb * 16 + ar, dp - 1);
  d4 acc = {0, 0, 0, 0};
  for (int64_t k0 = wave; k0 < nks; k0 += KB * NW) {
    double av[KB], bv[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int64_t ks = k0 + NW * q;
      const int64_t smp = ks * 4 + ak;
      const int64_t sc = smp < rows ? smp : rl;
      int64_t off = irow * sa.xsn;
      for (int p = 0; p < sa.xN; ++p)
        if (p != sa.xn) off += (int64_t)sa.idxs[(size_t)p * sa.im + sc] * sa.xstride[p];
      const double xa = sa.xdt == F32 ? (double)((const float*)sa.Xs)[off]
                                      : ((const double*)sa.Xs)[off];
      const double xb = sa.Gp[sc * dp + col] * (sa.Gw ? sa.Gw[sc] : 1.0);
      const bool ok = smp < rows && ks < nks;
      av[q] = ok && rok ? xa : 0.0;
      bv[q] = ok ? xb : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KB; ++q) acc = mfma16(av[q], bv[q], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) lds[wave * 256 + Acc<double>::row(lane, v) * 16 + ar] = acc[v];
  __syncthreads();
  if (tid < 256) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += lds[w * 256 + tid];
    const int64_t r = rb * 16 + (tid >> 4);
    const int c = cb * 16 + (tid & 15);
    if (r < sa.pIn && c < dp) sa.Pout[r * dp + c] = sum;
  }
}

template <int MAXT>
__global__ __launch_bounds__(1024) void k_side_mf(SideArgs sa) {
  extern __shared__ double lds[];
  __shared__ double dmax[16];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int ar = lane & 15, ak = lane >> 4;
  // 1. Gram of the previous core, spread over the grid (one upper-triangle
  //    tile per workgroup); the last workgroup to finish goes on with the
  //    chain, Q and the inverse while the others exit.  The workgroups past
  //    the Gram tiles form the sketched product's tiles, which nothing in
  //    this launch reads.
  if (sa.Gp) {
    const int nbp = (sa.Rpa * sa.Rpb + 15) >> 4;
    const int ngram = nbp * (nbp + 1) / 2;
    if ((int)blockIdx.x >= ngram) {
      sketch_ptile(sa, lds, tid, blockIdx.x - ngram);
      return;
    }
    if (sa.Gw)
      gram_tile<16, true>(sa, lds, tid, blockIdx.x);
    else
      gram_tile<16>(sa, lds, tid, blockIdx.x);
    if (!gram_arrive(sa.counter, (unsigned)ngram, tid)) return;
  }
  side_serial<16, MAXT>(sa, lds, dmax, tid);
}

// ---------------------------------------------------------------------------
// One mode of the STR update in one launch (Alg. 4): the first workgroups
// each form one upper-triangle tile of the Gram of the core updated just
// before, and the last of them to finish runs the rest of the side step
// (Gram chain, Q update, inverse) with its 4 waves; every other workgroup
// runs one MTTKRP tile.  The side step and the MTTKRP do not read what the
// other writes, and no workgroup waits for another; the split reduction and
// solve follow on the same stream.
// ---------------------------------------------------------------------------
// Two-factor chain product M = E_a E_p (E_a the older factor, already in
// LDS with padded rows; E_p the transfer layout of the Gram being formed)
// for R_p = 8: Gram index c = a + 8 b, E_p[(a1 + 8 a2)][(b1 + R' b2)] =
// Gram[a1 + 8 b1][a2 + 8 b2], so the 16 x 16 Gram tile (rb, cb) holds the
// whole columns b1 in {2 rb, 2 rb + 1}, b2 in {2 cb, 2 cb + 1} of E_p, and
// its mirror the columns with rb and cb exchanged.  Each Gram workgroup
// therefore forms those (up to 8) columns of M, one 16-row tile of M per
// wave on FP64 MFMAs (B operand: column n < 8 of the tile's set, zero
// beyond), and stores them to cbuf[0] with device-coherent stores before it
// counts itself in.
__device__ inline bool mcols_ok(const SideArgs& sa) {
  return sa.mcols && sa.nfac == 2 && sa.Rpa == 8 && sa.fr[0] == 64 && sa.fc[0] == 64;
}

__device__ inline void gram_chain_cols(const SideArgs& sa, const double* tl, const double* lds,
                                       int tid, int tile) {
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int Rb = sa.Rpb, d3 = Rb * Rb, dp = 8 * Rb, nbp = (dp + 15) >> 4;
  int rb = 0, cb = tile;
  while (cb >= nbp - rb) {
    cb -= nbp - rb;
    ++rb;
  }
  cb += rb;
  // this lane's B column n = l16: tile group (n < 4) or mirror group (n < 8)
  const int n = l16;
  const bool mir = n >= 4;
  const int u = n & 1, v = (n >> 1) & 1;
  const int b1 = mir ? 2 * cb + u : 2 * rb + u, b2 = mir ? 2 * rb + v : 2 * cb + v;
  const bool colok = n < (rb == cb ? 4 : 8) && b1 < Rb && b2 < Rb;
  constexpr int d2p = 65;                   // padded rows of the staged E_a
  // four accumulators (k-steps q mod 4): a dependent FP64 MFMA chain costs
  // its full latency per step
  d4 ac[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = 4 * q + g4;               // k = a1 + 8 a2
    const int a1 = k & 7, a2 = k >> 3;
    // tile (rb, cb) entry (a1 + 8 u, a2 + 8 v), or for the mirror group the
    // tile entry (a2 + 8 v, a1 + 8 u)
    const int ti = mir ? a2 + 8 * v : a1 + 8 * u, tj = mir ? a1 + 8 * u : a2 + 8 * v;
    const double bv = colok ? tl[ti * 16 + tj] : 0.0;
    ac[q & 3] = mfma16(lds[(16 * wave + l16) * d2p + k], bv, ac[q & 3]);
  }
  const d4 acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
  if (colok) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int row = 16 * wave + Acc<double>::row(lane, w);
      coherent_store(sa.cbuf[0] + (size_t)row * d3 + b1 + Rb * b2, acc[w]);
    }
  }
}

// MTTKRP workgroup w (of nw) of the fused launch -> (chunk, row tile).
// Workgroups go to the 8 XCDs round robin, so w and w + 8 share an XCD and
// its L2: with an even number of row tiles those two take row tiles 2k and
// 2k + 1 of one chunk, whose rows are adjacent in X when the row index is
// the unit-stride one (16 FP32 rows fill half of a 128-byte line, which the
// pair then fetches once).  A last incomplete group of 16 keeps the plain
// order.
__device__ inline void mode_tile(int w, int nw, int nsplit, int mtiles, int* chunk, int* mtile) {
  if (mtiles & 1) {
    *chunk = w % nsplit;
    *mtile = w / nsplit;
    return;
  }
  const int unit = w < (nw & ~15) ? (w & ~15) + 2 * (w & 7) + ((w >> 3) & 1) : w;
  const int pr = unit >> 1;
  *chunk = pr % nsplit;
  *mtile = 2 * (pr / nsplit) + (unit & 1);
}

template <typename T, typename TC, int NJ, int MAXT, int NG, bool PRV>
__global__ __launch_bounds__(256 * NG, 2 / NG) void k_mode(Geom g, MttkrpPlan p, const T* __restrict__ X,
                                                 CoreView cv,
                                                 typename Acc<T>::type* __restrict__ part,
                                                 SideArgs sa) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double dmax[4];
  const int nbp = (sa.Rpa * sa.Rpb + 15) >> 4;
  const int ngram = sa.Gp ? nbp * (nbp + 1) / 2 : 1;
  if ((int)blockIdx.x < ngram) {
    // four waves: with 8-wave workgroups the other four end here (a barrier
    // waits only for the waves that have not ended)
    if (NG > 1 && threadIdx.x >= 256) return;
    // the side step is the longer chain: its waves take issue priority over
    // the MTTKRP waves sharing the compute unit
    __builtin_amdgcn_s_setprio(3);
    double* lds = (double*)smem;
    __shared__ double tl[256];
    bool pre = false, mpre = false;
    if (sa.Gp) {
      FirstFactor ff;
      prestage_first_factor_load(sa, ff, threadIdx.x);
      const bool mc = mcols_ok(sa);
      gram_tile<4>(sa, lds, threadIdx.x, blockIdx.x, mc ? tl : nullptr);
      __syncthreads();
      prestage_first_factor_store(sa, ff, lds, threadIdx.x);
      pre = ff.ok;
      // (ff.ok holds whenever mcols_ok does: 64 x 64 factors)
      if (mc && ff.ok) {
        __syncthreads();
        gram_chain_cols(sa, tl, lds, threadIdx.x, blockIdx.x);
        mpre = true;
      }
      if (!gram_arrive(sa.counter, (unsigned)ngram, threadIdx.x)) return;
    }
    side_serial<4, MAXT>(sa, lds, dmax, threadIdx.x, pre, mpre);
    return;
  }
  int chunk, mtile;
  mode_tile(blockIdx.x - ngram, gridDim.x - ngram, p.nsplit, p.mtiles, &chunk, &mtile);
  mttkrp_body<T, TC, NJ, 0, NG, PRV>(g, p, X, cv, part, chunk, mtile, smem);
}

bool mode_fusable(const Geom& g, const SideArgs& sa) {
  return sa.Ra * sa.Rb <= 64 && g.d <= 64;
}

// The side step is latency-bound on one compute unit and slows down by
// about a tenth when an MTTKRP workgroup shares that unit, while an MTTKRP
// workgroup costs about 11 us per outer index (FP64 operands; 17 us with
// FP32 operands, whose core operand is still read in FP64) and is latency-
// rather than throughput-bound.  Measured on the 256 x 256 x 20 batch
// (side step about 33 us): with FP64 operands one workgroup per compute
// unit wins while it leaves each workgroup at most two outer indices
// (modes 1 and 2: 26-28 us of MTTKRP); otherwise (FP32 operands, the
// temporal mode) one outer index per workgroup, up to four workgroups per
// compute unit; larger batches keep the plan of about 512 workgroups.
// Pairs of outer indices on 8-wave workgroups (two groups of four waves,
// one outer index each at a time) when the plan gives every workgroup at
// least two and the workgroups fit beside the Gram workgroups one per
// compute unit (their LDS takes most of one); otherwise 4-wave workgroups.
static MttkrpPlan pair_groups(MttkrpPlan p, const Geom& g, int ncu, int ngram) {
  if (getenv("TRSTREAM_NG1") || p.Kout < 2) return p;
  const int64_t free_cu = ncu - ngram;
  if (p.upw == 1 && (int64_t)p.mtiles * ((p.Kout + 1) / 2) <= free_cu) {
    p.upw = 2;
    p.nsplit = (int)((p.Kout + 1) / 2);
  }
  if (p.upw >= 2 && (int64_t)p.nsplit * p.mtiles <= free_cu) p.ng = 2;
  return p;
}

MttkrpPlan plan_mode(const Geom& g, int xdtype, const SideArgs& sa, int ncu) {
  const int nbp = (sa.Rpa * sa.Rpb + 15) / 16;
  const int ngram = sa.Gp ? nbp * (nbp + 1) / 2 : 1;
  if (xdtype == F64 && ncu > ngram) {
    const MttkrpPlan p = plan_mttkrp(g, xdtype, ncu - ngram);
    if (p.upw <= 2) return pair_groups(p, g, ncu, ngram);
  }
  MttkrpPlan p = plan_mttkrp(g, xdtype);
  const int64_t wg1 = (int64_t)p.mtiles * p.Kout;   // one outer index per workgroup
  if (p.upw > 1 && wg1 <= 4 * (int64_t)ncu && !getenv("TRSTREAM_NSPLIT")) {
    p.upw = 1;
    p.nsplit = (int)p.Kout;
  }
  return pair_groups(p, g, ncu, ngram);
}

template <typename T, int NJ, int MAXT>
static hipError_t launch_mode_t(const Geom& g, const MttkrpPlan& p, const void* X,
                                const CoreView& cv, void* part, const SideArgs& sa,
                                hipStream_t st) {
  typedef typename Acc<T>::type PT;
  const int dfp = 16 * p.nbf;
  const int Rn1 = g.R[(g.n + 1) % g.N], Rf1 = g.R[(p.f + 1) % g.N];
  const int wst = 16 * ((Rn1 * Rf1 + 15) / 16);
  const size_t lmt = (size_t)(3 * 256 + 16 * wst) * sizeof(double) +
                     (size_t)(16 * dfp) * p.KS * sizeof(PT);
  // two groups of four waves (two outer indices at a time) when the plan
  // says so: per group its own region, and room in the second for the 16
  // doubles per thread that carry its sums to the first
  const int ng = p.ng == 2 && p.upw >= 2 ? 2 : 1;
  const size_t lgrp = (lmt + 15) & ~(size_t)15;
  const size_t lmg = ng == 2 ? lgrp + std::max(lgrp, (size_t)(16 * 256 * sizeof(double))) : lmt;
  const size_t lds = std::max(lmg, (size_t)SIDE_LDS_ALLOC * sizeof(double));
  // the per-row temporal form only on 8-wave workgroups (the planner's rule)
  if (p.prv && ng != 2) return hipErrorInvalidValue;
  auto fn = p.prv ? k_mode<T, double, NJ, MAXT, 2, true>
                  : (ng == 2 ? k_mode<T, double, NJ, MAXT, 2, false>
                             : k_mode<T, double, NJ, MAXT, 1, false>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int nbp = (sa.Rpa * sa.Rpb + 15) / 16;
  const unsigned ngram = sa.Gp ? (unsigned)(nbp * (nbp + 1) / 2) : 1u;
  const unsigned grid = ngram + (unsigned)p.nsplit * (unsigned)p.mtiles;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256 * ng), lds, st, g, p, (const T*)X, cv,
                     (typename Acc<T>::type*)part, sa);
  return hipGetLastError();
}

template <typename T, int MAXT>
static hipError_t launch_mode_j(const Geom& g, const MttkrpPlan& p, const void* X,
                                const CoreView& cv, void* part, const SideArgs& sa,
                                hipStream_t st) {
  const int nj = (p.nbf + 4 / p.KS - 1) / (4 / p.KS);
  switch (nj) {
    case 1: return launch_mode_t<T, 1, MAXT>(g, p, X, cv, part, sa, st);
    case 2: return launch_mode_t<T, 2, MAXT>(g, p, X, cv, part, sa, st);
    case 3: return launch_mode_t<T, 3, MAXT>(g, p, X, cv, part, sa, st);
    default: return launch_mode_t<T, 4, MAXT>(g, p, X, cv, part, sa, st);
  }
}

hipError_t launch_mode(const Geom& g, const MttkrpPlan& p, const void* X, int xdt,
                       const CoreView& cv, int cdt, void* part, const SideArgs& sa,
                       hipStream_t st) {
  if (cdt != F64 || !mode_fusable(g, sa)) return hipErrorInvalidValue;
  const int f = p.f;
  const int64_t xspan = (g.In - 1) * p.sm + (g.I[f] - 1) * p.sf + 1;
  const int64_t gspan = (g.I[f] - 1) * cv.si[f] + (g.R[f] - 1) * cv.sr[f] +
                        (g.R[(f + 1) % g.N] - 1) * cv.ss[f] + 1;
  if (xspan >= ((int64_t)1 << 31) || gspan >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  // four tiles per wave: the side step's column-owner elimination holds a
  // tile column (nb <= 4, guaranteed by mode_fusable) per wave
  if (xdt == F64) return launch_mode_j<double, 4>(g, p, X, cv, part, sa, st);
  if (xdt == F32) return launch_mode_j<float, 4>(g, p, X, cv, part, sa, st);
  return hipErrorInvalidValue;
}

template <int MAXT>
static hipError_t launch_side_mf(const SideArgs& a, int nb, hipStream_t st) {
  const size_t lds = (size_t)SIDE_LDS_MF_ALLOC * sizeof(double);
  auto fn = k_side_mf<MAXT>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  unsigned grid = 1;
  if (a.Gp) {
    const int nbp = (a.Rpa * a.Rpb + 15) / 16;
    grid = (unsigned)(nbp * (nbp + 1) / 2);
    if (a.Pout) grid += (unsigned)(((a.pIn + 15) / 16) * nbp);
  }
  hipLaunchKernelGGL(fn, dim3(grid), dim3(1024), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_side(const SideArgs& a, hipStream_t st) {
  const int d = a.Ra * a.Rb;
  if (d > 256) return hipErrorInvalidValue;
  const int nb = (d + 15) / 16;
  static const bool scalar_gj = getenv("TRSTREAM_SCALAR_GJ") != nullptr;
  // the sketched product tiles exist in the 16-wave kernel only
  if (a.Pout && (nb > 12 || scalar_gj || !a.Gp || a.pIn < 1)) return hipErrorInvalidValue;
  if (nb <= 12 && !scalar_gj) {
    // 16 waves over the nb (nb + 1) / 2 upper-triangle tiles
    const int ntri = nb * (nb + 1) / 2;
    if (ntri <= 16) return launch_side_mf<1>(a, nb, st);
    if (ntri <= 32) return launch_side_mf<2>(a, nb, st);
    if (ntri <= 48) return launch_side_mf<3>(a, nb, st);
    if (ntri <= 64) return launch_side_mf<4>(a, nb, st);
    return launch_side_mf<5>(a, nb, st);
  }
  const int B = (d + 31) / 32;
#define TRK_SIDE(BB) \
  hipLaunchKernelGGL(k_side<BB>, dim3(1), dim3(1024), 0, st, a)
  switch (B) {
    case 1: TRK_SIDE(1); break;
    case 2: TRK_SIDE(2); break;
    case 3: TRK_SIDE(3); break;
    case 4: TRK_SIDE(4); break;
    case 5: TRK_SIDE(5); break;
    case 6: TRK_SIDE(6); break;
    case 7: TRK_SIDE(7); break;
    default: TRK_SIDE(8); break;
  }
#undef TRK_SIDE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dtype conversion, fills, finite check
// ---------------------------------------------------------------------------
__device__ inline double load_as_double(const void* p, int dt, int64_t i) {
  if (dt == F64) return ((const double*)p)[i];
  if (dt == F32) return (double)((const float*)p)[i];
  return (double)__bfloat162float(((const __hip_bfloat16*)p)[i]);
}

__global__ void k_cast(const void* src, int sdt, void* dst, int ddt, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (sdt == F64 && ddt == F32) {
      ((float*)dst)[i] = (float)((const double*)src)[i];
    } else if (ddt == BF16) {
      // FP64 data is rounded to bfloat16 once, not through FP32
      if (sdt == F64)
        ((uint16_t*)dst)[i] = bf16_bits_rne(((const double*)src)[i]);
      else
        ((__hip_bfloat16*)dst)[i] = __float2bfloat16(((const float*)src)[i]);
    } else if (ddt == F64) {
      ((double*)dst)[i] = load_as_double(src, sdt, i);
    } else if (ddt == F32) {
      ((float*)dst)[i] = (float)load_as_double(src, sdt, i);
    }
  }
}

hipError_t launch_cast(const void* src, int sdt, void* dst, int ddt, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)blocks), dim3(256), 0, st, src, sdt, dst, ddt, n);
  return hipGetLastError();
}

__global__ void k_fill(double* y, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, y, v, n);
  return hipGetLastError();
}

__global__ void k_check_finite(const void* x, int dt, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = load_as_double(x, dt, i);
    if (!isfinite(v)) bad = true;
  }
  if (bad) flag[0] = 1;
}

hipError_t launch_check_finite(const void* x, int dt, int64_t n, int* flag, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, st, x, dt, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reconstruction error: per workgroup, 16 columns j of the temporal-mode
// unfolding X_[N] (j = lin(i_0..i_{N-2})), all T slices:
//   Xhat[j, t] = sum_c G_{N(2)}[t, c] G^{!=N}_[2][j, c]
// (the identity X_[N] = G_{N(2)} (G^{!=N}_[2])^T of eq. tr_als).  The 16
// subchain rows are formed in LDS; the product with the temporal core runs
// on FP64 16x16x4 MFMAs (A = subchain rows from LDS, B = the temporal core
// from a slice-major FP64 copy GNs[t * d + c]), one 16-slice tile per wave
// at a time with 8 k-steps of loads in flight, and the squared residual and
// norm are taken from the accumulators.
// ---------------------------------------------------------------------------
constexpr int RECON_JT = 16;

template <typename TX, typename TC, int RM>
__global__ __launch_bounds__(256) void k_recon_err(Geom g, const TX* __restrict__ X, CoreView cv,
                                                   const double* __restrict__ GNs,
                                                   double* __restrict__ wg_out) {
  constexpr int JT = RECON_JT;
  extern __shared__ __align__(16) char smem[];
  double* Bt = (double*)smem;                        // [JT][d+1]
  int* idx = (int*)(Bt + (size_t)JT * (g.d + 1));    // [JT][MAXN]
  __shared__ double red[2][256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int d = g.d;
  const int Rn = g.R[g.n], Rn1 = g.R[0];
  const int64_t J = g.L;                             // columns of X_[N]
  const int64_t T = g.In;
  const int64_t j0 = (int64_t)blockIdx.x * JT;
  // S(j) = G_0(i_0) V(o) with j = i_0 + I_0 o and V(o) the ring product of
  // the slices of modes 1..N-2 at o.  When the workgroup's columns share one
  // o, V(o) is formed once (in red[0], scratch red[1]) and each row tile is
  // a 16x16x16 product on MFMAs (wave w: columns 4w..4w+3); otherwise each
  // subchain row is formed on its own.
  const int64_t I0 = g.I[0];
  const int64_t oA = j0 / I0, oB = (j0 + JT - 1 < J ? j0 + JT - 1 : J - 1) / I0;
  if (oA == oB) {
    double* Vs = red[0];
    ring_product_lds<TC>(g, cv, oA, 1, g.N - 2, Vs, red[1], tid);
    const int R0 = g.R[0], R1 = g.R[1];
    const TC* __restrict__ G0 = (const TC*)cv.ptr[0];
    const int64_t sr0 = cv.sr[0], si0 = cv.si[0], ss0 = cv.ss[0];
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
      const int jj = wave * 4 + t4;
      const int64_t j = j0 + jj;
      const int64_t i0 = j < J ? j - oA * I0 : 0;
      d4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4) {
        const int b = k0 + g4;
        const bool ok = l16 < R0 && b < R1 && j < J;
        const double av =
            (double)G0[i0 * si0 + (ok ? l16 : 0) * sr0 + (ok ? b : 0) * ss0];
        acc = mfma16(ok ? av : 0.0, Vs[b * 16 + l16], acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sv = Acc<double>::row(lane, v);
        if (sv < R0 && l16 < Rn) Bt[jj * (d + 1) + l16 + Rn * sv] = acc[v];
      }
    }
  } else {
    for (int jj = tid; jj < JT; jj += 256) {
      const int64_t j = j0 + jj;
      if (j < J) decode_column(g, j, idx + jj * MAXN);
    }
    __syncthreads();
    for (int w = tid; w < JT * Rn1; w += 256) {
      const int jj = w / Rn1, s = w - jj * Rn1;
      TC v[RM];
      if (j0 + jj < J) {
        subchain_row<TC, RM>(g, cv, idx + jj * MAXN, s, v);
      } else {
#pragma unroll
        for (int r = 0; r < RM; ++r) v[r] = TC(0);
      }
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (r < Rn) Bt[jj * (d + 1) + r + Rn * s] = (double)v[r];
    }
  }
  __syncthreads();
  const int nks = (d + 3) >> 2;
  const int64_t ntt = (T + 15) >> 4;
  double err = 0.0, nrm = 0.0;
  for (int64_t tt = wave; tt < ntt; tt += 4) {
    const int64_t t = tt * 16 + l16;
    const int64_t tc = t < T ? t : T - 1;
    const double* __restrict__ gcol = GNs + tc * d;
    d4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < nks; k0 += 8) {
      double av[8], bv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = (k0 + q) * 4 + g4;
        const bool ok = k < d && k0 + q < nks;
        const int kc = k < d ? k : d - 1;
        const double b = gcol[kc];
        av[q] = ok ? Bt[l16 * (d + 1) + kc] : 0.0;
        bv[q] = ok && t < T ? b : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc = mfma16(av[q], bv[q], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jr = Acc<double>::row(lane, v);
      const int64_t j = j0 + jr;
      if (j < J && t < T) {
        const double x = (double)X[j + J * t];
        const double e = x - acc[v];
        err += e * e;
        nrm += x * x;
      }
    }
  }
  red[0][tid] = err;
  red[1][tid] = nrm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    wg_out[2 * blockIdx.x] = red[0][0];
    wg_out[2 * blockIdx.x + 1] = red[1][0];
  }
}

int recon_err_blocks(const Geom& g) { return (int)((g.L + RECON_JT - 1) / RECON_JT); }

template <typename TX, typename TC>
static hipError_t launch_recon_t(const Geom& g, const void* X, const CoreView& cv,
                                 const double* GNs, double* wg_out, int* nwg, hipStream_t st) {
  const int blocks = recon_err_blocks(g);
  const size_t lds =
      (size_t)RECON_JT * (g.d + 1) * sizeof(double) + (size_t)RECON_JT * MAXN * sizeof(int);
  int rmax = 1;
  for (int k = 0; k < g.N; ++k) rmax = g.R[k] > rmax ? g.R[k] : rmax;
  if (rmax <= 8)
    hipLaunchKernelGGL((k_recon_err<TX, TC, 8>), dim3(blocks), dim3(256), lds, st, g,
                       (const TX*)X, cv, GNs, wg_out);
  else
    hipLaunchKernelGGL((k_recon_err<TX, TC, 16>), dim3(blocks), dim3(256), lds, st, g,
                       (const TX*)X, cv, GNs, wg_out);
  *nwg = blocks;
  return hipGetLastError();
}

hipError_t launch_recon_err(const Geom& g, const void* X, int xdt, const CoreView& cv, int cdt,
                            const double* GNs, double* wg_out, int* nwg, hipStream_t st) {
  if (g.In <= 0 || g.L <= 0 || !GNs) return hipErrorInvalidValue;
  if (xdt == F64 && cdt == F64)
    return launch_recon_t<double, double>(g, X, cv, GNs, wg_out, nwg, st);
  if (xdt == F32 && cdt == F32)
    return launch_recon_t<float, float>(g, X, cv, GNs, wg_out, nwg, st);
  if (xdt == F32 && cdt == F64)
    return launch_recon_t<float, double>(g, X, cv, GNs, wg_out, nwg, st);
  return hipErrorInvalidValue;
}

__global__ void k_sum_pairs(const double* __restrict__ w, int n, double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < n; i += 256) {
    a += w[2 * i];
    b += w[2 * i + 1];
  }
  red[0][tid] = a;
  red[1][tid] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

hipError_t launch_sum_pairs(const double* wg_out, int nwg, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, st, wg_out, nwg, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fit-loss gradient assembly: out = scale * (G_(2) Q - P) in the caller's
// core layout (strides sr, si, ss) and dtype.  Workgroup: 16 rows i x 64
// columns; the 16 rows of G_(2) are staged in LDS (FP64), the product with
// Q runs on FP64 16x16x4 MFMAs (wave w: columns 16w..16w+15 of the block,
// 8 k-steps of Q loads in flight), P is subtracted from the accumulators.
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_grad_combine(const TC* __restrict__ G, int64_t sr,
                                                      int64_t si, int64_t ss, int64_t In,
                                                      int Ra, int Rb,
                                                      const double* __restrict__ Q,
                                                      const double* __restrict__ P,
                                                      double scale, TC* __restrict__ out) {
  extern __shared__ double Gs[];                       // [16][d + 1]
  const int d = Ra * Rb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g4 = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 16;
  for (int e = tid; e < 16 * d; e += 256) {
    const int ii = e / d, c = e - ii * d;
    const int r = c % Ra, q = c / Ra;
    const int64_t i = i0 + ii;
    Gs[ii * (d + 1) + c] = i < In ? (double)G[r * sr + i * si + q * ss] : 0.0;
  }
  __syncthreads();
  const int c2 = blockIdx.y * 64 + wave * 16 + l16;
  if (blockIdx.y * 64 + wave * 16 >= d) return;
  const int c2c = c2 < d ? c2 : d - 1;
  const int nks = (d + 3) >> 2;
  // four accumulators taking turns (independent MFMA chains), added in a
  // fixed order at the end
  d4 ac[4] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}, d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
  for (int k0 = 0; k0 < nks; k0 += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = (k0 + q) * 4 + g4;
      const bool ok = k < d && k0 + q < nks;
      const int kc = k < d ? k : d - 1;
      const double b = Q[(size_t)kc * d + c2c];
      av[q] = ok ? Gs[l16 * (d + 1) + kc] : 0.0;
      bv[q] = ok ? b : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) ac[q & 3] = mfma16(av[q], bv[q], ac[q & 3]);
  }
  const d4 acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
  if (c2 >= d) return;
  const int r2 = c2 % Ra, q2 = c2 / Ra;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t i = i0 + Acc<double>::row(lane, v);
    if (i < In) out[r2 * sr + i * si + q2 * ss] = (TC)(scale * (acc[v] - P[i * d + c2]));
  }
}

hipError_t launch_grad_combine(const void* Gsrc, int cdt, int64_t sr, int64_t si, int64_t ss,
                               int64_t In, int Ra, int Rb, const double* Q, const double* P,
                               double scale, void* out, hipStream_t st) {
  const int d = Ra * Rb;
  if (In <= 0 || d <= 0 || d > 256) return hipErrorInvalidValue;
  dim3 grid((unsigned)((In + 15) / 16), (unsigned)((d + 63) / 64));
  const size_t lds = (size_t)16 * (d + 1) * sizeof(double);
  if (cdt == F64)
    hipLaunchKernelGGL(k_grad_combine<double>, grid, dim3(256), lds, st, (const double*)Gsrc, sr,
                       si, ss, In, Ra, Rb, Q, P, scale, (double*)out);
  else
    hipLaunchKernelGGL(k_grad_combine<float>, grid, dim3(256), lds, st, (const float*)Gsrc, sr, si,
                       ss, In, Ra, Rb, Q, P, scale, (float*)out);
  return hipGetLastError();
}

__global__ void k_core_to_slices(const void* src, int cdt, int64_t sr, int64_t si, int64_t ss,
                                 int64_t I, int Ra, int Rb, double* dst) {
  const int d = Ra * Rb;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= I * d) return;
  const int64_t i = e / d;
  const int c = (int)(e - i * d);
  const int r = c % Ra, s = c / Ra;
  const int64_t off = r * sr + i * si + s * ss;
  dst[e] = cdt == F64 ? ((const double*)src)[off] : (double)((const float*)src)[off];
}

hipError_t launch_core_to_slices(const void* src, int cdt, int64_t sr, int64_t si, int64_t ss,
                                 int64_t I, int Ra, int Rb, double* dst, hipStream_t st) {
  const int64_t n = I * Ra * Rb;
  hipLaunchKernelGGL(k_core_to_slices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     cdt, sr, si, ss, I, Ra, Rb, dst);
  return hipGetLastError();
}

}  // namespace trk
