// Internal declarations shared by the kernel and runtime translation units
// of the gfx950 streaming tensor-ring library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trk {

constexpr int MAXN = 8;     // maximum tensor order
constexpr int RMAXC = 16;   // maximum TR-rank
constexpr int KC = 32;      // K columns staged per MTTKRP chunk

// Strided view of N TR-cores: element (r, i, s) of core k (r < R_k,
// i < I_k, s < R_{k+1}) sits at ptr[k] + r*sr[k] + i*si[k] + s*ss[k].
struct CoreView {
  const void* ptr[MAXN];
  int64_t sr[MAXN], si[MAXN], ss[MAXN];
};

// Geometry of one mode-n product: X has dims I[0..N-1] (column-major),
// R[k] = R_k, R_{N} == R_0.  For mode n the columns of X_[n] are split as
// k = l + L*rr with l = lin(i_0..i_{n-1}) and rr = lin(i_{n+1}..i_{N-1}).
struct Geom {
  int N, n;
  int64_t I[MAXN];
  int R[MAXN];
  int64_t L, In, Rr;
  int d;            // R_n * R_{n+1}
};

Geom make_geom(int N, const int64_t* I, const int* R, int n);

enum DType { F64 = 0, F32 = 1, BF16 = 2 };

// Work decomposition of one mode-n product.  The columns of X_[n] are
// enumerated as (outer o, fast index i_f): f is the fastest-varying mode
// other than n (f = 0 for n >= 1, f = 1 for n = 0), and o runs over all
// remaining indices.  Workgroup (chunk, mtile) owns rows [16 mtile, +16)
// and the outer indices [chunk*upw, (chunk+1)*upw).
struct MttkrpPlan {
  int MT;          // rows per tile (16); rows per workgroup when zform (16, 32, 64)
  int mtiles;      // ceil(In / 16)
  int nsplit;      // number of outer-index chunks (partials)
  int psize;       // bytes per partial element (8 f64 path, 4 f32 path)
  int f;           // fast mode
  int nbf;         // 16-column tiles of R_f R_{f+1}
  int KS;          // waves splitting K = I_f (4, 2 or 1)
  int Q;           // consecutive i_f per lane group
  int64_t Kout;    // number of outer indices
  int64_t upw;     // outer indices per workgroup
  int64_t sf, sm;  // X strides of i_f and of the row index i_n
  int prv;         // 1: order-3 temporal MTTKRP in mode 1's GEMM geometry (rows
                   // i_1, outer index t) with the row-dependent slice G_1(i_1)
                   // applied per row; partial = row tile, output row = t
  int prv_in;      // output rows when prv (the batch's slices)
  int ng;          // fused launch: groups of four waves per workgroup, each
                   // taking one outer index of a pair at a time (1 or 2)
  int zform;       // 1: subchain blocks formed per outer index in LDS (FP32,
                   // order <= 4, ranks <= 16, I_f <= 64; MT rows per workgroup)
};

// max_wg > 0 caps the workgroup count (nsplit * mtiles) at about max_wg.
// bulk: allow the formed-subchain kernel for FP32 operands over many outer
// indices (FP32 accumulation across the chunk).
MttkrpPlan plan_mttkrp(const Geom& g, int xdtype, int max_wg = 0, bool bulk = false);
size_t mttkrp_partial_bytes(const Geom& g, const MttkrpPlan& p);

// ---- launchers (all asynchronous on `st`) --------------------------------

// Partials part[split][m][c] of X_[n] * G^{!=n}_[2] for the cores in cv
// (core dtype cdt: F64 or F32), X of dtype xdt.
hipError_t launch_mttkrp(const Geom& g, const MttkrpPlan& p, const void* X, int xdt,
                         const CoreView& cv, int cdt, void* part, hipStream_t st);

// Sum the split partials (fixed order) into rows; optionally accumulate into
// and store P; optionally multiply by Minv (d x d) and write rows of
// out (FP64), and with out32 also an FP32 copy of them.
hipError_t launch_reduce_solve(const void* part, int psize, int nsplit, int64_t In, int d,
                               double* P, int accumulate, const double* Minv,
                               double* out, hipStream_t st, float* out32 = nullptr);

// E_k[(a + Ra*a'), (b + Rb*b')] = sum_i G(i)[a,b] G(i)[a',b'] for rows
// i in [0, rows) of a slice-major FP64 core (slice i at G + i*Ra*Rb).
hipError_t launch_gram_E(const double* G, int64_t rows, int Ra, int Rb, double* E,
                         hipStream_t st);

// E (transfer layout) of a Gram tensor Z in the paper's R_{k+1} x R_k x
// R_{k+1} x R_k column-major layout (R = R_k, R1 = R_{k+1}).
hipError_t launch_z_to_E(const double* Z, int R, int R1, double* E, hipStream_t st);

// C (d1 x d3) = A (d1 x d2) * B (d2 x d3), row-major FP64.
hipError_t launch_matmul(const double* A, const double* B, double* C, int d1, int d2, int d3,
                         hipStream_t st);

// Q-layout matrix from an E-layout chain product M (rows (s + Rb*s'),
// columns (r + Ra*r')), optionally added to / stored in Q, then optionally
// inverted in place by Gauss-Jordan into Qinv.  A non-positive or tiny
// pivot sends the workgroup to the pseudo-inverse fallback.
// With m_plain = 1, M is already a d x d matrix in the Q layout.
// Q (+)= the Q-layout image of the Gram-chain product M (Rb^2 x Ra^2),
// no inverse.
hipError_t launch_assemble_q(const double* M, int Ra, int Rb, double* Q, int accumulate,
                             hipStream_t st);
// When a pivot fails, Qinv receives the pseudo-inverse instead (one-sided
// Jacobi from the stored Q; scratch `work` of 2 d^2 + d doubles); without a
// stored Q or work, status[0] is set to 1.
hipError_t launch_invert_spd(const double* M, int Ra, int Rb, double* Q, int accumulate,
                             int store_Q, double* Qinv, int* status, hipStream_t st,
                             int m_plain = 0, double* work = nullptr);

// Fused per-mode side step (workgroups of 1024 threads): optionally the
// transfer-layout Gram E_p of `rows_p` slice-major rows Gp (written to Ep,
// one workgroup per upper-triangle 16x16 tile; the last to finish goes on),
// then the ring product of the nfac transfer-layout factors fac[0..nfac)
// (fac[j] is fr[j] x fc[j]; a null entry stands for Ep), then the Q-layout
// assembly / accumulation into Q and the Gauss-Jordan inverse into Qinv
// (the pseudo-inverse of the stored Q when a pivot fails its test and pw is
// given: callers that do not keep Q pass a scratch Q with accumulate = 0).
// With row weights Gw (rows_p of them) the Gram is sum_s Gw[s] Gp_s^T Gp_s
// (the weighted sketched Gram, with Rpa = d and Rpb = 1).
struct SideArgs {
  const double* Gp;
  const double* Gw;
  int64_t rows_p;
  int Rpa, Rpb;
  double* Ep;
  int nfac;
  const double* fac[MAXN];
  int fr[MAXN], fc[MAXN];
  double* cbuf[2];
  int Ra, Rb;
  double* Q;
  int accumulate, store_Q;
  double* Qinv;
  int* status;         // [0] failure flag, [2] fallback count, [3] this solve fell back
  unsigned* counter;   // arrival counter of the Gram workgroups (zero between launches)
  double* pw;          // 2 d^2 + d doubles of scratch for the pseudo-inverse fallback
  // k_mode, two-factor chains (order 3) with R_p = 8: the Gram workgroups
  // also form the chain product's columns that their tile determines, so the
  // side step starts from the finished product (cbuf[0])
  int mcols;
  // Sketched product tiles beside the Gram tiles (k_side_mf; none when Pout
  // is null): Pout[i * d + c] = sum_s Gw[s] X[xoff(s) + i * xsn] Gp[s * d + c]
  // over the rows_p samples for i < pIn, in FP64, with
  // xoff(s) = sum_{q != xn} idxs[q * im + s] * xstride[q] over the xN modes.
  double* Pout;
  const void* Xs;
  int xdt, xN, xn, im;
  const int* idxs;
  int64_t pIn, xsn;
  int64_t xstride[MAXN];
};
hipError_t launch_side(const SideArgs& a, hipStream_t st);

// One mode in one launch: the side step of `sa` in workgroup 0 (4 waves)
// beside the MTTKRP of (g, p) in the other workgroups.  Valid when
// mode_fusable (R_nR_{n+1} <= 64 for the mode and its side step); state
// cores in FP64.
bool mode_fusable(const Geom& g, const SideArgs& sa);
// MTTKRP plan of the fused launch on a device with ncu compute units.
MttkrpPlan plan_mode(const Geom& g, int xdtype, const SideArgs& sa, int ncu);
hipError_t launch_mode(const Geom& g, const MttkrpPlan& p, const void* X, int xdt,
                       const CoreView& cv, int cdt, void* part, const SideArgs& sa,
                       hipStream_t st);

// Elementwise dtype conversion of n elements (round to nearest even).
hipError_t launch_cast(const void* src, int sdt, void* dst, int ddt, int64_t n, hipStream_t st);

// Per-workgroup sums of (X - Xhat)^2 and X^2 over a tensor whose last mode
// has T slices, with Xhat from the cores in cv (temporal core slices are
// the T rows of core N-1); GNs is the temporal core as slice-major FP64
// rows (GNs[t * d + r + R_{N-1} s] = G_{N-1}[r, t, s]); writes nwg pairs
// into wg_out and returns nwg.
hipError_t launch_recon_err(const Geom& gN, const void* X, int xdt, const CoreView& cv,
                            int cdt, const double* GNs, double* wg_out, int* nwg_out,
                            hipStream_t st);
// Sum of squared residuals and of X^2 for FP32 data and cores through the
// formed-subchain blocks (orders <= 4, ranks <= 16, I_f <= 64): one pair per
// workgroup into wg_out (at most max_wg pairs).  hipErrorNotSupported when
// the shape does not qualify (nothing launched).
hipError_t launch_recon_z(const Geom& g, const float* X, const CoreView& cv, double* wg_out,
                          int max_wg, int* nwg, hipStream_t st);
int recon_err_blocks(const Geom& gN);

// out[0..1] = fixed-order sums of the pairs in wg_out.
hipError_t launch_sum_pairs(const double* wg_out, int nwg, double* out, hipStream_t st);

// y[i] = alpha * y[i] + beta * x[i] for FP64 vectors (small helpers).
hipError_t launch_fill(double* y, double v, int64_t n, hipStream_t st);

// Finite check: flag[0] = 1 if any of the n elements is NaN/Inf.
hipError_t launch_check_finite(const void* x, int dt, int64_t n, int* flag, hipStream_t st);

// grads for the fit loss: out = scale * (G_(2) Q - P), written in the
// core layout of view cv entry n with dtype cdt.
hipError_t launch_grad_combine(const void* Gsrc, int cdt, int64_t sr, int64_t si, int64_t ss,
                               int64_t In, int Ra, int Rb, const double* Q, const double* P,
                               double scale, void* out, hipStream_t st);

// Copy a strided core into slice-major FP64 rows and back.
hipError_t launch_core_to_slices(const void* src, int cdt, int64_t sr, int64_t si, int64_t ss,
                                 int64_t I, int Ra, int Rb, double* dst, hipStream_t st);

// ---- randomized variant (sketch.hip) --------------------------------------

uint64_t rng_key(uint64_t seed, uint64_t step, uint64_t core, uint64_t kind);

// Initial core (Ra x I x Rb) from the stream `key` (Irwin-Hall normals),
// as slice-major FP64 rows.
hipError_t launch_init_normal(uint64_t key, int Ra, int64_t I, int Rb, double* G,
                              hipStream_t st);

// m uniform draws over [I] / from the distribution p (cdf: I doubles of
// scratch) into idx.
hipError_t launch_draw_uniform(uint64_t key, int m, int64_t I, int* idx, hipStream_t st);
hipError_t launch_draw_dist(uint64_t key, int m, int64_t I, const double* p, double* cdf,
                            int* idx, hipStream_t st);

// Leverage distribution of I slice-major rows of width d.  With K null,
// Zinv is the (pseudo-)inverse of the column Gram G^T G (I > d) and
// l_i = g_i Zinv g_i^T.  With K given (the row Gram G G^T, I <= d) and its
// (pseudo-)inverse in Zinv, every score is 1 unless *fell_back (the
// inverse was the pseudo-inverse: rank below I), when l_i = (K Zinv)_ii.
// p = l / sum(l), or uniform when every score is zero.
hipError_t launch_leverage(const double* G, int64_t I, int d, const double* Zinv,
                           const double* K, const int* fell_back, double* p, hipStream_t st);

// Sampled subchain rows A (m x d) of mode g.n and their weights w; idxs is
// N x m (row q = samples of core q); probs (device array of N device
// pointers) selects leverage weights, else every weight is wconst.
hipError_t launch_sample_rows(const Geom& g, const CoreView& cv, const int* idxs, int m,
                              const double* const* probs, double wconst, double* A, double* w,
                              hipStream_t st);

struct SketchPlan {
  int MT, mtiles, nsplit, cpw, psize;
};
SketchPlan plan_sketch(const Geom& g, int m, int xdtype);

// part[split][i][c] = sum_s X_S[i][s] w[s] A[s][c] over the split's samples.
hipError_t launch_sketch_gemm(const Geom& g, const SketchPlan& p, const void* X, int xdt,
                              const int* idxs, int m, const double* A, const double* w,
                              void* part, hipStream_t st);

// out = A^T diag(w) A (d x d, plain layout); w may be nullptr.
hipError_t launch_wgram(const double* A, const double* w, int64_t rows, int d, double* out,
                        hipStream_t st);
// K = G G^T for I slice-major rows of width d.
hipError_t launch_row_gram(const double* G, int64_t I, int d, double* K, hipStream_t st);

// ---- KSRFT-sketched variant (ksrft.hip) ------------------------------------

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ inline uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// n random signs (+1 / -1, FP64) of the stream `key`.
hipError_t launch_signs(uint64_t key, int64_t n, double* out, hipStream_t st);
// The signs of up to MAXN streams in one launch (stream k: n[k] signs of
// key[k] into out[k]).
struct SignsAll {
  uint64_t key[MAXN];
  int64_t n[MAXN];
  double* out[MAXN];
  int count;
};
hipError_t launch_signs_all(const SignsAll& a, hipStream_t st);

// Mixing matrix of one mode (2I x mix_k_padded(I, pin), row-major, dtype
// cdt) for a real (pin = 1) or complex (pin = 2, stacked planes) input.
int mix_k_padded(int64_t I, int pin);
hipError_t launch_mix_weights(int64_t I, int pin, const double* D, int cdt, void* W,
                              hipStream_t st);
// The mixing matrices of up to MAXN modes in one launch (mode k into W[k]).
struct MixWeightsAll {
  int64_t I[MAXN];
  int pin[MAXN];
  const double* D[MAXN];
  void* W[MAXN];
  int count;
};
hipError_t launch_mix_weights_all(const MixWeightsAll& a, int cdt, hipStream_t st);
// out (2 planes, dtype F64 for cdt F64, else F32) = W applied along a mode
// of stride S and size I (C = product of the slower modes) of `in` (pin
// planes of dtype idt, plane strides ips / ops elements).
hipError_t launch_mix_mode(const void* in, int idt, int pin, int64_t ips, void* out,
                           int64_t ops, int64_t S, int64_t I, int64_t C, const void* W, int cdt,
                           hipStream_t st);
// GS (2 planes of m x d) = sampled rows idx of the mixed core (F D) G.
hipError_t launch_mix_slices(const double* G, int64_t I, int d, const double* D, const int* idx,
                             int m, double* GS, hipStream_t st);
// The sampled mixed slices of up to MAXN cores in one launch (core k: I[k]
// slice-major rows of width d[k], at most 448 rows; m samples each).
struct MixSlicesAll {
  const double* G[MAXN];
  const double* D[MAXN];
  const int* idx[MAXN];
  double* GS[MAXN];
  int I[MAXN], d[MAXN];
  int m, count;
};
hipError_t launch_mix_slices_all(const MixSlicesAll& a, hipStream_t st);
// Complex sampled subchain rows of mode g.n from the sampled mixed slices
// GS (device array of N pointers): Ast (2m x d), Bst (2m x 2d), w2 (2m).
hipError_t launch_sample_rows_c(const Geom& g, const double* const* GS, int m, double w,
                                int literal, double* Ast, double* Bst, double* w2,
                                hipStream_t st);

struct SgemmPlan {
  int MT, mtiles, nsplit, kchunks, psize, nblk;
};
SgemmPlan plan_sgemm(const Geom& g, int m, int dB, int cdt);
// part[split][i][c] = sum_k Xg[i][k] B[k][c] over stacked planes (see ksrft.hip).
hipError_t launch_sgemm(const Geom& g, const SgemmPlan& p, int dB, int64_t pstride,
                        const void* X, int cdt, const int* idxs, int m, const double* B,
                        void* part, hipStream_t st);
// dP (I x d) = Re(D F^* Z) for Z = [Re | Im] (I x 2d).
hipError_t launch_unmix(const double* Z, int64_t I, int d, const double* D, double* dP,
                        hipStream_t st);

}  // namespace trk
