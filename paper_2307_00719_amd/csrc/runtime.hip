// Host runtime and C ABI of the gfx950 streaming tensor-ring tracker.
//
// The handle keeps the streaming state of Alg. 4 on the device in FP64:
//   G[k]   cores k < N-1 as slice-major rows (row i = G_{k(2)}[i, :], the
//          column index r + R_k*s of Sec. 2's mode-2 unfolding);
//   G[N-1] the temporal core, all slices seen so far (capacity `cap`);
//   E[k]   Gram matrices of the cores in transfer layout (Z_k of Alg. 4);
//   E[N-1] the Gram matrix of the newest temporal rows (Z_N^new);
//   P[n], Q[n] the complementary matrices of Sec. 3.1 (row-major).
// One time step (Alg. 4, update stage) is, per mode: the Gram chain and
// the inverse of the normal-equation matrix, the MTTKRP-like product split
// over K, the fixed-order split reduction fused with P += and the solve,
// and the Gram refresh of the updated core.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tr_internal.h"
#include "tr_stream.h"

using namespace trk;

struct tr_stream {
  int N = 0;
  int64_t I[MAXN] = {};  // I[0..N-2]; I[N-1] is the current batch size when used
  int R[MAXN] = {};
  int dt = F64;
  int sketch = 0;
  int64_t m = 0;
  int rescale = 1, temporal_literal = 1, check_finite = 0;
  int sweeps = 1;               // passes of the update stage over each batch
  uint64_t seed = 0;
  int device = 0;
  int ncu = 0;                  // compute units of the device
  hipStream_t st = nullptr;
  bool own_stream = false;
  int64_t t_total = 0, cap = 0;
  int64_t last_t = 0;           // slices of the newest temporal block (init or last batch)
  double* G[MAXN] = {};
  double* E[MAXN] = {};
  double* P[MAXN] = {};
  double* Q[MAXN] = {};
  double* Minv = nullptr;
  double* MinvM[MAXN] = {};    // per-mode inverses (two-stream STR update)
  double* Pold[MAXN] = {};     // P_n, Q_n before the batch (multi-pass updates)
  double* Qold[MAXN] = {};
  double* pinvH = nullptr;     // matrix copy and scratch of the pseudo-inverse fallback
  double* pinvW = nullptr;
  int32_t init_sweeps = 0;     // batch TR-ALS sweeps run by the initialiser
  double init_err = 0.0;       // its final relative error
  std::vector<double> next_signs;  // injected D_k of the next step (KSRFT)
  int64_t next_signs_t = 0;
  double* chain[2] = {};
  unsigned* sidecnt = nullptr;  // arrival counter of the side kernel's Gram workgroups
  hipStream_t side = nullptr;  // second stream: Gram refresh, chain, inverse
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_inv[MAXN] = {}, ev_rs[MAXN] = {};  // MTTKRP done (main), solve done (side)
  void* xcast = nullptr;
  size_t xcast_bytes = 0;
  double* xf64 = nullptr;
  size_t xf64_bytes = 0;
  void* part = nullptr;
  size_t part_bytes = 0;
  // FP32 copies of the cores (k < N-1) and of the new temporal rows (N-1)
  // for the formed-subchain MTTKRP of the FP32-operand two-stream update
  void* G32[MAXN] = {};
  size_t G32_bytes[MAXN] = {};
  double* wg = nullptr;
  size_t wg_n = 0;
  double* pair = nullptr;
  int* dstatus = nullptr;
  double* hpinned = nullptr;
  size_t hpinned_bytes = 0;
  hipEvent_t copy_done = nullptr;
  bool copy_pending = false;
  std::string err;
  tr_status poisoned = TR_OK;
  // randomized variant state (rSTR-U / rSTR-L)
  int64_t step = 0;          // time step counter (0 = initialisation)
  int* idxs = nullptr;       // N x m sample indices
  double* probs[MAXN] = {};  // leverage distributions (temporal: newest rows)
  int64_t probs_cap_t = 0;
  double** dprobs = nullptr; // device copy of probs[]
  double* cdf = nullptr;
  int64_t cdf_cap = 0;
  double* SA = nullptr;      // m x dmax sampled subchain rows
  double* Sw = nullptr;      // m weights
  double* Zb = nullptr;      // dmax^2 (or I^2 <= 256^2) scratch Gram
  double* Zi = nullptr;      // its inverse
  // KSRFT state (rSTR-K)
  double* dsign[MAXN] = {};  // diagonal of D_k (temporal: ksign_cap entries)
  int64_t ksign_cap = 0;
  double* GSc[MAXN] = {};    // sampled mixed slices: 2 planes of m x d_k
  double** dGSc = nullptr;   // device copy of GSc[]
  double* Ast = nullptr;     // [Re A; Im A], 2m x dmax
  double* Bst = nullptr;     // product operand, 2m x 2 dmax
  double* Sw2 = nullptr;     // 2m weights
  void* Wmix = nullptr;      // mixing matrices of all modes
  size_t Wmix_bytes = 0;
  void* xh[2] = {};          // mixed batch, 2 planes (ping-pong)
  size_t xh_bytes[2] = {};
  double* Zk = nullptr;      // reduced sketched product, I x 2d
  size_t Zk_bytes = 0;
  double* dPk = nullptr;     // unmixed increment, I x d
  size_t dPk_bytes = 0;
  // event profiling (tr_stream_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> rec_kind;
  std::vector<size_t> rec_ev;

  int d(int k) const { return R[k] * R[(k + 1) % N]; }
};

namespace {

tr_status fail(tr_stream* s, tr_status code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

tr_status poison(tr_stream* s, tr_status code, const std::string& msg) {
  s->err = msg;
  s->poisoned = TR_ERR_STATE;
  return code;
}

#define TR_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return poison(s, TR_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

hipError_t ensure(void** p, size_t* have, size_t need) {
  if (need <= *have && *p) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  size_t n = std::max(need, (size_t)256);
  hipError_t e = hipMalloc(p, n);
  if (e == hipSuccess) *have = n;
  return e;
}

CoreView state_view(const tr_stream* s, const double* temporal) {
  CoreView v;
  for (int k = 0; k < MAXN; ++k) {
    v.ptr[k] = nullptr;
    v.sr[k] = v.si[k] = v.ss[k] = 0;
  }
  for (int k = 0; k < s->N; ++k) {
    v.ptr[k] = (k == s->N - 1) ? (const void*)temporal : (const void*)s->G[k];
    v.sr[k] = 1;
    v.si[k] = s->d(k);
    v.ss[k] = s->R[k];
  }
  return v;
}

CoreView colmajor_view(int N, const int64_t* dims, const int* R, const void* const* cores) {
  CoreView v;
  for (int k = 0; k < MAXN; ++k) {
    v.ptr[k] = nullptr;
    v.sr[k] = v.si[k] = v.ss[k] = 0;
  }
  for (int k = 0; k < N; ++k) {
    v.ptr[k] = cores[k];
    v.sr[k] = 1;
    v.si[k] = R[k];
    v.ss[k] = (int64_t)R[k] * dims[k];
  }
  return v;
}

// Product of the transfer-layout Gram matrices E_{n+1} ... E_{n-1} in ring
// order (the Gram chain of Alg. 4 / Prop. subchain Gram), with `temporal`
// standing for the temporal factor.  Returns the device pointer holding
// the R_{n+1}^2 x R_n^2 product.
const double* chain_product(tr_stream* s, int n, const double* temporal, hipError_t* err,
                            hipStream_t on = nullptr) {
  if (!on) on = s->st;
  const int N = s->N;
  std::vector<int> order;
  for (int j = 1; j < N; ++j) order.push_back((n + j) % N);
  auto fac = [&](int q) -> const double* { return q == N - 1 ? temporal : s->E[q]; };
  const double* cur = fac(order[0]);
  int rows = s->R[order[0]] * s->R[order[0]];
  int cols = s->R[(order[0] + 1) % N] * s->R[(order[0] + 1) % N];
  int pp = 0;
  *err = hipSuccess;
  for (size_t j = 1; j < order.size(); ++j) {
    const int q = order[j];
    const int c2 = s->R[(q + 1) % N] * s->R[(q + 1) % N];
    *err = launch_matmul(cur, fac(q), s->chain[pp], rows, cols, c2, on);
    if (*err != hipSuccess) return nullptr;
    cur = s->chain[pp];
    pp ^= 1;
    cols = c2;
  }
  return cur;
}

int dtype_size(int dt) { return dt == F64 ? 8 : (dt == F32 ? 4 : 2); }

tr_status check_host_finite(tr_stream* s, const void* x, int dt, int64_t n) {
  if (dt == F64) {
    const double* p = (const double*)x;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(p[i])) return fail(s, TR_ERR_NONFINITE, "input holds NaN or Inf");
  } else if (dt == F32) {
    const float* p = (const float*)x;
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(p[i])) return fail(s, TR_ERR_NONFINITE, "input holds NaN or Inf");
  }
  return TR_OK;
}

// Brings a batch (host or device, any supported dtype) to the device in the
// compute dtype; returns the device pointer through *out.
tr_status stage_batch(tr_stream* s, const void* X, int xdt, int64_t n, int x_is_device,
                      const void** out) {
  const size_t bytes = (size_t)n * dtype_size(xdt);
  const void* dsrc = X;
  if (!x_is_device) {
    tr_status c = check_host_finite(s, X, xdt, n);
    if (c != TR_OK) return c;
    if (s->copy_pending) {
      TR_HIP(hipEventSynchronize(s->copy_done));
      s->copy_pending = false;
    }
    if (bytes > s->hpinned_bytes) {
      if (s->hpinned) TR_HIP(hipHostFree(s->hpinned));
      s->hpinned = nullptr;
      TR_HIP(hipHostMalloc((void**)&s->hpinned, bytes, hipHostMallocDefault));
      s->hpinned_bytes = bytes;
    }
    std::memcpy(s->hpinned, X, bytes);
    TR_HIP(ensure((void**)&s->xf64, &s->xf64_bytes, bytes));
    TR_HIP(hipMemcpyAsync(s->xf64, s->hpinned, bytes, hipMemcpyHostToDevice, s->st));
    TR_HIP(hipEventRecord(s->copy_done, s->st));
    s->copy_pending = true;
    dsrc = s->xf64;
  } else if (s->check_finite) {
    TR_HIP(hipMemsetAsync(s->dstatus + 1, 0, sizeof(int), s->st));
    TR_HIP(launch_check_finite(X, xdt, n, s->dstatus + 1, s->st));
    int flag = 0;
    TR_HIP(hipMemcpyAsync(&flag, s->dstatus + 1, sizeof(int), hipMemcpyDeviceToHost, s->st));
    TR_HIP(hipStreamSynchronize(s->st));
    if (flag) return fail(s, TR_ERR_NONFINITE, "input holds NaN or Inf");
  }
  if (xdt == s->dt) {
    *out = dsrc;
    return TR_OK;
  }
  TR_HIP(ensure(&s->xcast, &s->xcast_bytes, (size_t)n * dtype_size(s->dt)));
  TR_HIP(launch_cast(dsrc, xdt, s->xcast, s->dt, n, s->st));
  *out = s->xcast;
  return TR_OK;
}

// Workgroups of the formed-subchain MTTKRP in the two-stream update: the
// side kernel sets the pace, so the split is sized for about 3.3 MB of
// partials (fewer partials shorten the reduction after the side kernel),
// between 64 and 256 workgroups.
int stream_zwg(const Geom& g) {
  const int64_t w = (int64_t)3300000 / (g.In * g.d * 4);
  return (int)std::min<int64_t>(256, std::max<int64_t>(64, w));
}

tr_status ensure_partials(tr_stream* s, const Geom& g, const MttkrpPlan& p) {
  TR_HIP(ensure(&s->part, &s->part_bytes, mttkrp_partial_bytes(g, p)));
  return TR_OK;
}

tr_status grow_temporal(tr_stream* s, int64_t need) {
  if (need <= s->cap) return TR_OK;
  int64_t ncap = std::max(need, 2 * s->cap);
  const int dN = s->d(s->N - 1);
  double* nb = nullptr;
  TR_HIP(dev_alloc(&nb, (size_t)ncap * dN));
  TR_HIP(hipMemcpyAsync(nb, s->G[s->N - 1], (size_t)s->t_total * dN * sizeof(double),
                        hipMemcpyDeviceToDevice, s->st));
  TR_HIP(hipStreamSynchronize(s->st));
  TR_HIP(hipFree(s->G[s->N - 1]));
  s->G[s->N - 1] = nb;
  s->cap = ncap;
  return TR_OK;
}

enum { PK_MTT_T = 0, PK_MTT_N = 1, PK_CHAIN = 2, PK_SOLVE = 3, PK_GRAM = 4, PK_STEP = 5 };

// Starts a profiled region of `kind`; returns its record index or -1.
long prof_begin(tr_stream* s, int kind, hipStream_t on = nullptr) {
  if (!s->prof) return -1;
  if (!on) on = s->st;
  while (s->ev_used + 2 > s->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    s->ev_pool.push_back(e);
  }
  const size_t a = s->ev_used;
  s->ev_used += 2;
  if (hipEventRecord(s->ev_pool[a], on) != hipSuccess) return -1;
  s->rec_kind.push_back(kind);
  s->rec_ev.push_back(a);
  return (long)s->rec_kind.size() - 1;
}

void prof_end(tr_stream* s, long rec, hipStream_t on = nullptr) {
  if (rec < 0) return;
  (void)hipEventRecord(s->ev_pool[s->rec_ev[rec] + 1], on ? on : s->st);
}

// Device status words: [0] 1 = an elimination failed with no fallback
// scratch, 2 = a normal-equation matrix held NaN or Inf; [1] finite check
// of a device batch; [2] count of pseudo-inverse fallbacks; [3] whether the
// last solve fell back.
tr_status read_status(tr_stream* s) {
  int st[2] = {0, 0};
  TR_HIP(hipMemcpyAsync(st, s->dstatus, sizeof(int), hipMemcpyDeviceToHost, s->st));
  TR_HIP(hipStreamSynchronize(s->st));
  if (st[0] == 2) return poison(s, TR_ERR_NONFINITE, "a normal-equation matrix holds NaN or Inf");
  if (st[0]) return poison(s, TR_ERR_SINGULAR, "a normal-equation matrix was not positive definite");
  return TR_OK;
}

int64_t prod_dims_except(const tr_stream* s, int skip) {
  int64_t J = 1;
  for (int k = 0; k < s->N - 1; ++k)
    if (k != skip) J *= s->I[k];
  return J;
}

// Leverage distribution (Lemma on leverage estimation) of `rows` slice-major
// rows of core k into p.
// The sketched product P = X_S W A of mode g.n, formed beside the Gram of
// the same sampled rows A (weights W) by the side kernel (d <= 192).
struct SketchProduct {
  const Geom* g;
  const void* X;
  double* P;
};
tr_status gram_update_invert(tr_stream* s, hipStream_t on, double* M, int Ra, int Rb, double* Q,
                             int accumulate, double* Qinv, const double* A = nullptr,
                             const double* w = nullptr, int64_t rows = 0,
                             const SketchProduct* sp = nullptr);

tr_status leverage_probs(tr_stream* s, int k, const double* rows, int64_t I, double* p) {
  const int Ra = s->R[k], Rb = s->R[(k + 1) % s->N], d = Ra * Rb;
  if (I > d) {
    // G^T G of the rows and its inverse (one side kernel for d <= 192)
    tr_status c = gram_update_invert(s, s->st, s->Zb, Ra, Rb, nullptr, 0, s->Zi, rows, nullptr, I);
    if (c != TR_OK) return c;
    TR_HIP(launch_leverage(rows, I, d, s->Zi, nullptr, nullptr, p, s->st));
  } else {
    if (I > 256) return poison(s, TR_ERR_UNSUPPORTED, "leverage rank check needs I <= 256");
    // full row rank: the row Gram G G^T passes the positivity test of the
    // elimination (its inverse is not used); otherwise the elimination's
    // pseudo-inverse K^+ gives the scores diag(K K^+)
    TR_HIP(launch_row_gram(rows, I, d, s->Zb, s->st));
    tr_status c = gram_update_invert(s, s->st, s->Zb, (int)I, 1, nullptr, 0, s->Zi);
    if (c != TR_OK) return c;
    TR_HIP(launch_leverage(rows, I, d, s->Zi, s->Zb, s->dstatus + 3, p, s->st));
  }
  return TR_OK;
}

// idxs(:, k) <- Randsample over [size] (uniform, or from probs[k]).
tr_status draw_samples(tr_stream* s, int k, int64_t size) {
  const uint64_t key = rng_key(s->seed, (uint64_t)s->step, (uint64_t)k, 0);
  int* out = s->idxs + (size_t)k * s->m;
  if (s->sketch == TR_SKETCH_LEVERAGE) {
    if (size > s->cdf_cap) {
      if (s->cdf) TR_HIP(hipFree(s->cdf));
      TR_HIP(dev_alloc(&s->cdf, (size_t)size));
      s->cdf_cap = size;
    }
    TR_HIP(launch_draw_dist(key, (int)s->m, size, s->probs[k], s->cdf, out, s->st));
  } else {
    TR_HIP(launch_draw_uniform(key, (int)s->m, size, out, s->st));
  }
  return TR_OK;
}

tr_status ensure_temporal_probs(tr_stream* s, int64_t t) {
  if (s->sketch != TR_SKETCH_LEVERAGE || t <= s->probs_cap_t) return TR_OK;
  const int N = s->N;
  if (s->probs[N - 1]) {
    TR_HIP(hipStreamSynchronize(s->st));
    TR_HIP(hipFree(s->probs[N - 1]));
  }
  TR_HIP(dev_alloc(&s->probs[N - 1], (size_t)t));
  s->probs_cap_t = t;
  TR_HIP(hipMemcpyAsync(s->dprobs, s->probs, N * sizeof(double*), hipMemcpyHostToDevice, s->st));
  return TR_OK;
}

// Q (+)= M for a d x d Gram matrix M already in the Q layout and exactly
// symmetric (the sketched Grams), then Qinv = Q^{-1} when Qinv is given:
// the 16x16-pivot-block MFMA Gauss-Jordan of the side kernel (one
// workgroup of 16 waves, the Gram passed as a single ring-product factor
// with R_a = d, R_b = 1) for d <= 192, the scalar elimination beyond.
// With rows A (`rows` x d, row weights w, or weights 1 when w is null) the
// Gram M = sum_s w_s A_s^T A_s is formed first into M: for d <= 192 by the
// side kernel's own tile workgroups (the last to finish goes on with the
// inverse), else by the weighted-Gram kernel.  Launched on stream `on`.
tr_status gram_update_invert(tr_stream* s, hipStream_t on, double* M, int Ra, int Rb, double* Q,
                             int accumulate, double* Qinv, const double* A, const double* w,
                             int64_t rows, const SketchProduct* sp) {
  const int d = Ra * Rb;
  if (sp && (d > 192 || !A)) return poison(s, TR_ERR_UNSUPPORTED, "sketched product tiles");
  if (d <= 192) {
    SideArgs a;
    std::memset(&a, 0, sizeof(a));
    if (A) {
      a.Gp = A;
      a.Gw = w;
      a.rows_p = rows;
      a.Rpa = d;
      a.Rpb = 1;
      a.Ep = M;
    }
    if (sp) {
      const Geom& g = *sp->g;
      a.Pout = sp->P;
      a.Xs = sp->X;
      a.xdt = s->dt;
      a.xN = g.N;
      a.xn = g.n;
      a.im = (int)s->m;
      a.idxs = s->idxs;
      a.pIn = g.In;
      int64_t acc = 1;
      for (int q = 0; q < g.N; ++q) {
        a.xstride[q] = acc;
        acc *= g.I[q];
      }
      a.xsn = a.xstride[g.n];
    }
    a.nfac = 1;
    a.fac[0] = M;
    a.fr[0] = d;
    a.fc[0] = 1;
    a.cbuf[0] = s->chain[0];
    a.cbuf[1] = s->chain[1];
    a.Ra = d;
    a.Rb = 1;
    a.Q = Q ? Q : s->pinvH;          // the fallback's input is the stored matrix
    a.accumulate = Q ? accumulate : 0;
    a.store_Q = 1;
    a.Qinv = Qinv;
    a.status = s->dstatus;
    a.counter = s->sidecnt;
    a.pw = s->pinvW;
    TR_HIP(launch_side(a, on));
    return TR_OK;
  }
  if (A) TR_HIP(launch_wgram(A, w, rows, d, M, on));
  TR_HIP(launch_invert_spd(M, Ra, Rb, Q ? Q : s->pinvH, Q ? accumulate : 0, 1, Qinv, s->dstatus,
                           on, 1, s->pinvW));
  return TR_OK;
}

// The sketched Gram's Q update and inverse occupy one compute unit and are
// latency-bound, and the sketched product does not read what they write: in
// rSTR-K, whose mixed product, reduction and unmixing take less time than
// the inverse, the product chain goes to the second stream (fork) while the
// caller's stream runs the Gram and the inverse, and then waits for the
// product chain before the solve (join).  rSTR-U/L keep one stream: their
// product tiles ride in the side kernel itself.
tr_status fork_side(tr_stream* s) {
  TR_HIP(hipEventRecord(s->ev_fork, s->st));
  TR_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  return TR_OK;
}
tr_status join_side(tr_stream* s) {
  TR_HIP(hipEventRecord(s->ev_join, s->side));
  TR_HIP(hipStreamWaitEvent(s->st, s->ev_join, 0));
  return TR_OK;
}

// One sketched P/Q increment of mode n (Alg. 5: P_n += X_S G_S, Q_n += G_S^T G_S
// with the rescaling of the sketch), X of `t` slices, temporal rows Gt.
tr_status sketch_increment(tr_stream* s, int n, const void* Xd, int64_t t, const double* Gt,
                           int accumulate, const double* Minv_solve) {
  const int N = s->N;
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = t;
  Geom g = make_geom(N, gd.data(), s->R, n);
  const CoreView cv = state_view(s, Gt);
  const int m = (int)s->m;
  double wconst = 1.0;
  if (s->rescale) wconst = (double)prod_dims_except(s, n) * (double)t / (double)m;
  const bool lev = s->sketch == TR_SKETCH_LEVERAGE && s->rescale;
  TR_HIP(launch_sample_rows(g, cv, s->idxs, m, lev ? (const double* const*)s->dprobs : nullptr,
                            wconst, s->SA, s->Sw, s->st));
  if (g.d <= 192) {
    // the product's tiles ride in the side kernel beside the Gram
    TR_HIP(ensure(&s->part, &s->part_bytes, (size_t)g.In * g.d * 8));
    const SketchProduct spp = {&g, Xd, (double*)s->part};
    tr_status c = gram_update_invert(s, s->st, s->Zb, s->R[n], s->R[(n + 1) % N], s->Q[n],
                                     accumulate, Minv_solve ? s->Minv : nullptr, s->SA, s->Sw, m,
                                     &spp);
    if (c != TR_OK) return c;
    TR_HIP(launch_reduce_solve(s->part, 8, 1, g.In, g.d, s->P[n], accumulate,
                               Minv_solve ? s->Minv : nullptr, s->G[n], s->st));
    return TR_OK;
  }
  SketchPlan sp = plan_sketch(g, m, s->dt);
  const size_t pb = (size_t)sp.nsplit * g.In * g.d * sp.psize;
  TR_HIP(ensure(&s->part, &s->part_bytes, pb));
  tr_status c = gram_update_invert(s, s->st, s->Zb, s->R[n], s->R[(n + 1) % N], s->Q[n],
                                   accumulate, Minv_solve ? s->Minv : nullptr, s->SA, s->Sw, m);
  if (c != TR_OK) return c;
  TR_HIP(launch_sketch_gemm(g, sp, Xd, s->dt, s->idxs, m, s->SA, s->Sw, s->part, s->st));
  TR_HIP(launch_reduce_solve(s->part, sp.psize, sp.nsplit, g.In, g.d, s->P[n], accumulate,
                             Minv_solve ? s->Minv : nullptr, s->G[n], s->st));
  return TR_OK;
}

tr_status sketch_init(tr_stream* s, const void* Xd, int64_t t_init) {
  const int N = s->N;
  s->step = 0;
  if (s->sketch == TR_SKETCH_LEVERAGE) {
    tr_status c = ensure_temporal_probs(s, t_init);
    if (c != TR_OK) return c;
    for (int k = 0; k < N; ++k) {
      const int64_t I = k == N - 1 ? t_init : s->I[k];
      c = leverage_probs(s, k, s->G[k], I, s->probs[k]);
      if (c != TR_OK) return c;
    }
  }
  for (int k = 0; k < N; ++k) {
    tr_status c = draw_samples(s, k, k == N - 1 ? t_init : s->I[k]);
    if (c != TR_OK) return c;
  }
  for (int n = 0; n < N - 1; ++n) {
    tr_status c = sketch_increment(s, n, Xd, t_init, s->G[N - 1], 0, nullptr);
    if (c != TR_OK) return c;
  }
  return TR_OK;
}

// One time step of rSTR-U / rSTR-L (Alg. 7 / Alg. 8).
tr_status sketch_update(tr_stream* s, const void* Xd, int64_t t_new, double* Gnew) {
  const int N = s->N;
  s->step += 1;
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = t_new;
  const int m = (int)s->m;
  // temporal mode: G_N^new = (X_S D)((D G_S)^T)^+ through the normal equations
  {
    Geom g = make_geom(N, gd.data(), s->R, N - 1);
    const CoreView cv = state_view(s, Gnew);
    double wconst = 1.0;
    if (s->rescale) wconst = (double)prod_dims_except(s, -1) / (double)m;
    const bool lev = s->sketch == TR_SKETCH_LEVERAGE && s->rescale;
    TR_HIP(launch_sample_rows(g, cv, s->idxs, m, lev ? (const double* const*)s->dprobs : nullptr,
                              wconst, s->SA, s->Sw, s->st));
    if (g.d <= 192) {
      // the product's tiles ride in the side kernel beside the Gram
      TR_HIP(ensure(&s->part, &s->part_bytes, (size_t)g.In * g.d * 8));
      const SketchProduct spp = {&g, Xd, (double*)s->part};
      tr_status c0 = gram_update_invert(s, s->st, s->Zb, s->R[N - 1], s->R[0], nullptr, 0,
                                        s->Minv, s->SA, s->Sw, m, &spp);
      if (c0 != TR_OK) return c0;
      TR_HIP(launch_reduce_solve(s->part, 8, 1, g.In, g.d, nullptr, 0, s->Minv, Gnew, s->st));
    } else {
      SketchPlan sp = plan_sketch(g, m, s->dt);
      TR_HIP(ensure(&s->part, &s->part_bytes, (size_t)sp.nsplit * g.In * g.d * sp.psize));
      tr_status c0 = gram_update_invert(s, s->st, s->Zb, s->R[N - 1], s->R[0], nullptr, 0,
                                        s->Minv, s->SA, s->Sw, m);
      if (c0 != TR_OK) return c0;
      TR_HIP(launch_sketch_gemm(g, sp, Xd, s->dt, s->idxs, m, s->SA, s->Sw, s->part, s->st));
      TR_HIP(launch_reduce_solve(s->part, sp.psize, sp.nsplit, g.In, g.d, nullptr, 0, s->Minv,
                                 Gnew, s->st));
    }
  }
  tr_status c;
  if (s->sketch == TR_SKETCH_LEVERAGE) {
    c = ensure_temporal_probs(s, t_new);
    if (c != TR_OK) return c;
    c = leverage_probs(s, N - 1, Gnew, t_new, s->probs[N - 1]);
    if (c != TR_OK) return c;
  }
  c = draw_samples(s, N - 1, t_new);
  if (c != TR_OK) return c;
  for (int n = 0; n < N - 1; ++n) {
    c = sketch_increment(s, n, Xd, t_new, Gnew, 1, s->Minv);
    if (c != TR_OK) return c;
    if (s->sketch == TR_SKETCH_LEVERAGE) {
      c = leverage_probs(s, n, s->G[n], s->I[n], s->probs[n]);
      if (c != TR_OK) return c;
    }
    c = draw_samples(s, n, s->I[n]);
    if (c != TR_OK) return c;
  }
  return TR_OK;
}

// ---- rSTR-K (Alg. 9) --------------------------------------------------------

// D_k of the current step for every mode (the temporal one over t entries).
tr_status ksrft_signs(tr_stream* s, int64_t t) {
  const int N = s->N;
  if (t > s->ksign_cap) {
    if (s->dsign[N - 1]) {
      TR_HIP(hipStreamSynchronize(s->st));
      TR_HIP(hipFree(s->dsign[N - 1]));
    }
    TR_HIP(dev_alloc(&s->dsign[N - 1], (size_t)t));
    s->ksign_cap = t;
  }
  if (!s->next_signs.empty()) {
    // injected D_k (tr_stream_set_samples): checked against t by the update
    int64_t off = 0;
    for (int k = 0; k < N; ++k) {
      const int64_t n = k == N - 1 ? t : s->I[k];
      TR_HIP(hipMemcpyAsync(s->dsign[k], s->next_signs.data() + off, n * sizeof(double),
                            hipMemcpyHostToDevice, s->st));
      off += n;
    }
    TR_HIP(hipStreamSynchronize(s->st));
    s->next_signs.clear();
    s->next_signs_t = 0;
    return TR_OK;
  }
  SignsAll a = {};
  a.count = N;
  for (int k = 0; k < N; ++k) {
    a.key[k] = rng_key(s->seed, (uint64_t)s->step, (uint64_t)k, 1);
    a.n[k] = k == N - 1 ? t : s->I[k];
    a.out[k] = s->dsign[k];
  }
  TR_HIP(launch_signs_all(a, s->st));
  return TR_OK;
}

// Xhat = X x_1 (F_1 D_1) ... x_N (F_N D_N) (Alg. 6) of a batch of t slices in
// the compute dtype; *xhat receives the two planes (F64, or F32 for the F32
// and BF16 paths).
tr_status ksrft_mix(tr_stream* s, const void* Xd, int64_t t, const void** xhat) {
  const int N = s->N;
  std::vector<int64_t> dims(N);
  int64_t total = 1;
  for (int k = 0; k < N; ++k) {
    dims[k] = k == N - 1 ? t : s->I[k];
    total *= dims[k];
  }
  const size_t xs = s->dt == F64 ? 8 : 4;
  const size_t ws = s->dt == F64 ? 8 : (s->dt == F32 ? 4 : 2);
  for (int b = 0; b < 2; ++b) TR_HIP(ensure(&s->xh[b], &s->xh_bytes[b], 2 * (size_t)total * xs));
  // the mixing matrices of all modes (mode 0 acts on the real data, the
  // others on two planes), formed in one launch into consecutive slots
  MixWeightsAll wa = {};
  wa.count = N;
  size_t woff[MAXN], wneed = 0;
  for (int k = 0; k < N; ++k) {
    woff[k] = wneed;
    const int pk = k == 0 ? 1 : 2;
    wneed += ((size_t)2 * dims[k] * mix_k_padded(dims[k], pk) * ws + 255) / 256 * 256;
  }
  TR_HIP(ensure(&s->Wmix, &s->Wmix_bytes, wneed));
  for (int k = 0; k < N; ++k) {
    wa.I[k] = dims[k];
    wa.pin[k] = k == 0 ? 1 : 2;
    wa.D[k] = s->dsign[k];
    wa.W[k] = (char*)s->Wmix + woff[k];
  }
  TR_HIP(launch_mix_weights_all(wa, s->dt, s->st));
  const void* in = Xd;
  int idt = s->dt, pin = 1, cur = 0;
  int64_t S = 1;
  for (int k = 0; k < N; ++k) {
    const int64_t Ik = dims[k], C = total / (S * Ik);
    TR_HIP(launch_mix_mode(in, idt, pin, total, s->xh[cur], total, S, Ik, C, wa.W[k], s->dt,
                           s->st));
    in = s->xh[cur];
    idt = s->dt == F64 ? F64 : F32;
    pin = 2;
    cur ^= 1;
    S *= Ik;
  }
  *xhat = in;
  return TR_OK;
}

// Sampled mixed slices of core k: rows of (F_k D_k) G_k at idxs(:, k).
tr_status ksrft_slices(tr_stream* s, int k, const double* rows, int64_t I) {
  TR_HIP(launch_mix_slices(rows, I, s->d(k), s->dsign[k], s->idxs + (size_t)k * s->m, (int)s->m,
                           s->GSc[k], s->st));
  return TR_OK;
}

// One mode of Alg. 9: Re(Q_n) += Re(Ghat_S^T W conj(Ghat_S)) and
// Re(P_n) += Re(D_n F_n^* Xhat_S W conj(Ghat_S)), then G_n = Re(P_n) Re(Q_n)^-1
// when `solve`; for the temporal mode (n = N-1) the rows G_N^new are written
// to Gout: by default in the printed form Re(D F^* Xhat_S) (Re(Ghat_S)^T)^+
// (the KSRFT paragraph of Sec. 3.3, Alg. 9), or, with temporal_literal
// cleared, from the increments alone (real-constrained normal equations).
tr_status ksrft_increment(tr_stream* s, int n, const void* xhat, int64_t t, int accumulate,
                          bool solve, double* Gout) {
  const int N = s->N;
  std::vector<int64_t> gd(N);
  int64_t total = 1;
  for (int k = 0; k < N; ++k) {
    gd[k] = k == N - 1 ? t : s->I[k];
    total *= gd[k];
  }
  Geom g = make_geom(N, gd.data(), s->R, n);
  const int m = (int)s->m, d = g.d;
  const bool temporal = n == N - 1;
  const bool literal = temporal && s->temporal_literal;
  double w = 1.0;
  if (s->rescale && !literal)
    w = temporal ? (double)prod_dims_except(s, -1) / m : (double)prod_dims_except(s, n) * t / m;
  TR_HIP(launch_sample_rows_c(g, (const double* const*)s->dGSc, m, w, literal ? 1 : 0, s->Ast,
                              s->Bst, s->Sw2, s->st));
  // the (re-)Gram of the sampled subchain: both planes with the sketch
  // weights, or the real plane unweighted for the literal temporal reading
  const double* gw = literal ? nullptr : s->Sw2;
  const int64_t grows = literal ? (int64_t)m : 2 * (int64_t)m;
  SgemmPlan sp = plan_sgemm(g, m, 2 * d, s->dt);
  TR_HIP(ensure(&s->part, &s->part_bytes, (size_t)sp.nsplit * g.In * 2 * d * sp.psize));
  TR_HIP(ensure((void**)&s->Zk, &s->Zk_bytes, (size_t)g.In * 2 * d * sizeof(double)));
  TR_HIP(ensure((void**)&s->dPk, &s->dPk_bytes, (size_t)g.In * d * sizeof(double)));
  // the mixed product, its reduction and the unmixing on the second stream;
  // the Gram and the inverse (the longer chain) on the caller's stream,
  // which the solve then follows with no cross-stream wait of its own
  // unless the product chain is still running
  {
    tr_status c0 = fork_side(s);
    if (c0 != TR_OK) return c0;
  }
  TR_HIP(launch_sgemm(g, sp, 2 * d, total, xhat, s->dt, s->idxs, m, s->Bst, s->part, s->side));
  TR_HIP(launch_reduce_solve(s->part, sp.psize, sp.nsplit, g.In, 2 * d, s->Zk, 0, nullptr,
                             nullptr, s->side));
  TR_HIP(launch_unmix(s->Zk, g.In, d, s->dsign[n], s->dPk, s->side));
  {
    tr_status c0 = temporal
                       ? gram_update_invert(s, s->st, s->Zb, s->R[n], s->R[(n + 1) % N], nullptr,
                                            0, s->Minv, s->Ast, gw, grows)
                       : gram_update_invert(s, s->st, s->Zb, s->R[n], s->R[(n + 1) % N], s->Q[n],
                                            accumulate, solve ? s->Minv : nullptr, s->Ast, gw,
                                            grows);
    if (c0 != TR_OK) return c0;
    c0 = join_side(s);
    if (c0 != TR_OK) return c0;
  }
  TR_HIP(launch_reduce_solve(s->dPk, 8, 1, g.In, d, temporal ? nullptr : s->P[n], accumulate,
                             solve ? s->Minv : nullptr, Gout, s->st));
  return TR_OK;
}

tr_status ksrft_init(tr_stream* s, const void* Xd, int64_t t_init) {
  const int N = s->N;
  s->step = 0;
  tr_status c = ksrft_signs(s, t_init);
  if (c != TR_OK) return c;
  const void* xhat = nullptr;
  c = ksrft_mix(s, Xd, t_init, &xhat);
  if (c != TR_OK) return c;
  for (int k = 0; k < N; ++k) {
    c = draw_samples(s, k, k == N - 1 ? t_init : s->I[k]);
    if (c != TR_OK) return c;
  }
  for (int k = 0; k < N; ++k) {
    c = ksrft_slices(s, k, s->G[k], k == N - 1 ? t_init : s->I[k]);
    if (c != TR_OK) return c;
  }
  for (int n = 0; n < N - 1; ++n) {
    c = ksrft_increment(s, n, xhat, t_init, 0, false, nullptr);
    if (c != TR_OK) return c;
  }
  return TR_OK;
}

// One time step of rSTR-K (Alg. 9).
tr_status ksrft_update(tr_stream* s, const void* Xd, int64_t t_new, double* Gnew) {
  const int N = s->N;
  s->step += 1;
  tr_status c = ksrft_signs(s, t_new);
  if (c != TR_OK) return c;
  const void* xhat = nullptr;
  c = ksrft_mix(s, Xd, t_new, &xhat);
  if (c != TR_OK) return c;
  // this step's signs change every core's sampled mixed slices: the
  // non-temporal ones in one launch
  {
    bool tiled = true;
    for (int k = 0; k < N - 1; ++k) tiled = tiled && s->I[k] <= 448;
    if (tiled) {
      MixSlicesAll a = {};
      a.count = N - 1;
      a.m = (int)s->m;
      for (int k = 0; k < N - 1; ++k) {
        a.G[k] = s->G[k];
        a.I[k] = (int)s->I[k];
        a.d[k] = s->d(k);
        a.D[k] = s->dsign[k];
        a.idx[k] = s->idxs + (size_t)k * s->m;
        a.GS[k] = s->GSc[k];
      }
      TR_HIP(launch_mix_slices_all(a, s->st));
    } else {
      for (int k = 0; k < N - 1; ++k) {
        c = ksrft_slices(s, k, s->G[k], s->I[k]);
        if (c != TR_OK) return c;
      }
    }
  }
  c = ksrft_increment(s, N - 1, xhat, t_new, 0, true, Gnew);
  if (c != TR_OK) return c;
  c = draw_samples(s, N - 1, t_new);
  if (c != TR_OK) return c;
  c = ksrft_slices(s, N - 1, Gnew, t_new);
  if (c != TR_OK) return c;
  for (int n = 0; n < N - 1; ++n) {
    c = ksrft_increment(s, n, xhat, t_new, 1, true, s->G[n]);
    if (c != TR_OK) return c;
    c = draw_samples(s, n, s->I[n]);
    if (c != TR_OK) return c;
    c = ksrft_slices(s, n, s->G[n], s->I[n]);
    if (c != TR_OK) return c;
  }
  return TR_OK;
}

// Validates a configuration whose first temporal block holds t_first slices
// (t_init at initialisation; the newest batch when a saved state is loaded).
tr_status check_config(const tr_config* cfg, int64_t t_first) {
  const int N = cfg->order;
  if (N < 3 || N > MAXN || !cfg->dims || !cfg->ranks) return TR_ERR_ARG;
  if (t_first < 1) return TR_ERR_SHAPE;
  for (int k = 0; k < N - 1; ++k)
    if (cfg->dims[k] < 1) return TR_ERR_SHAPE;
  for (int k = 0; k < N; ++k)
    if (cfg->ranks[k] < 1) return TR_ERR_SHAPE;
  for (int k = 0; k < N; ++k)
    if (cfg->ranks[k] > RMAXC) return TR_ERR_UNSUPPORTED;
  if (cfg->sketch != TR_SKETCH_NONE && cfg->sketch != TR_SKETCH_UNIFORM &&
      cfg->sketch != TR_SKETCH_LEVERAGE && cfg->sketch != TR_SKETCH_KSRFT)
    return TR_ERR_ARG;
  if (cfg->compute_dtype != TR_F64 && cfg->compute_dtype != TR_F32 &&
      !(cfg->compute_dtype == TR_BF16 && cfg->sketch == TR_SKETCH_KSRFT))
    return TR_ERR_UNSUPPORTED;
  if (cfg->sketch == TR_SKETCH_KSRFT) {
    // the mixing kernels take modes of up to 256 indices per batch
    for (int k = 0; k < N - 1; ++k)
      if (cfg->dims[k] > 256) return TR_ERR_UNSUPPORTED;
    if (t_first > 256) return TR_ERR_UNSUPPORTED;
  }
  if (cfg->sketch != TR_SKETCH_NONE) {
    if (cfg->sketch_size < 1 || cfg->sketch_size > (1 << 24)) return TR_ERR_ARG;
    for (int k = 0; k < N; ++k)
      if (cfg->sketch_size < (int64_t)cfg->ranks[k] * cfg->ranks[(k + 1) % N])
        return TR_ERR_UNSUPPORTED;
  }
  for (int k = 0; k < N; ++k)
    if (cfg->ranks[k] * cfg->ranks[(k + 1) % N] > 256) return TR_ERR_UNSUPPORTED;
  if (cfg->sweeps < 0 || cfg->init_max_sweeps < 0) return TR_ERR_ARG;
  if (cfg->sweeps > 1 && cfg->sketch != TR_SKETCH_NONE) return TR_ERR_UNSUPPORTED;
  return TR_OK;
}

// Creates a handle for a validated configuration and allocates its device
// state, with room for at least t_slices temporal slices.  *out receives
// the handle even on failure (the caller destroys it).
tr_status create_handle(const tr_config* cfg, int64_t t_slices, tr_stream** out) {
  const int N = cfg->order;
  tr_stream* s = new tr_stream();
  s->N = N;
  for (int k = 0; k < N - 1; ++k) s->I[k] = cfg->dims[k];
  for (int k = 0; k < N; ++k) s->R[k] = cfg->ranks[k];
  s->dt = cfg->compute_dtype;
  s->sketch = cfg->sketch;
  s->m = cfg->sketch_size;
  s->rescale = cfg->rescale;
  s->temporal_literal = cfg->temporal_normal_eq ? 0 : 1;
  s->sweeps = cfg->sweeps > 1 ? cfg->sweeps : 1;
  s->seed = cfg->seed;
  s->check_finite = cfg->check_finite;
  s->device = cfg->device;
  *out = s;

  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->device));
  if (cfg->hip_stream) {
    s->st = (hipStream_t)cfg->hip_stream;
  } else {
    TR_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    s->own_stream = true;
  }
  TR_HIP(hipEventCreateWithFlags(&s->copy_done, hipEventDisableTiming));

  int dmax = 0;
  for (int k = 0; k < N; ++k) dmax = std::max(dmax, s->d(k));
  s->cap = std::max<int64_t>(cfg->max_slices, t_slices + 1024);
  for (int k = 0; k < N - 1; ++k) {
    TR_HIP(dev_alloc(&s->G[k], (size_t)s->I[k] * s->d(k)));
    TR_HIP(dev_alloc(&s->P[k], (size_t)s->I[k] * s->d(k)));
    TR_HIP(dev_alloc(&s->Q[k], (size_t)s->d(k) * s->d(k)));
  }
  TR_HIP(dev_alloc(&s->G[N - 1], (size_t)s->cap * s->d(N - 1)));
  for (int k = 0; k < N; ++k) {
    const int rk = s->R[k], rk1 = s->R[(k + 1) % N];
    TR_HIP(dev_alloc(&s->E[k], (size_t)rk * rk * rk1 * rk1));
  }
  TR_HIP(dev_alloc(&s->Minv, (size_t)dmax * dmax));
  for (int k = 0; k < N; ++k) TR_HIP(dev_alloc(&s->MinvM[k], (size_t)dmax * dmax));
  // pseudo-inverse fallback: the largest matrix an elimination inverts is
  // d x d, or the row Gram of a leverage rank check (at most 256 x 256)
  const int dfb = s->sketch == TR_SKETCH_NONE ? dmax : 256;
  TR_HIP(dev_alloc(&s->pinvH, (size_t)dfb * dfb));
  TR_HIP(dev_alloc(&s->pinvW, (size_t)2 * dfb * dfb + dfb));
  if (s->sweeps > 1)
    for (int k = 0; k < N - 1; ++k) {
      TR_HIP(dev_alloc(&s->Pold[k], (size_t)s->I[k] * s->d(k)));
      TR_HIP(dev_alloc(&s->Qold[k], (size_t)s->d(k) * s->d(k)));
    }
  TR_HIP(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
  // ordering events between the two streams of one device: a device-scope
  // release suffices (each kernel's dispatch already releases its writes to
  // the device), and the default system-scope writeback costs ~15 us per
  // event on the dependent path
  const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
  TR_HIP(hipEventCreateWithFlags(&s->ev_fork, evf));
  TR_HIP(hipEventCreateWithFlags(&s->ev_join, evf));
  for (int k = 0; k < N; ++k) {
    TR_HIP(hipEventCreateWithFlags(&s->ev_inv[k], evf));
    TR_HIP(hipEventCreateWithFlags(&s->ev_rs[k], evf));
  }
  int emax = 0;
  for (int k = 0; k < N; ++k) emax = std::max(emax, s->R[k] * s->R[k]);
  TR_HIP(dev_alloc(&s->chain[0], (size_t)emax * emax));
  TR_HIP(dev_alloc(&s->chain[1], (size_t)emax * emax));
  TR_HIP(dev_alloc(&s->pair, 2));
  TR_HIP(dev_alloc(&s->dstatus, 4));
  TR_HIP(hipMemsetAsync(s->dstatus, 0, 4 * sizeof(int), s->st));
  TR_HIP(dev_alloc(&s->sidecnt, 1));
  TR_HIP(hipMemsetAsync(s->sidecnt, 0, sizeof(unsigned), s->st));
  if (s->sketch != TR_SKETCH_NONE) {
    TR_HIP(dev_alloc(&s->idxs, (size_t)N * s->m));
    TR_HIP(dev_alloc(&s->SA, (size_t)s->m * dmax));
    TR_HIP(dev_alloc(&s->Sw, (size_t)s->m));
    TR_HIP(dev_alloc(&s->Zb, (size_t)256 * 256));
    TR_HIP(dev_alloc(&s->Zi, (size_t)256 * 256));
    TR_HIP(dev_alloc(&s->dprobs, (size_t)N));
    if (s->sketch == TR_SKETCH_LEVERAGE)
      for (int k = 0; k < N - 1; ++k) TR_HIP(dev_alloc(&s->probs[k], (size_t)s->I[k]));
    TR_HIP(hipMemcpyAsync(s->dprobs, s->probs, N * sizeof(double*), hipMemcpyHostToDevice, s->st));
  }
  if (s->sketch == TR_SKETCH_KSRFT) {
    for (int k = 0; k < N - 1; ++k) TR_HIP(dev_alloc(&s->dsign[k], (size_t)s->I[k]));
    for (int k = 0; k < N; ++k) TR_HIP(dev_alloc(&s->GSc[k], (size_t)2 * s->m * s->d(k)));
    TR_HIP(dev_alloc(&s->dGSc, (size_t)N));
    TR_HIP(hipMemcpyAsync(s->dGSc, s->GSc, N * sizeof(double*), hipMemcpyHostToDevice, s->st));
    TR_HIP(dev_alloc(&s->Ast, (size_t)2 * s->m * dmax));
    TR_HIP(dev_alloc(&s->Bst, (size_t)4 * s->m * dmax));
    TR_HIP(dev_alloc(&s->Sw2, (size_t)2 * s->m));
  }
  return TR_OK;
}

// ---- saved state (tr_stream_save / tr_stream_load) --------------------------

const char kSaveMagic[8] = {'T', 'R', 'S', 'T', 'A', 'T', 'E', '2'};

struct SaveHeader {
  char magic[8];
  int32_t N, dt, sketch, rescale, temporal_literal, check_finite, sweeps, pad;
  int64_t m, t_total, step, last_t;
  uint64_t seed;
  int64_t dims[MAXN];
  int32_t ranks[MAXN];
  uint64_t payload_bytes, checksum;
};

struct SaveArray {
  void* dev;
  size_t bytes;
};

// The device arrays that carry the state from one time step to the next, in
// file order: per core k < N-1 its rows, P_k and Q_k; the temporal rows; the
// Gram matrices; the sample indices (randomized variants) and the leverage
// distributions of the non-temporal cores.  Everything else is rebuilt by
// the next update (inverses, scratch, signs, sampled mixed slices).
std::vector<SaveArray> save_arrays(const tr_stream* s) {
  const int N = s->N;
  std::vector<SaveArray> v;
  for (int k = 0; k < N - 1; ++k) {
    const size_t rows = (size_t)s->I[k] * s->d(k) * sizeof(double);
    v.push_back({s->G[k], rows});
    v.push_back({s->P[k], rows});
    v.push_back({s->Q[k], (size_t)s->d(k) * s->d(k) * sizeof(double)});
  }
  v.push_back({s->G[N - 1], (size_t)s->t_total * s->d(N - 1) * sizeof(double)});
  for (int k = 0; k < N; ++k) {
    const size_t a = (size_t)s->R[k] * s->R[k], b = (size_t)s->R[(k + 1) % N] * s->R[(k + 1) % N];
    v.push_back({s->E[k], a * b * sizeof(double)});
  }
  if (s->sketch != TR_SKETCH_NONE) v.push_back({s->idxs, (size_t)N * s->m * sizeof(int32_t)});
  if (s->sketch == TR_SKETCH_LEVERAGE)
    for (int k = 0; k < N - 1; ++k) v.push_back({s->probs[k], (size_t)s->I[k] * sizeof(double)});
  return v;
}

// 64-bit FNV-1a hash (Fowler, Noll, Vo) of the payload, to reject a torn or
// altered file before any device state is created.
uint64_t fnv1a(const char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Cores in the column-major core layout (FP64, host or device; core N-1
// with T slices) to the slice-major state rows.
tr_status load_cores(tr_stream* s, const double* const* cores, int on_device, int64_t T) {
  const int N = s->N;
  std::vector<int64_t> dims(N);
  for (int k = 0; k < N - 1; ++k) dims[k] = s->I[k];
  dims[N - 1] = T;
  size_t maxcore = 0;
  for (int k = 0; k < N; ++k) maxcore = std::max(maxcore, (size_t)dims[k] * s->d(k));
  double* tmp = nullptr;
  if (!on_device) TR_HIP(dev_alloc(&tmp, maxcore));
  tr_status c = TR_OK;
  for (int k = 0; k < N && c == TR_OK; ++k) {
    const size_t cnt = (size_t)dims[k] * s->d(k);
    const double* src = cores[k];
    if (!src) {
      c = poison(s, TR_ERR_ARG, "null core pointer");
      break;
    }
    if (!on_device) {
      TR_HIP(hipMemcpyAsync(tmp, src, cnt * sizeof(double), hipMemcpyHostToDevice, s->st));
      src = tmp;
    }
    TR_HIP(launch_core_to_slices(src, F64, 1, s->R[k], (int64_t)s->R[k] * dims[k], dims[k],
                                 s->R[k], s->R[(k + 1) % N], s->G[k], s->st));
    if (!on_device) TR_HIP(hipStreamSynchronize(s->st));
  }
  if (tmp) TR_HIP(hipFree(tmp));
  return c;
}

// ---- batch TR-ALS with normal equations (Alg. 2) ----------------------------

// ||X - TR(G)|| / ||X|| of the state cores over the T slices of Xd (compute
// dtype), synchronous.
tr_status state_error(tr_stream* s, const void* Xd, int64_t T, double* out) {
  const int N = s->N;
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = T;
  Geom g = make_geom(N, gd.data(), s->R, N - 1);
  const int nwg = recon_err_blocks(g);
  if ((size_t)nwg * 2 > s->wg_n) {
    if (s->wg) {
      TR_HIP(hipStreamSynchronize(s->st));
      TR_HIP(hipFree(s->wg));
    }
    TR_HIP(dev_alloc(&s->wg, (size_t)nwg * 2));
    s->wg_n = (size_t)nwg * 2;
  }
  int got = 0;
  TR_HIP(launch_recon_err(g, Xd, s->dt, state_view(s, s->G[N - 1]), F64, s->G[N - 1], s->wg, &got,
                          s->st));
  TR_HIP(launch_sum_pairs(s->wg, got, s->pair, s->st));
  double h[2];
  TR_HIP(hipMemcpyAsync(h, s->pair, sizeof(h), hipMemcpyDeviceToHost, s->st));
  TR_HIP(hipStreamSynchronize(s->st));
  *out = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return TR_OK;
}

// Batch TR-ALS with normal equations (Alg. 2) on the state cores, over the
// T slices of Xd: per sweep the modes n = 0..N-1 in order, each with
//   H^{!=n} from the Gram tensors of the other cores (Gram refresh of the
//   core updated just before, Gram chain, (pseudo-)inverse: side kernel),
//   M_n = X_[n] G^{!=n}_[2] (MTTKRP over all T slices),
//   G_{n(2)} = M_n (H^{!=n}_<2>)^dagger (reduction + solve),
// and the relative error after the sweep; it stops when the error changes
// by less than `tol` or after max_sweeps (the stopping rule of the Sec. 4
// protocol).  errs receives the error of the starting cores and of every
// sweep.  The Gram tensors of the final cores are left in E.
tr_status als_run(tr_stream* s, const void* Xd, int64_t T, int max_sweeps, double tol,
                  std::vector<double>* errs) {
  const int N = s->N;
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = T;
  for (int k = 0; k < N; ++k)
    TR_HIP(launch_gram_E(s->G[k], gd[k], s->R[k], s->R[(k + 1) % N], s->E[k], s->st));
  double e = 0.0;
  tr_status c = state_error(s, Xd, T, &e);
  if (c != TR_OK) return c;
  errs->push_back(e);
  const CoreView cv = state_view(s, s->G[N - 1]);
  int sw = 0;
  while (sw < max_sweeps) {
    for (int n = 0; n < N; ++n) {
      const int p = (n + N - 1) % N;
      SideArgs a;
      std::memset(&a, 0, sizeof(a));
      a.Gp = s->G[p];
      a.rows_p = gd[p];
      a.Rpa = s->R[p];
      a.Rpb = s->R[(p + 1) % N];
      a.Ep = s->E[p];
      a.nfac = N - 1;
      for (int j = 0; j < N - 1; ++j) {
        const int q = (n + 1 + j) % N;
        a.fac[j] = s->E[q];
        a.fr[j] = s->R[q] * s->R[q];
        a.fc[j] = s->R[(q + 1) % N] * s->R[(q + 1) % N];
      }
      a.cbuf[0] = s->chain[0];
      a.cbuf[1] = s->chain[1];
      a.Ra = s->R[n];
      a.Rb = s->R[(n + 1) % N];
      a.Q = s->pinvH;                // H^{!=n} kept for the fallback
      a.store_Q = 1;
      a.Qinv = s->MinvM[n];
      a.status = s->dstatus;
      a.counter = s->sidecnt;
      a.pw = s->pinvW;
      TR_HIP(launch_side(a, s->st));
      Geom g = make_geom(N, gd.data(), s->R, n);
      MttkrpPlan pl = plan_mttkrp(g, s->dt);
      c = ensure_partials(s, g, pl);
      if (c != TR_OK) return c;
      TR_HIP(launch_mttkrp(g, pl, Xd, s->dt, cv, F64, s->part, s->st));
      TR_HIP(launch_reduce_solve(s->part, pl.psize, pl.nsplit, g.In, g.d, nullptr, 0, s->MinvM[n],
                                 s->G[n], s->st));
    }
    ++sw;
    c = state_error(s, Xd, T, &e);
    if (c != TR_OK) return c;
    errs->push_back(e);
    if (std::fabs((*errs)[errs->size() - 2] - e) < tol) break;
  }
  TR_HIP(launch_gram_E(s->G[N - 1], T, s->R[N - 1], s->R[0], s->E[N - 1], s->st));
  s->init_sweeps = sw;
  s->init_err = e;
  return read_status(s);
}

// Random start of the batch TR-ALS: core k (slice-major state rows) from
// the initial-core stream of the counter-based generator (kind 2).
tr_status random_cores(tr_stream* s, int64_t T) {
  const int N = s->N;
  for (int k = 0; k < N; ++k) {
    const int64_t I = k == N - 1 ? T : s->I[k];
    TR_HIP(launch_init_normal(rng_key(s->seed, 0, (uint64_t)k, 2), s->R[k], I, s->R[(k + 1) % N],
                              s->G[k], s->st));
  }
  return TR_OK;
}

// One pass of the STR update stage (Alg. 4) over the batch Xd of t_new
// slices (compute dtype), writing the new temporal rows at Gnew.
tr_status str_pass(tr_stream* s, const void* Xd, int64_t t_new, double* Gnew) {
  // Per mode: the side step (Gram refresh of the core updated just before,
  // Gram chain, Q update, inverse), the MTTKRP, then the split reduction +
  // solve, which needs both.  When every mode fits the fused launch the side
  // step and the MTTKRP share one kernel on the caller's stream.  Otherwise
  // the side stream carries the serial chain (side kernel, then solve) and
  // the caller's stream the MTTKRPs, each after the solve before it.
  const int N = s->N;
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = t_new;
  tr_status c;
  hipStream_t side = s->side;
  long pr;
  auto side_args = [&](int n, int p, const double* Gp, int64_t rows_p) {
    // every field not set below (the Gram's row weights Gw among them) is
    // zero: the kernels test those pointers
    SideArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Gp = Gp;
    a.rows_p = rows_p;
    a.Rpa = s->R[p];
    a.Rpb = s->R[(p + 1) % N];
    a.Ep = s->E[p];
    a.nfac = N - 1;
    for (int j = 0; j < N - 1; ++j) {
      const int q = (n + 1 + j) % N;
      a.fac[j] = s->E[q];
      a.fr[j] = s->R[q] * s->R[q];
      a.fc[j] = s->R[(q + 1) % N] * s->R[(q + 1) % N];
    }
    a.cbuf[0] = s->chain[0];
    a.cbuf[1] = s->chain[1];
    a.Ra = s->R[n];
    a.Rb = s->R[(n + 1) % N];
    // the temporal mode's H^{!=N} is not kept, but stored to scratch for the
    // pseudo-inverse fallback
    a.Q = n == N - 1 ? s->pinvH : s->Q[n];
    a.accumulate = n == N - 1 ? 0 : 1;
    a.store_Q = 1;
    a.Qinv = s->MinvM[n];
    a.status = s->dstatus;
    a.counter = s->sidecnt;
    a.pw = s->pinvW;
    a.mcols = 1;                     // used by the fused launch where it applies
    return a;
  };
  auto side_of = [&](int n) {
    if (n == N - 1) return side_args(N - 1, N - 2, s->G[N - 2], s->I[N - 2]);
    if (n == 0) return side_args(0, N - 1, Gnew, t_new);
    return side_args(n, n - 1, s->G[n - 1], s->I[n - 1]);
  };
  // one stream when every mode fits the fused launch: per mode the side
  // step and the MTTKRP in one kernel, then the split reduction + solve
  bool fused = true;
  for (int n = 0; n < N; ++n) fused = fused && mode_fusable(make_geom(N, gd.data(), s->R, n), side_of(n));
  if (fused) {
    for (int j = 0; j < N; ++j) {
      const int n = j == 0 ? N - 1 : j - 1;
      const bool temporal = n == N - 1;
      Geom g = make_geom(N, gd.data(), s->R, n);
      const SideArgs sa = side_of(n);
      // order 3: the temporal MTTKRP runs in mode 1's GEMM geometry (rows
      // i_1, outer index t; no padding of the batch's rows to 16) with the
      // slice G_1(i_1) applied per row, one partial per row tile
      // (on 8-wave workgroups: the planner must give outer-index pairs)
      bool prv = temporal && N == 3 && !getenv("TRSTREAM_NOPRV");
      Geom gm = g;
      MttkrpPlan p;
      if (prv) {
        gm = make_geom(N, gd.data(), s->R, 1);
        p = plan_mode(gm, s->dt, sa, s->ncu);
        prv = p.ng == 2;
        p.prv = prv ? 1 : 0;
        p.prv_in = (int)g.In;
      }
      if (!prv) {
        gm = g;
        p = plan_mode(g, s->dt, sa, s->ncu);
      }
      c = ensure_partials(s, gm, p);
      if (c != TR_OK) return c;
      const CoreView cv = state_view(s, Gnew);
      pr = prof_begin(s, temporal ? PK_MTT_T : PK_MTT_N);
      TR_HIP(launch_mode(gm, p, Xd, s->dt, cv, F64, s->part, sa, s->st));
      prof_end(s, pr);
      pr = prof_begin(s, PK_SOLVE);
      if (temporal)
        TR_HIP(launch_reduce_solve(s->part, p.psize, prv ? p.mtiles : p.nsplit, g.In, g.d,
                                   nullptr, 0, s->MinvM[N - 1], Gnew, s->st));
      else
        TR_HIP(launch_reduce_solve(s->part, p.psize, p.nsplit, g.In, g.d, s->P[n], 1,
                                   s->MinvM[n], s->G[n], s->st));
      prof_end(s, pr);
    }
    return TR_OK;
  }
  // otherwise two streams.  Modes in order: temporal (its side kernel also
  // refreshes Z_{N-1} of the previous step's last core), then n = 0..N-2
  // (mode n's side kernel refreshes the Gram of the core updated just
  // before it; Z_N^new for n = 0)
  TR_HIP(hipEventRecord(s->ev_fork, s->st));
  TR_HIP(hipStreamWaitEvent(side, s->ev_fork, 0));
  // FP32 operands: the MTTKRPs that qualify run on formed subchain blocks
  // (split as stream_zwg says)
  // (FP32 cores and accumulation); the cores are copied to FP32 once per
  // pass on the main stream (beside the first side kernel) and each solve
  // writes the FP32 copy of the rows it produces
  bool zf[MAXN] = {};
  bool any_zf = false;
  if (s->dt == F32) {
    for (int n = 0; n < N; ++n) {
      const Geom gz = make_geom(N, gd.data(), s->R, n);
      zf[n] = plan_mttkrp(gz, F32, stream_zwg(gz), true).zform != 0;
      any_zf = any_zf || zf[n];
    }
  }
  CoreView cv32 = state_view(s, Gnew);
  if (any_zf) {
    for (int k = 0; k < N; ++k) {
      const int64_t rows = k == N - 1 ? t_new : s->I[k];
      TR_HIP(ensure(&s->G32[k], &s->G32_bytes[k], (size_t)rows * s->d(k) * sizeof(float)));
      if (k < N - 1) TR_HIP(launch_cast(s->G[k], F64, s->G32[k], F32, rows * s->d(k), s->st));
      cv32.ptr[k] = s->G32[k];
    }
  }
  for (int j = 0; j < N; ++j) {
    const int n = j == 0 ? N - 1 : j - 1;
    const bool temporal = n == N - 1;
    pr = prof_begin(s, PK_CHAIN, side);
    TR_HIP(launch_side(side_of(n), side));
    prof_end(s, pr, side);
    if (!temporal) TR_HIP(hipStreamWaitEvent(s->st, s->ev_rs[n == 0 ? N - 1 : n - 1], 0));
    Geom g = make_geom(N, gd.data(), s->R, n);
    MttkrpPlan p = zf[n] ? plan_mttkrp(g, F32, stream_zwg(g), true) : plan_mttkrp(g, s->dt);
    c = ensure_partials(s, g, p);
    if (c != TR_OK) return c;
    const CoreView cv = state_view(s, Gnew);
    pr = prof_begin(s, temporal ? PK_MTT_T : PK_MTT_N);
    if (zf[n])
      TR_HIP(launch_mttkrp(g, p, Xd, F32, cv32, F32, s->part, s->st));
    else
      TR_HIP(launch_mttkrp(g, p, Xd, s->dt, cv, F64, s->part, s->st));
    prof_end(s, pr);
    TR_HIP(hipEventRecord(s->ev_inv[n], s->st));
    TR_HIP(hipStreamWaitEvent(side, s->ev_inv[n], 0));
    pr = prof_begin(s, PK_SOLVE, side);
    float* g32 = any_zf ? (float*)s->G32[n] : nullptr;
    if (temporal)
      TR_HIP(launch_reduce_solve(s->part, p.psize, p.nsplit, g.In, g.d, nullptr, 0,
                                 s->MinvM[N - 1], Gnew, side, g32));
    else
      TR_HIP(launch_reduce_solve(s->part, p.psize, p.nsplit, g.In, g.d, s->P[n], 1,
                                 s->MinvM[n], s->G[n], side, g32));
    prof_end(s, pr, side);
    TR_HIP(hipEventRecord(s->ev_rs[n], side));
  }
  TR_HIP(hipEventRecord(s->ev_join, side));
  TR_HIP(hipStreamWaitEvent(s->st, s->ev_join, 0));
  return TR_OK;
}

}  // namespace

extern "C" {

tr_status tr_stream_init(const tr_config* cfg, const double* X_init, int64_t t_init,
                         int32_t x_is_device, const double* const* cores_init,
                         int32_t cores_on_device, tr_stream** out) {
  if (!cfg || !out || !X_init) return TR_ERR_ARG;
  *out = nullptr;
  tr_status c = check_config(cfg, t_init);
  if (c != TR_OK) return c;
  c = create_handle(cfg, t_init, out);
  tr_stream* s = *out;
  if (c != TR_OK) return c;
  const int N = s->N;

  if (cores_init) {
    c = load_cores(s, cores_init, cores_on_device, t_init);
    if (c != TR_OK) return c;
  }
  s->t_total = t_init;
  s->last_t = t_init;

  // X_init on the device in the compute dtype
  int64_t J = 1;
  for (int k = 0; k < N - 1; ++k) J *= s->I[k];
  const void* Xd = nullptr;
  c = stage_batch(s, X_init, F64, J * t_init, x_is_device, &Xd);
  if (c != TR_OK) return c;
  if (!cores_init) {
    // no initial cores: batch TR-ALS (Alg. 2) on X_init from the random
    // start, as the protocol of Sec. 4 initialises the trackers
    c = random_cores(s, t_init);
    if (c != TR_OK) return c;
    std::vector<double> errs;
    c = als_run(s, Xd, t_init, cfg->init_max_sweeps > 0 ? cfg->init_max_sweeps : 100,
                cfg->init_tol > 0 ? cfg->init_tol : 1e-8, &errs);
    if (c != TR_OK) return c;
  }
  // Gram matrices (Alg. 4 initialisation; Z_N over the initial temporal rows)
  for (int k = 0; k < N; ++k) {
    const int64_t rows = k == N - 1 ? t_init : s->I[k];
    TR_HIP(launch_gram_E(s->G[k], rows, s->R[k], s->R[(k + 1) % N], s->E[k], s->st));
  }

  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = t_init;
  const CoreView cv = state_view(s, s->G[N - 1]);
  if (s->sketch != TR_SKETCH_NONE) {
    c = s->sketch == TR_SKETCH_KSRFT ? ksrft_init(s, Xd, t_init) : sketch_init(s, Xd, t_init);
    if (c != TR_OK) return c;
    TR_HIP(hipStreamSynchronize(s->st));
    s->copy_pending = false;
    return read_status(s);
  }
  for (int n = 0; n < N - 1; ++n) {
    Geom g = make_geom(N, gd.data(), s->R, n);
    MttkrpPlan p = plan_mttkrp(g, s->dt);
    c = ensure_partials(s, g, p);
    if (c != TR_OK) return c;
    TR_HIP(launch_mttkrp(g, p, Xd, s->dt, cv, F64, s->part, s->st));
    TR_HIP(launch_reduce_solve(s->part, p.psize, p.nsplit, g.In, g.d, s->P[n], 0, nullptr,
                               nullptr, s->st));
    hipError_t he;
    const double* M = chain_product(s, n, s->E[N - 1], &he);
    TR_HIP(he);
    TR_HIP(launch_assemble_q(M, s->R[n], s->R[(n + 1) % N], s->Q[n], 0, s->st));
  }
  TR_HIP(hipStreamSynchronize(s->st));
  s->copy_pending = false;
  return TR_OK;
}

tr_status tr_stream_update(tr_stream* s, const void* X_new, int32_t x_dtype, int64_t t_new,
                           int32_t x_is_device) {
  if (!s) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  if (!X_new) return fail(s, TR_ERR_ARG, "null batch");
  if (t_new < 1) return fail(s, TR_ERR_SHAPE, "t_new must be positive");
  if (x_dtype != TR_F64 && x_dtype != TR_F32) return fail(s, TR_ERR_UNSUPPORTED, "batch dtype");
  if (!s->next_signs.empty() && s->next_signs_t != t_new)
    return fail(s, TR_ERR_SHAPE, "injected temporal signs do not match the batch size");
  const int N = s->N;
  TR_HIP(hipSetDevice(s->device));
  int64_t J = 1;
  for (int k = 0; k < N - 1; ++k) J *= s->I[k];
  tr_status c = grow_temporal(s, s->t_total + t_new);
  if (c != TR_OK) return c;
  const void* Xd = nullptr;
  c = stage_batch(s, X_new, x_dtype, J * t_new, x_is_device, &Xd);
  if (c != TR_OK) return c;

  const int dN = s->d(N - 1);
  double* Gnew = s->G[N - 1] + (size_t)s->t_total * dN;

  if (s->sketch != TR_SKETCH_NONE) {
    const long pst = prof_begin(s, PK_STEP);
    if (s->sketch == TR_SKETCH_KSRFT && t_new > 256)
      return fail(s, TR_ERR_UNSUPPORTED, "KSRFT batches hold at most 256 slices");
    c = s->sketch == TR_SKETCH_KSRFT ? ksrft_update(s, Xd, t_new, Gnew)
                                     : sketch_update(s, Xd, t_new, Gnew);
    if (c != TR_OK) return c;
    prof_end(s, pst);
    s->t_total += t_new;
    s->last_t = t_new;
    return TR_OK;
  }
  // STR: one pass of the update stage (Alg. 4), or `sweeps` passes that
  // each start again from the P_n, Q_n held before the batch and rewrite the
  // new temporal rows (the multi-pass extension)
  const long pstep = prof_begin(s, PK_STEP);
  for (int k = 0; k < s->sweeps; ++k) {
    for (int n = 0; n < N - 1 && s->sweeps > 1; ++n) {
      const size_t pb = (size_t)s->I[n] * s->d(n) * sizeof(double);
      const size_t qb = (size_t)s->d(n) * s->d(n) * sizeof(double);
      if (k == 0) {
        TR_HIP(hipMemcpyAsync(s->Pold[n], s->P[n], pb, hipMemcpyDeviceToDevice, s->st));
        TR_HIP(hipMemcpyAsync(s->Qold[n], s->Q[n], qb, hipMemcpyDeviceToDevice, s->st));
      } else {
        TR_HIP(hipMemcpyAsync(s->P[n], s->Pold[n], pb, hipMemcpyDeviceToDevice, s->st));
        TR_HIP(hipMemcpyAsync(s->Q[n], s->Qold[n], qb, hipMemcpyDeviceToDevice, s->st));
      }
    }
    c = str_pass(s, Xd, t_new, Gnew);
    if (c != TR_OK) return c;
  }
  prof_end(s, pstep);
  s->t_total += t_new;
  s->last_t = t_new;
  return TR_OK;
}

tr_status tr_stream_sync(tr_stream* s) {
  if (!s) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipStreamSynchronize(s->st));
  s->copy_pending = false;
  return read_status(s);
}

tr_status tr_reconstruct_error(tr_stream* s, const double* X_all, int64_t t_all,
                               int32_t x_is_device, double* rel_err) {
  if (!s || !X_all || !rel_err) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  if (t_all != s->t_total) return fail(s, TR_ERR_SHAPE, "t_all differs from the slices seen");
  const int N = s->N;
  TR_HIP(hipSetDevice(s->device));
  tr_status c = read_status(s);
  if (c != TR_OK) return c;
  int64_t J = 1;
  for (int k = 0; k < N - 1; ++k) J *= s->I[k];
  const double* Xd = X_all;
  double* tmp = nullptr;
  if (!x_is_device) {
    TR_HIP(dev_alloc(&tmp, (size_t)J * t_all));
    TR_HIP(hipMemcpy(tmp, X_all, (size_t)J * t_all * sizeof(double), hipMemcpyHostToDevice));
    Xd = tmp;
  }
  std::vector<int64_t> gd(N);
  for (int k = 0; k < N - 1; ++k) gd[k] = s->I[k];
  gd[N - 1] = t_all;
  Geom g = make_geom(N, gd.data(), s->R, N - 1);
  const int nwg = recon_err_blocks(g);
  if ((size_t)nwg * 2 > s->wg_n) {
    if (s->wg) TR_HIP(hipFree(s->wg));
    TR_HIP(dev_alloc(&s->wg, (size_t)nwg * 2));
    s->wg_n = (size_t)nwg * 2;
  }
  int got = 0;
  TR_HIP(launch_recon_err(g, Xd, F64, state_view(s, s->G[N - 1]), F64, s->G[N - 1], s->wg, &got,
                          s->st));
  TR_HIP(launch_sum_pairs(s->wg, got, s->pair, s->st));
  double h[2];
  TR_HIP(hipMemcpyAsync(h, s->pair, sizeof(h), hipMemcpyDeviceToHost, s->st));
  TR_HIP(hipStreamSynchronize(s->st));
  if (tmp) TR_HIP(hipFree(tmp));
  *rel_err = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return TR_OK;
}

tr_status tr_stream_get_cores(tr_stream* s, double* const* cores_out) {
  if (!s || !cores_out) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  tr_status c = read_status(s);
  if (c != TR_OK) return c;
  const int N = s->N;
  for (int k = 0; k < N; ++k) {
    if (!cores_out[k]) return fail(s, TR_ERR_ARG, "null output core");
    const int64_t I = k == N - 1 ? s->t_total : s->I[k];
    const int Ra = s->R[k], Rb = s->R[(k + 1) % N], dk = Ra * Rb;
    std::vector<double> h((size_t)I * dk);
    TR_HIP(hipMemcpy(h.data(), s->G[k], h.size() * sizeof(double), hipMemcpyDeviceToHost));
    double* o = cores_out[k];
    for (int64_t i = 0; i < I; ++i)
      for (int b = 0; b < Rb; ++b)
        for (int a = 0; a < Ra; ++a) o[a + Ra * (i + I * b)] = h[(size_t)i * dk + a + Ra * b];
  }
  return TR_OK;
}

tr_status tr_stream_get_PQ(tr_stream* s, int32_t n, double* P, double* Q) {
  if (!s) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  if (n < 0 || n >= s->N - 1) return fail(s, TR_ERR_ARG, "mode out of range");
  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipStreamSynchronize(s->st));
  const int dn = s->d(n);
  if (P) TR_HIP(hipMemcpy(P, s->P[n], (size_t)s->I[n] * dn * sizeof(double), hipMemcpyDeviceToHost));
  if (Q) TR_HIP(hipMemcpy(Q, s->Q[n], (size_t)dn * dn * sizeof(double), hipMemcpyDeviceToHost));
  return TR_OK;
}

tr_status tr_stream_profile(tr_stream* s, int32_t enable) {
  if (!s) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipStreamSynchronize(s->st));
  if (enable) {
    s->ev_used = 0;
    s->rec_kind.clear();
    s->rec_ev.clear();
  }
  s->prof = enable != 0;
  return TR_OK;
}

tr_status tr_stream_profile_read(tr_stream* s, int32_t kind, double* total_ms,
                                 int64_t* launches) {
  if (!s || !total_ms || !launches) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipStreamSynchronize(s->st));
  double tot = 0.0;
  int64_t cnt = 0;
  for (size_t r = 0; r < s->rec_kind.size(); ++r) {
    const int k = s->rec_kind[r];
    if (!(k == kind || (kind == 6 && (k == PK_MTT_T || k == PK_MTT_N)))) continue;
    float ms = 0.f;
    TR_HIP(hipEventElapsedTime(&ms, s->ev_pool[s->rec_ev[r]], s->ev_pool[s->rec_ev[r] + 1]));
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return TR_OK;
}

tr_status tr_stream_get_samples(tr_stream* s, int32_t* idxs) {
  if (!s || !idxs) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  if (s->sketch == TR_SKETCH_NONE) return fail(s, TR_ERR_ARG, "no sketch configured");
  TR_HIP(hipSetDevice(s->device));
  TR_HIP(hipStreamSynchronize(s->st));
  TR_HIP(hipMemcpy(idxs, s->idxs, (size_t)s->N * s->m * sizeof(int32_t), hipMemcpyDeviceToHost));
  return TR_OK;
}

tr_status tr_stream_set_samples(tr_stream* s, const int32_t* idxs, const int8_t* signs,
                                int64_t t_signs) {
  if (!s || (!idxs && !signs)) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  if (s->sketch == TR_SKETCH_NONE) return fail(s, TR_ERR_ARG, "no sketch configured");
  if (signs && s->sketch != TR_SKETCH_KSRFT)
    return fail(s, TR_ERR_ARG, "signs are injected only into the KSRFT sketch");
  const int N = s->N;
  if (idxs)
    for (int k = 0; k < N; ++k) {
      const int64_t size = k == N - 1 ? s->last_t : s->I[k];
      for (int64_t j = 0; j < s->m; ++j) {
        const int32_t v = idxs[(size_t)k * s->m + j];
        if (v < 0 || v >= size) return fail(s, TR_ERR_ARG, "sample index out of range");
      }
    }
  std::vector<double> sg;
  if (signs) {
    if (t_signs < 1 || t_signs > 256) return fail(s, TR_ERR_ARG, "t_signs out of range");
    int64_t total = t_signs;
    for (int k = 0; k < N - 1; ++k) total += s->I[k];
    sg.resize(total);
    for (int64_t j = 0; j < total; ++j) {
      if (signs[j] != 1 && signs[j] != -1) return fail(s, TR_ERR_ARG, "a sign is not +1 or -1");
      sg[j] = (double)signs[j];
    }
  }
  TR_HIP(hipSetDevice(s->device));
  if (idxs) {
    // (the sampled slices are gathered again with these indices where the
    // next step uses them: the KSRFT step re-gathers its mixed slices after
    // drawing the new signs)
    TR_HIP(hipMemcpyAsync(s->idxs, idxs, (size_t)N * s->m * sizeof(int32_t),
                          hipMemcpyHostToDevice, s->st));
    TR_HIP(hipStreamSynchronize(s->st));
  }
  if (signs) {
    s->next_signs.swap(sg);
    s->next_signs_t = t_signs;
  }
  return TR_OK;
}

tr_status tr_stream_get_stats(tr_stream* s, tr_stats* out) {
  if (!s || !out) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  int st[4] = {0, 0, 0, 0};
  TR_HIP(hipMemcpyAsync(st, s->dstatus, sizeof(st), hipMemcpyDeviceToHost, s->st));
  TR_HIP(hipStreamSynchronize(s->st));
  out->pinv_fallbacks = st[2];
  out->init_sweeps = s->init_sweeps;
  out->init_rel_err = s->init_err;
  return TR_OK;
}

tr_status tr_stream_save(tr_stream* s, const char* path) {
  if (!s || !path) return TR_ERR_ARG;
  if (s->poisoned != TR_OK) return s->poisoned;
  TR_HIP(hipSetDevice(s->device));
  tr_status c = read_status(s);  // synchronises the stream
  if (c != TR_OK) return c;
  s->copy_pending = false;
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kSaveMagic, sizeof(h.magic));
  h.N = s->N;
  h.dt = s->dt;
  h.sketch = s->sketch;
  h.rescale = s->rescale;
  h.temporal_literal = s->temporal_literal;
  h.check_finite = s->check_finite;
  h.sweeps = s->sweeps;
  h.m = s->m;
  h.t_total = s->t_total;
  h.step = s->step;
  h.last_t = s->last_t;
  h.seed = s->seed;
  for (int k = 0; k < s->N - 1; ++k) h.dims[k] = s->I[k];
  for (int k = 0; k < s->N; ++k) h.ranks[k] = s->R[k];
  std::vector<char> payload;
  for (const SaveArray& a : save_arrays(s)) {
    const size_t off = payload.size();
    payload.resize(off + a.bytes);
    TR_HIP(hipMemcpy(payload.data() + off, a.dev, a.bytes, hipMemcpyDeviceToHost));
  }
  h.payload_bytes = payload.size();
  h.checksum = fnv1a(payload.data(), payload.size());
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(s, TR_ERR_ARG, "cannot open " + tmp + " for writing");
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
            (payload.empty() || std::fwrite(payload.data(), payload.size(), 1, f) == 1);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(s, TR_ERR_ARG, std::string("writing ") + path + " failed");
  }
  return TR_OK;
}

tr_status tr_stream_load(const char* path, const tr_config* cfg, tr_stream** out) {
  if (!path || !out) return TR_ERR_ARG;
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return TR_ERR_ARG;
  SaveHeader h;
  std::vector<char> payload;
  bool ok = std::fread(&h, sizeof(h), 1, f) == 1 &&
            std::memcmp(h.magic, kSaveMagic, sizeof(h.magic)) == 0 && h.N >= 3 && h.N <= MAXN &&
            h.payload_bytes < ((uint64_t)1 << 40);
  if (ok) {
    payload.resize(h.payload_bytes);
    ok = payload.empty() || std::fread(payload.data(), payload.size(), 1, f) == 1;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
  }
  std::fclose(f);
  if (!ok || fnv1a(payload.data(), payload.size()) != h.checksum) return TR_ERR_ARG;
  tr_config fc;
  std::memset(&fc, 0, sizeof(fc));
  fc.order = h.N;
  fc.dims = h.dims;
  fc.ranks = h.ranks;
  fc.compute_dtype = h.dt;
  fc.sketch = h.sketch;
  fc.sketch_size = h.m;
  fc.rescale = h.rescale;
  fc.temporal_normal_eq = h.temporal_literal ? 0 : 1;
  fc.sweeps = h.sweeps;
  fc.seed = h.seed;
  fc.check_finite = h.check_finite;
  if (cfg) {
    if (cfg->order != 0) {
      if (cfg->order != h.N || !cfg->dims || !cfg->ranks) return TR_ERR_SHAPE;
      for (int k = 0; k < h.N - 1; ++k)
        if (cfg->dims[k] != h.dims[k]) return TR_ERR_SHAPE;
      for (int k = 0; k < h.N; ++k)
        if (cfg->ranks[k] != h.ranks[k]) return TR_ERR_SHAPE;
      if (cfg->compute_dtype != h.dt || cfg->sketch != h.sketch ||
          (h.sketch != TR_SKETCH_NONE && cfg->sketch_size != h.m))
        return TR_ERR_SHAPE;
    }
    fc.max_slices = cfg->max_slices;
    fc.device = cfg->device;
    fc.hip_stream = cfg->hip_stream;
  }
  if (h.t_total < 1 || h.last_t < 1 || h.last_t > h.t_total || h.step < 0) return TR_ERR_ARG;
  tr_status c = check_config(&fc, h.last_t);
  if (c != TR_OK) return c;
  c = create_handle(&fc, h.t_total, out);
  tr_stream* s = *out;
  if (c != TR_OK) return c;
  s->t_total = h.t_total;
  s->last_t = h.last_t;
  s->step = h.step;
  size_t need = 0;
  const std::vector<SaveArray> arrs = save_arrays(s);
  for (const SaveArray& a : arrs) need += a.bytes;
  if (need != payload.size()) return fail(s, TR_ERR_ARG, "saved state does not match its header");
  size_t off = 0;
  for (const SaveArray& a : arrs) {
    TR_HIP(hipMemcpy(a.dev, payload.data() + off, a.bytes, hipMemcpyHostToDevice));
    off += a.bytes;
  }
  TR_HIP(hipStreamSynchronize(s->st));
  return TR_OK;
}

int64_t tr_stream_num_slices(const tr_stream* s) { return s ? s->t_total : -1; }

const char* tr_last_error(const tr_stream* s) { return s ? s->err.c_str() : "null handle"; }

void tr_stream_destroy(tr_stream* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  if (s->st) (void)hipStreamSynchronize(s->st);
  for (int k = 0; k < MAXN; ++k) {
    if (s->G[k]) (void)hipFree(s->G[k]);
    if (s->E[k]) (void)hipFree(s->E[k]);
    if (s->P[k]) (void)hipFree(s->P[k]);
    if (s->Q[k]) (void)hipFree(s->Q[k]);
  }
  for (int k = 0; k < MAXN; ++k) {
    if (s->G32[k]) (void)hipFree(s->G32[k]);
    if (s->probs[k]) (void)hipFree(s->probs[k]);
    if (s->dsign[k]) (void)hipFree(s->dsign[k]);
    if (s->GSc[k]) (void)hipFree(s->GSc[k]);
  }
  void* kbufs[] = {s->dGSc, s->Ast, s->Bst, s->Sw2, s->Wmix, s->xh[0], s->xh[1], s->Zk, s->dPk};
  for (void* b : kbufs)
    if (b) (void)hipFree(b);
  void* bufs[] = {s->sidecnt, s->Minv, s->chain[0], s->chain[1], s->xcast, s->xf64, s->part,
                  s->wg,   s->pair,     s->dstatus,  s->idxs,  s->SA,   s->Sw,
                  s->Zb,   s->Zi,       s->dprobs,   s->cdf,   s->pinvH, s->pinvW};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  if (s->side) (void)hipStreamSynchronize(s->side);
  for (int k = 0; k < MAXN; ++k) {
    if (s->MinvM[k]) (void)hipFree(s->MinvM[k]);
    if (s->Pold[k]) (void)hipFree(s->Pold[k]);
    if (s->Qold[k]) (void)hipFree(s->Qold[k]);
    if (s->ev_inv[k]) (void)hipEventDestroy(s->ev_inv[k]);
    if (s->ev_rs[k]) (void)hipEventDestroy(s->ev_rs[k]);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->hpinned) (void)hipHostFree(s->hpinned);
  if (s->copy_done) (void)hipEventDestroy(s->copy_done);
  if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

// ---------------------------------------------------------------------------
// Stateless entry points (fit loss and its pieces)
// ---------------------------------------------------------------------------

namespace {

struct WsLayout {
  size_t slices[MAXN];  // offsets of slice-major FP64 core copies
  size_t E[MAXN];
  size_t chain0, chain1, Q, P, part, wg, pair, total;
};

bool valid_shape(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt) {
  if (N < 3 || N > MAXN || !dims || !ranks) return false;
  if (dt != TR_F64 && dt != TR_F32) return false;
  for (int k = 0; k < N; ++k) {
    if (dims[k] < 1 || ranks[k] < 1 || ranks[k] > RMAXC) return false;
    if (ranks[k] * ranks[(k + 1) % N] > 256) return false;
  }
  return true;
}

WsLayout ws_layout(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt) {
  WsLayout w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  int dmax = 0, emax = 0;
  size_t pmax = 0, partmax = 0;
  for (int k = 0; k < N; ++k) {
    const int dk = ranks[k] * ranks[(k + 1) % N];
    dmax = std::max(dmax, dk);
    emax = std::max(emax, ranks[k] * ranks[k]);
    w.slices[k] = take((size_t)dims[k] * dk * 8);
    w.E[k] = take((size_t)dk * dk * 8);
    pmax = std::max(pmax, (size_t)dims[k] * dk * 8);
    Geom g = make_geom(N, dims, ranks, k);
    MttkrpPlan p = plan_mttkrp(g, dt);
    partmax = std::max(partmax, mttkrp_partial_bytes(g, p));
    MttkrpPlan pb = plan_mttkrp(g, dt, 0, true);   // the fit-loss gradients' plan
    partmax = std::max(partmax, mttkrp_partial_bytes(g, pb));
  }
  w.chain0 = take((size_t)emax * emax * 8);
  w.chain1 = take((size_t)emax * emax * 8);
  w.Q = take((size_t)dmax * dmax * 8);
  w.P = take(pmax);
  w.part = take(partmax);
  Geom gN = make_geom(N, dims, ranks, N - 1);
  w.wg = take((size_t)recon_err_blocks(gN) * 2 * 8);
  w.pair = take(16);
  w.total = off;
  return w;
}

__global__ void k_half_loss(const double* pair, double* loss) {
  if (threadIdx.x == 0) loss[0] = 0.5 * pair[0];
}

}  // namespace

size_t tr_workspace_bytes(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt) {
  if (!valid_shape(N, dims, ranks, dt)) return 0;
  return ws_layout(N, dims, ranks, dt).total;
}

tr_status tr_mttkrp(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt, int32_t n,
                    const void* X, const void* const* cores, double* P_dev, int32_t accumulate,
                    void* ws, size_t ws_bytes, void* hip_stream) {
  if (!valid_shape(N, dims, ranks, dt) || !X || !cores || !P_dev || !ws) return TR_ERR_ARG;
  if (n < 0 || n >= N) return TR_ERR_ARG;
  WsLayout w = ws_layout(N, dims, ranks, dt);
  if (ws_bytes < w.total) return TR_ERR_SHAPE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* base = (char*)ws;
  Geom g = make_geom(N, dims, ranks, n);
  MttkrpPlan p = plan_mttkrp(g, dt);
  CoreView cv = colmajor_view(N, dims, ranks, cores);
  if (launch_mttkrp(g, p, X, dt, cv, dt, base + w.part, st) != hipSuccess) return TR_ERR_DEVICE;
  if (launch_reduce_solve(base + w.part, p.psize, p.nsplit, g.In, g.d, P_dev, accumulate, nullptr,
                          nullptr, st) != hipSuccess)
    return TR_ERR_DEVICE;
  return TR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free MTTKRP (tr_mttkrp_noalloc): the split-K partials live in a
// file-scope device array instead of a caller workspace.  Each device holds
// its own copy of the array; its address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept.  Every call on
// a device shares that device's array, so calls that overlap on one device
// race; the partials are fully written by the MTTKRP before the reduction
// reads them, so nothing has to be cleared between calls.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;   // 16 MiB per device
constexpr int kScratchDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's `scratch` (resolved on first use).
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t tr_mttkrp_noalloc_max_bytes(void) { return kScratchBytes; }

tr_status tr_mttkrp_noalloc(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt,
                            int32_t n, const void* X, const void* const* cores, double* P_dev,
                            int32_t accumulate, void* hip_stream) {
  if (!valid_shape(N, dims, ranks, dt) || !X || !cores || !P_dev) return TR_ERR_ARG;
  if (n < 0 || n >= N) return TR_ERR_ARG;
  Geom g = make_geom(N, dims, ranks, n);
  MttkrpPlan p = plan_mttkrp(g, dt);
  // the partials of the same plan as tr_mttkrp, so both give the same bits
  if (mttkrp_partial_bytes(g, p) > kScratchBytes) return TR_ERR_UNSUPPORTED;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return TR_ERR_DEVICE;
  void* part = nullptr;
  if (scratch_address(device, &part) != hipSuccess) return TR_ERR_DEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  CoreView cv = colmajor_view(N, dims, ranks, cores);
  if (launch_mttkrp(g, p, X, dt, cv, dt, part, st) != hipSuccess) return TR_ERR_DEVICE;
  if (launch_reduce_solve(part, p.psize, p.nsplit, g.In, g.d, P_dev, accumulate, nullptr, nullptr,
                          st) != hipSuccess)
    return TR_ERR_DEVICE;
  return TR_OK;
}

static tr_status gram_chain_into(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt,
                                 int32_t n, const void* const* cores, double* Q_dev, char* base,
                                 const WsLayout& w, hipStream_t st, bool grams_ready,
                                 int accumulate = 0) {
  if (!grams_ready) {
    for (int k = 0; k < N; ++k) {
      const int Ra = ranks[k], Rb = ranks[(k + 1) % N];
      double* sl = (double*)(base + w.slices[k]);
      if (launch_core_to_slices(cores[k], dt, 1, Ra, (int64_t)Ra * dims[k], dims[k], Ra, Rb, sl,
                                st) != hipSuccess)
        return TR_ERR_DEVICE;
      if (launch_gram_E(sl, dims[k], Ra, Rb, (double*)(base + w.E[k]), st) != hipSuccess)
        return TR_ERR_DEVICE;
    }
  }
  double* cbuf[2] = {(double*)(base + w.chain0), (double*)(base + w.chain1)};
  const double* cur = (const double*)(base + w.E[(n + 1) % N]);
  int q0 = (n + 1) % N;
  int rows = ranks[q0] * ranks[q0];
  int cols = ranks[(q0 + 1) % N] * ranks[(q0 + 1) % N];
  int pp = 0;
  for (int j = 2; j < N; ++j) {
    const int q = (n + j) % N;
    const int c2 = ranks[(q + 1) % N] * ranks[(q + 1) % N];
    if (launch_matmul(cur, (const double*)(base + w.E[q]), cbuf[pp], rows, cols, c2, st) !=
        hipSuccess)
      return TR_ERR_DEVICE;
    cur = cbuf[pp];
    pp ^= 1;
    cols = c2;
  }
  if (launch_assemble_q(cur, ranks[n], ranks[(n + 1) % N], Q_dev, accumulate, st) != hipSuccess)
    return TR_ERR_DEVICE;
  return TR_OK;
}

tr_status tr_gram_chain(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t n,
                        const double* const* Z_dev, double* Q_dev, int32_t accumulate, void* ws,
                        size_t ws_bytes, void* hip_stream) {
  if (!valid_shape(N, dims, ranks, TR_F64) || !Z_dev || !Q_dev || !ws) return TR_ERR_ARG;
  if (n < 0 || n >= N) return TR_ERR_ARG;
  for (int k = 0; k < N; ++k)
    if (k != n && !Z_dev[k]) return TR_ERR_ARG;
  // only the Gram matrices and the chain buffers of the workspace are used;
  // their offsets do not depend on the operand dtype of the sizing call
  WsLayout w = ws_layout(N, dims, ranks, TR_F64);
  int emax = 0;
  for (int k = 0; k < N; ++k) emax = std::max(emax, ranks[k] * ranks[k]);
  if (ws_bytes < w.chain1 + (size_t)emax * emax * 8) return TR_ERR_SHAPE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* base = (char*)ws;
  for (int k = 0; k < N; ++k)
    if (k != n && launch_z_to_E(Z_dev[k], ranks[k], ranks[(k + 1) % N], (double*)(base + w.E[k]),
                                st) != hipSuccess)
      return TR_ERR_DEVICE;
  return gram_chain_into(N, dims, ranks, TR_F64, n, nullptr, Q_dev, base, w, st, true,
                         accumulate);
}

tr_status tr_batch_als(const tr_config* cfg, const double* X, int64_t T, int32_t x_is_device,
                       const double* const* cores_in, int32_t cores_on_device,
                       int32_t max_sweeps, double tol, double* const* cores_out,
                       double* rel_errs, int32_t* sweeps_done) {
  if (!cfg || !X || !cores_out || max_sweeps < 0) return TR_ERR_ARG;
  tr_config c2 = *cfg;
  c2.sketch = TR_SKETCH_NONE;
  c2.sketch_size = 0;
  c2.sweeps = 0;
  c2.max_slices = T;
  tr_status c = check_config(&c2, T);
  if (c != TR_OK) return c;
  tr_stream* s = nullptr;
  c = create_handle(&c2, T, &s);
  if (c == TR_OK) {
    s->t_total = T;
    s->last_t = T;
    c = cores_in ? load_cores(s, cores_in, cores_on_device, T) : random_cores(s, T);
  }
  const void* Xd = nullptr;
  if (c == TR_OK) {
    int64_t J = 1;
    for (int k = 0; k < s->N - 1; ++k) J *= s->I[k];
    c = stage_batch(s, X, F64, J * T, x_is_device, &Xd);
  }
  std::vector<double> errs;
  if (c == TR_OK) c = als_run(s, Xd, T, max_sweeps, tol, &errs);
  if (c == TR_OK) c = tr_stream_get_cores(s, cores_out);
  if (c == TR_OK) {
    if (rel_errs)
      for (size_t j = 0; j < errs.size(); ++j) rel_errs[j] = errs[j];
    if (sweeps_done) *sweeps_done = s->init_sweeps;
  }
  tr_stream_destroy(s);
  return c;
}

tr_status tr_fit_loss_fwd(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt,
                          const void* X, const void* const* cores, double* loss_dev, void* ws,
                          size_t ws_bytes, void* hip_stream) {
  if (!valid_shape(N, dims, ranks, dt) || !X || !cores || !loss_dev || !ws) return TR_ERR_ARG;
  WsLayout w = ws_layout(N, dims, ranks, dt);
  if (ws_bytes < w.total) return TR_ERR_SHAPE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* base = (char*)ws;
  Geom g = make_geom(N, dims, ranks, N - 1);
  CoreView cv = colmajor_view(N, dims, ranks, cores);
  int nwg = 0;
  hipError_t e = hipErrorNotSupported;
  if (dt == TR_F32)
    e = launch_recon_z(g, (const float*)X, cv, (double*)(base + w.wg), recon_err_blocks(g), &nwg,
                       st);
  if (e == hipErrorNotSupported) {
    // the temporal core as slice-major FP64 rows for the MFMA product
    double* gns = (double*)(base + w.slices[N - 1]);
    const int RaN = ranks[N - 1], RbN = ranks[0];
    if (launch_core_to_slices(cores[N - 1], dt, 1, RaN, (int64_t)RaN * dims[N - 1], dims[N - 1],
                              RaN, RbN, gns, st) != hipSuccess)
      return TR_ERR_DEVICE;
    e = launch_recon_err(g, X, dt, cv, dt, gns, (double*)(base + w.wg), &nwg, st);
  }
  if (e != hipSuccess) return TR_ERR_DEVICE;
  if (launch_sum_pairs((double*)(base + w.wg), nwg, (double*)(base + w.pair), st) != hipSuccess)
    return TR_ERR_DEVICE;
  hipLaunchKernelGGL(k_half_loss, dim3(1), dim3(64), 0, st, (const double*)(base + w.pair),
                     loss_dev);
  return hipGetLastError() == hipSuccess ? TR_OK : TR_ERR_DEVICE;
}

tr_status tr_fit_loss_bwd(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t dt,
                          const void* X, const void* const* cores, double grad_scale,
                          void* const* grads, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!valid_shape(N, dims, ranks, dt) || !X || !cores || !grads || !ws) return TR_ERR_ARG;
  WsLayout w = ws_layout(N, dims, ranks, dt);
  if (ws_bytes < w.total) return TR_ERR_SHAPE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* base = (char*)ws;
  CoreView cv = colmajor_view(N, dims, ranks, cores);
  double* Q = (double*)(base + w.Q);
  double* P = (double*)(base + w.P);
  for (int n = 0; n < N; ++n) {
    tr_status c = gram_chain_into(N, dims, ranks, dt, n, cores, Q, base, w, st, n > 0);
    if (c != TR_OK) return c;
    Geom g = make_geom(N, dims, ranks, n);
    MttkrpPlan p = plan_mttkrp(g, dt, 0, true);
    if (launch_mttkrp(g, p, X, dt, cv, dt, base + w.part, st) != hipSuccess) return TR_ERR_DEVICE;
    if (launch_reduce_solve(base + w.part, p.psize, p.nsplit, g.In, g.d, P, 0, nullptr, nullptr,
                            st) != hipSuccess)
      return TR_ERR_DEVICE;
    const int Ra = ranks[n], Rb = ranks[(n + 1) % N];
    if (launch_grad_combine(cores[n], dt, 1, Ra, (int64_t)Ra * dims[n], dims[n], Ra, Rb, Q, P,
                            grad_scale, grads[n], st) != hipSuccess)
      return TR_ERR_DEVICE;
  }
  return TR_OK;
}

}  // extern "C"
