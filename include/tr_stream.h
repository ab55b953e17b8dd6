/*
 * tr_stream.h -- C ABI of the MI355X (gfx950) streaming tensor-ring tracker.
 *
 * Implements the per-batch ALS update of streaming TR decomposition (STR,
 * Alg. 4 of Yu & Li, "Tracking Tensor Ring Decompositions of Streaming
 * Tensors", arXiv 2307.00719) and its randomized variant (rSTR, Alg. 5, with
 * the uniform / leverage-score / KSRFT sketches of Algs. 7-9), plus the TR
 * fit loss 1/2 ||TR(G) - X||_F^2 with its core gradient G_{n(2)} Q_n - P_n
 * (the normal equation of Sec. 3.1).
 *
 * Layout contract (Sec. 2, the multi-index with the first index fastest):
 *   - a data tensor X of size I_1 x ... x I_{N-1} x t is column-major:
 *       X[i_1, .., i_{N-1}, t] at  i_1 + I_1*(i_2 + I_2*(... + I_{N-1}*t));
 *     a batch of t_new temporal slices is therefore one contiguous block;
 *   - a TR-core G_n (R_n x I_n x R_{n+1}, Sec. 1) is column-major:
 *       G_n[r, i, s] at  r + R_n*(i + I_n*s).
 *   All indices in this header are 0-based; mode N-1 is the temporal mode.
 *
 * Ownership: inputs are borrowed for the duration of a call.  A host X is
 * copied before the call returns.  A device X must stay valid until the
 * handle's stream has passed the call.  Outputs go to caller-allocated
 * buffers.  A handle belongs to its caller, is used by one thread at a time
 * and is freed only by tr_stream_destroy.
 *
 * Errors: every function returns a tr_status; nothing is thrown across the
 * ABI.  Arguments and shapes are validated before any state changes.  A
 * singular or rank-deficient normal-equation matrix is not an error: the
 * solve takes the pseudo-inverse (the dagger of Alg. 4 and Algs. 7-9, with
 * singular values at or below d * eps * sigma_max taken as zero) and the
 * handle counts the fallback (tr_stream_get_stats).  A device-side failure
 * (a HIP error, a normal-equation matrix holding NaN or Inf) marks the
 * handle TR_ERR_STATE and every later call on it returns that status;
 * tr_last_error() gives the message.
 */
#ifndef TR_STREAM_H
#define TR_STREAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tr_stream tr_stream;

typedef enum {
  TR_OK = 0,
  TR_ERR_ARG = 1,         /* a null pointer or an invalid option           */
  TR_ERR_SHAPE = 2,       /* sizes inconsistent with the configuration     */
  TR_ERR_NOMEM = 3,       /* device or host allocation failed              */
  TR_ERR_DEVICE = 4,      /* a HIP call failed                             */
  TR_ERR_NONFINITE = 5,   /* NaN or Inf in an input batch                  */
  TR_ERR_STATE = 6,       /* the handle was poisoned by an earlier failure */
  TR_ERR_SINGULAR = 7,    /* an elimination failed with no fallback available */
  TR_ERR_UNSUPPORTED = 8  /* a size or option outside what is built         */
} tr_status;

typedef enum { TR_F64 = 0, TR_F32 = 1, TR_BF16 = 2 } tr_dtype;

typedef enum {
  TR_SKETCH_NONE = 0,     /* STR, Alg. 4                                  */
  TR_SKETCH_UNIFORM = 1,  /* rSTR-U, Alg. 7                               */
  TR_SKETCH_LEVERAGE = 2, /* rSTR-L, Alg. 8                               */
  TR_SKETCH_KSRFT = 3     /* rSTR-K, Alg. 9                               */
} tr_sketch;

typedef struct {
  int32_t order;          /* N >= 3 (the temporal mode is the last)         */
  const int64_t *dims;    /* I_1..I_{N-1}: N-1 entries                      */
  const int32_t *ranks;   /* R_1..R_N: N entries, each 1..16                */
  int32_t compute_dtype;  /* tr_dtype of the subchain/MTTKRP operands; the
                             Gram tensors, P_n, Q_n and all solves are FP64 */
  int32_t sketch;         /* tr_sketch                                      */
  int64_t sketch_size;    /* m (sample rows) for the randomized variants    */
  int32_t rescale;        /* 1: apply the rescaling D of the sketch (default
                             reading); 0: ignore it (Sec. 3.3 remark)        */
  int32_t temporal_normal_eq; /* KSRFT temporal rows.  0 (default): the
                             printed form of the KSRFT paragraph of Sec. 3.3
                             and Alg. 9, G_N^new = Re(Xhat_S) (Re(Ghat_S^T))^+;
                             1: the real-constrained normal equations
                             Re(Xhat_S conj Ghat_S) Re(Ghat_S^T conj Ghat_S)^+ */
  uint64_t seed;          /* key of the counter-based sample generator      */
  int64_t max_slices;     /* capacity of the temporal core in slices; 0 lets
                             the library grow it (a growth synchronises)     */
  int32_t check_finite;   /* 1: reject batches holding NaN/Inf (a device
                             batch then costs one extra pass and a sync)     */
  int32_t device;         /* HIP device ordinal                             */
  void *hip_stream;       /* hipStream_t to run on; NULL = library-owned    */
  int32_t sweeps;         /* STR only: passes of the update stage over each
                             batch (0 or 1: one pass, Alg. 4).  Pass k > 1
                             starts again from the P_n, Q_n held before the
                             batch (Sec. 3.1 splits them into the old part
                             and the new batch's part) and recomputes the new
                             temporal rows and increments with the refreshed
                             cores.  An extension, not in the paper.        */
  int32_t init_max_sweeps;/* initialiser without cores (tr_stream_init with
                             cores_init NULL): batch TR-ALS sweeps at most
                             (0: 100)                                        */
  double init_tol;        /* ... and its stopping threshold on the change of
                             the relative error between sweeps (<= 0: 1e-8) */
} tr_config;

/* Counters of a handle (tr_stream_get_stats). */
typedef struct {
  int64_t pinv_fallbacks; /* normal-equation solves that took the
                             pseudo-inverse (rank-deficient or numerically
                             singular matrix) since the handle was created  */
  int32_t init_sweeps;    /* batch TR-ALS sweeps run by the initialiser
                             (0 when the cores were given)                  */
  double init_rel_err;    /* relative error on X_init after them            */
} tr_stats;

/* Initialisation stage of Alg. 4 / Algs. 7-9: store the initial cores, form
 * the Gram tensors and the complementary matrices P_n, Q_n (n < N-1) from
 * X_init (I_1 x .. x I_{N-1} x t_init, FP64).  cores_init[n] points to core n
 * in the column-major core layout; core N-1 has t_init slices.  Pointers are
 * host pointers unless x_is_device (X_init) / cores_on_device are set.
 * cores_init == NULL: the cores are computed on the device by batch TR-ALS
 * with normal equations (Alg. 2) on X_init, started from random cores of
 * the counter-based generator (stream kind 2 of cfg->seed: Irwin-Hall
 * normals) and stopped by cfg->init_tol / cfg->init_max_sweeps, as the
 * protocol of Sec. 4 initialises every tracker (remark after Alg. 4: any
 * method may give the initial cores).                                     */
tr_status tr_stream_init(const tr_config *cfg, const double *X_init, int64_t t_init,
                         int32_t x_is_device, const double *const *cores_init,
                         int32_t cores_on_device, tr_stream **out);

/* One time step (Alg. 4 update stage, or Alg. 7/8/9's): temporal rows
 * G_N^new for the t_new new slices, then modes n = 0..N-2 in order, each
 * using the cores already updated in this step.  X_new has dtype x_dtype;
 * it is cast to the compute dtype if they differ.  Asynchronous on the
 * handle's stream when X_new is on the device.                            */
tr_status tr_stream_update(tr_stream *s, const void *X_new, int32_t x_dtype,
                           int64_t t_new, int32_t x_is_device);

/* ||X_all - TR(G)||_F / ||X_all||_F over all slices seen so far (the error
 * measure of the experimental protocol, Sec. 4); X_all is FP64 with
 * t_all == tr_stream_num_slices(s).  Synchronous.                          */
tr_status tr_reconstruct_error(tr_stream *s, const double *X_all, int64_t t_all,
                               int32_t x_is_device, double *rel_err);

/* Host copies of the cores in the column-major core layout; core N-1 holds
 * tr_stream_num_slices(s) slices.  Synchronous.                           */
tr_status tr_stream_get_cores(tr_stream *s, double *const *cores_out);

/* Test hook: host copies of P_n (I_n x R_nR_{n+1}) and Q_n
 * (R_nR_{n+1} square), both row-major, column index r + R_n*s.           */
tr_status tr_stream_get_PQ(tr_stream *s, int32_t n, double *P, double *Q);

/* Test hook (randomized variants): host copy of the current sample indices,
 * N x m int32 row-major (row q = the m indices into core q, the temporal
 * row indexing the newest batch), as drawn by the counter-based generator. */
tr_status tr_stream_get_samples(tr_stream *s, int32_t *idxs);

/* Test hook (randomized variants, the generator bypassed).
 * idxs (may be NULL): replaces the current sample indices of Alg. 3's
 * Randsample with a host N x m int32 row-major array laid out as
 * tr_stream_get_samples returns it.  Row q < N-1 indexes core q
 * (0 <= idx < I_q); row N-1 indexes the newest temporal block
 * (0 <= idx < t of the last update, or t_init).  The next update uses the
 * injected rows until each is redrawn right after its core is updated,
 * exactly where drawn indices would be used.
 * signs (may be NULL; KSRFT only): the diagonals of D_1..D_N (Def. KSRFT)
 * for the next time step instead of the generator's, int8 entries +1 / -1
 * laid out as I_1 entries for D_1, then I_2 for D_2, .., then t_signs for
 * the temporal D_N; the next update must bring t_signs slices
 * (TR_ERR_SHAPE otherwise, before any state changes).
 * Out-of-range indices, signs other than +-1, signs without the KSRFT
 * sketch, both pointers NULL or no sketch configured give TR_ERR_ARG and
 * change nothing.  Synchronous: the caller may reuse the arrays on return. */
tr_status tr_stream_set_samples(tr_stream *s, const int32_t *idxs, const int8_t *signs,
                                int64_t t_signs);

/* Counters of the handle (see tr_stats).  Synchronises the handle's stream. */
tr_status tr_stream_get_stats(tr_stream *s, tr_stats *out);

/* Checkpoint of the streaming state between time steps (the quantities
 * Alg. 4 / Algs. 7-9 carry from one step to the next: the cores, the Gram
 * tensors Z_k, P_n and Q_n, and for the randomized variants the step
 * counter, the sample indices and the leverage distributions) written to a
 * host file at `path` (written to path.tmp, then renamed).  Synchronises
 * the handle's stream.  A stream resumed by tr_stream_load produces the
 * same results, bit for bit, as the uninterrupted one.  The file is a
 * private binary format for the same library build and byte order.
 * Errors: TR_ERR_ARG if the file cannot be written.                       */
tr_status tr_stream_save(tr_stream *s, const char *path);

/* Creates a handle from a file written by tr_stream_save.  cfg may be NULL
 * (device 0, library-owned stream, default capacity).  Otherwise its
 * device, hip_stream and max_slices are used, and when cfg->order is
 * non-zero its order, dims, ranks, compute_dtype, sketch and sketch_size
 * must equal the saved ones (TR_ERR_SHAPE if not).  A missing, truncated or
 * altered file (checked by a 64-bit hash of its contents) gives TR_ERR_ARG
 * before any device work.  On a failure after the handle exists, *out holds
 * it so that tr_last_error can explain; destroy it.                       */
tr_status tr_stream_load(const char *path, const tr_config *cfg, tr_stream **out);

/* Blocks until the handle's stream has finished all submitted work and
 * reports any device-side failure.                                        */
tr_status tr_stream_sync(tr_stream *s);

/* Profiling aid: with profiling on, the handle brackets each kernel of an
 * update with HIP events on its stream.  tr_stream_profile_read
 * synchronises, returns the summed duration (ms) and launch count of one
 * kind since profiling was switched on, and keeps the records.
 * Kinds: 0 temporal-mode MTTKRP, 1 non-temporal MTTKRP, 2 Gram chain and
 * normal-equation inverse, 3 split reduction and solve, 4 Gram refresh,
 * 5 whole update, 6 every MTTKRP (0 and 1).                               */
tr_status tr_stream_profile(tr_stream *s, int32_t enable);
tr_status tr_stream_profile_read(tr_stream *s, int32_t kind, double *total_ms,
                                 int64_t *launches);

int64_t tr_stream_num_slices(const tr_stream *s);
const char *tr_last_error(const tr_stream *s);
void tr_stream_destroy(tr_stream *s);

/* ---- stateless entry points (device pointers, caller's stream) ---------
 * dims: all N sizes (the last is the slice count of X); cores column-major
 * on the device in the dtype dt (F64 or F32).  ws/ws_bytes: caller-owned
 * device workspace; tr_workspace_bytes() gives the size needed.           */

size_t tr_workspace_bytes(int32_t N, const int64_t *dims, const int32_t *ranks,
                          int32_t dt);

/* P_n = X_[n] G^{!=n}_[2] (the MTTKRP-like product of Sec. 3.1, eq. partial),
 * I_n x R_nR_{n+1} row-major FP64 on the device; accumulate=1 adds.       */
tr_status tr_mttkrp(int32_t N, const int64_t *dims, const int32_t *ranks, int32_t dt,
                    int32_t n, const void *X, const void *const *cores,
                    double *P_dev, int32_t accumulate, void *ws, size_t ws_bytes,
                    void *hip_stream);

/* tr_mttkrp without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same work split as tr_mttkrp,
 * so the same bits, with the split-K partials in a file-scope device array
 * of tr_mttkrp_noalloc_max_bytes() (16 MiB) held by each device the library
 * runs on until the process ends.  The call allocates nothing and runs on
 * the current device and the caller's stream.  A problem whose partials
 * need more than that gives TR_ERR_UNSUPPORTED before any device work (use
 * tr_mttkrp).  Every call on a device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race.             */
tr_status tr_mttkrp_noalloc(int32_t N, const int64_t *dims, const int32_t *ranks, int32_t dt,
                            int32_t n, const void *X, const void *const *cores,
                            double *P_dev, int32_t accumulate, void *hip_stream);
size_t tr_mttkrp_noalloc_max_bytes(void);

/* Q_n = (G^{!=n}_[2])^T G^{!=n}_[2] = H^{!=n}_<2> through the chain of the
 * Gram tensors (Prop. subchain Gram; Alg. 2's H^{!=n}).  Z_dev[k] (k != n,
 * FP64 on the device) is the Gram tensor of core k, Z_k[b, a, b2, a2] =
 * sum_i G_k[a, i, b] G_k[a2, i, b2], of size R_{k+1} x R_k x R_{k+1} x R_k
 * stored column-major (Z_dev[n] is not read).  Q_dev: R_nR_{n+1} square,
 * row-major, row/column index r + R_n s; accumulate = 1 adds to it (Q_n +=
 * H_new of Alg. 4).  ws: the caller-owned workspace of tr_workspace_bytes
 * (the chain's intermediate products; FP64 sizing), so the call allocates
 * nothing.  dims are those of the stateless calls (all N sizes).          */
tr_status tr_gram_chain(int32_t N, const int64_t *dims, const int32_t *ranks, int32_t n,
                        const double *const *Z_dev, double *Q_dev, int32_t accumulate,
                        void *ws, size_t ws_bytes, void *hip_stream);

/* Batch TR-ALS with normal equations (Alg. 2) on the device over a whole
 * tensor X (I_1 x .. x I_{N-1} x T, FP64, host or device): the "Hot" batch
 * baseline of the experiments (Sec. 4) when started from the previous
 * cores, or a cold start from the counter-based random cores (cores_in
 * NULL, stream kind 2 of cfg->seed).  cfg gives order, dims, ranks,
 * compute_dtype, seed and device/stream (its sketch fields are ignored).
 * Sweeps: modes 1..N in order, each solving G_{n(2)} H^{!=n}_<2> = M_n with
 * the pseudo-inverse rule; it stops when the relative error changes by less
 * than tol between sweeps or after max_sweeps.  cores_out: N host buffers
 * in the column-major core layout (core N-1 with T slices).  rel_errs (host,
 * may be NULL) receives the error of the start and after each sweep
 * (*sweeps_done + 1 values, at most max_sweeps + 1); synchronous.          */
tr_status tr_batch_als(const tr_config *cfg, const double *X, int64_t T, int32_t x_is_device,
                       const double *const *cores_in, int32_t cores_on_device,
                       int32_t max_sweeps, double tol, double *const *cores_out,
                       double *rel_errs, int32_t *sweeps_done);

/* Fit loss 1/2 ||TR(G) - X||_F^2 by direct residual; *loss_dev (FP64,
 * device) is written on the stream.                                       */
tr_status tr_fit_loss_fwd(int32_t N, const int64_t *dims, const int32_t *ranks,
                          int32_t dt, const void *X, const void *const *cores,
                          double *loss_dev, void *ws, size_t ws_bytes, void *hip_stream);

/* Core gradients of the fit loss, grads[n] = grad_scale * (G_{n(2)} Q_n - P_n)
 * folded to the column-major core layout in dtype dt (device).            */
tr_status tr_fit_loss_bwd(int32_t N, const int64_t *dims, const int32_t *ranks,
                          int32_t dt, const void *X, const void *const *cores,
                          double grad_scale, void *const *grads, void *ws,
                          size_t ws_bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TR_STREAM_H */
