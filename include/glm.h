/*
 * glm.h -- C interface of the MI355X (gfx950) library that evaluates the
 * Bayesian logistic-regression log-posterior and its gradient in one fused
 * pass over a tall design matrix.
 *
 * The quantity (Mahani & Sharabiani, "SIMD Parallel MCMC Sampling with
 * Applications for Big-Data Bayesian Analytics"):
 *
 *   u_n  = x_n . beta                                   (the "LA map", Sec. 3.2)
 *   f    = sum_n [ y_n u_n - softplus(u_n) ]            (Sec. 3.1.1, eq-loglike-binlogit,
 *          - prec/2 |beta - m|^2                         rewritten; Gaussian prior on beta)
 *   g    = sum_n (y_n - sigmoid(u_n)) x_n               (Sec. 4.2, eq-grad-expanded /
 *          - prec (beta - m)                             eq-grad-compact: X^t g_f)
 *
 * The paper's routine takes beta, X, y, N, K and returns f while writing g
 * (Sec. 4.2, the loglike_fg routines); glm_logpost_grad keeps that contract
 * with device buffers and an explicit stream, glm_logpost_grad_host keeps it
 * with host buffers.  The Gaussian prior's parameters are left open in
 * Sec. 3.1.1; here it is N(m, prec^-1 I) with the normalising constant
 * dropped, so f(0) = -N ln 2 when m = 0.
 *
 * Conventions for every call:
 *   - Every function returns a glm_status: GLM_OK (0), GLM_PENDING (1, only
 *     from glm_server_poll) or a negative error code.  On an error nothing is
 *     launched and no output is written; glm_last_error() returns a message
 *     describing the last error raised on the calling thread.
 *   - "device" pointers are addresses in the GPU memory of the context's
 *     device (hipMalloc, or a torch CUDA tensor's data_ptr()); "host"
 *     pointers are ordinary process memory.  The library never frees memory
 *     it did not allocate.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Device-buffer calls are asynchronous and stream-ordered: the output is
 *     valid once the stream has reached the call.
 *   - Results are FP64.  For a fixed data set, launch plan and input, a call
 *     is bitwise reproducible (all reductions run in a fixed order; no
 *     floating-point atomics).
 *   - No C++ exception crosses this interface.
 */
#ifndef GLM_H
#define GLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t glm_status;

#define GLM_OK           0
#define GLM_PENDING      1   /* glm_server_poll: the ticket is not finished yet   */
#define GLM_EINVAL      -1   /* an argument is out of range or a pointer is NULL  */
#define GLM_EDTYPE      -2   /* unknown storage dtype                               */
#define GLM_EHIP        -3   /* a HIP runtime call or kernel launch failed          */
#define GLM_ENOTFOUND   -4   /* unknown data set id, group set or ticket            */
#define GLM_EBUDGET     -5   /* a data set does not fit the server's HBM budget     */
#define GLM_ECANCELLED  -6   /* the server was destroyed before the ticket finished */
#define GLM_EAGAIN      -7   /* the server's request ring is full; retry            */
#define GLM_ENOMEM      -8   /* device or host allocation failed                    */

/* Storage type of X.  F64 and F32 are IEEE binary64 / binary32; BF16 is the
 * upper half of a binary32; FP8_E4M3 is the OCP E4M3FN byte (bias 7, max
 * +-448, no infinities) multiplied by a per-column FP32 scale. */
typedef enum {
    GLM_F64 = 0,
    GLM_F32 = 1,
    GLM_BF16 = 2,
    GLM_FP8_E4M3 = 3
} glm_dtype;

/* Response model (the per-row map; the linear algebra is the same for all,
 * as the paper notes for GLMs other than the logistic one, Sec. 3.4):
 *   GLM_LOGISTIC  y in {0, 1}:  t = y u - softplus(u),  r = y - sigmoid(u)
 *                 (Sec. 3.1.1, eq-loglike-binlogit)
 *   GLM_POISSON   y in {0 .. 255} (counts, log link):  t = y u - exp(u),
 *                 r = y - exp(u); the constant -sum_n log(y_n!) is left out
 * f = sum_n t_n - prior,  g = sum_n r_n x_n - prior gradient. */
typedef enum {
    GLM_LOGISTIC = 0,
    GLM_POISSON = 1
} glm_family;

/* Largest number of columns K any entry point accepts. */
#define GLM_K_MAX 4096

typedef struct glm_ctx glm_ctx;
typedef int64_t glm_dataset_id;

/* A data set: X (N x K, row-major, element (n,k) at X[n*ldx + k]) and the
 * response y of the chosen family.  All pointers are device pointers owned by the caller,
 * who keeps them alive and unchanged until the data set is unregistered.
 *   X          device, N*ldx elements of dtype (may be NULL when N == 0)
 *   ldx        leading dimension in elements, ldx >= K
 *   dtype      a glm_dtype
 *   col_scale  device, K FP32 scales s_k (value = code * s_k); FP8_E4M3 only,
 *              must be NULL for the other dtypes
 *   y          device, N bytes: 0 or 1 for GLM_LOGISTIC (other values:
 *              result undefined), counts 0..255 for GLM_POISSON
 *   N          rows, N >= 0 (N == 0 evaluates the prior alone)
 *   K          columns, 1 <= K <= GLM_K_MAX and K * sizeof(dtype) <= 4096
 *              bytes (F64 512, F32 1024, BF16 2048, FP8 4096 columns)
 *   family     a glm_family
 * The kernels read rows as 16-byte chunks, so rows must start on 16-byte
 * boundaries: X 16-byte aligned and ldx * sizeof(dtype) a multiple of 16
 * (glm_dataset_register rejects other layouts with GLM_EINVAL).  K itself is
 * free: columns K .. ldx-1 may hold anything and are never used. */
typedef struct {
    const void* X;
    int64_t ldx;
    int32_t dtype;
    const float* col_scale;
    const uint8_t* y;
    int64_t N;
    int32_t K;
    int32_t family;   /* a glm_family; 0 (zero-initialised) is logistic */
} glm_dataset_desc;

/* Gaussian prior N(m, prec^-1 I) on beta (Sec. 3.1.1 leaves it open).
 *   prec   precision 1/sigma^2 >= 0 (0 = flat prior)
 *   mean   NULL (zero mean), or K doubles (device for device-buffer calls,
 *          host for the _host call); for glm_logpost_grad_batched, G x K
 *          doubles when mean_per_group != 0. */
typedef struct {
    double prec;
    const double* mean;
    int32_t mean_per_group;
} glm_prior;

/* ------------------------------------------------------------------ context */

/* Creates a context on HIP device `device` (ordinal).  The context owns the
 * per-stream scratch buffers (partial sums and completion counters) and the
 * launch plans.  Errors: GLM_EINVAL (out NULL, bad ordinal), GLM_EHIP. */
glm_status glm_create(int device, glm_ctx** out);

/* Frees everything the context allocated, after synchronising its device.
 * Data sets and group sets still registered are released (not the caller's
 * buffers).  NULL is accepted.  Everything is freed even when a HIP call
 * fails; the first failure is then returned as GLM_EHIP (its message in
 * glm_last_error) after the context is gone. */
glm_status glm_destroy(glm_ctx* ctx);

/* Context options: launch-shape choices that change row order or kernel
 * form, so that two contexts with the same options give the same bits.
 *   GLM_OPT_BLOCKS_PER_CU  persistent-grid blocks per compute unit, 1..8
 *                          (default 1); read when a data set is registered
 *                          (it fixes that set's plan and merge shape).
 *   GLM_OPT_INTERLEAVE     1 (default): the waves sweep row batches grid-
 *                          strided; 0: one contiguous range per wave.  Read
 *                          at registration.
 *   GLM_OPT_MATRIX_CORES   1 (default): BF16 passes of 3 or more vectors with
 *                          rows of at most 512 columns run the linear
 *                          predictors on the matrix cores; 0: on the VALU.
 *                          Read when a several-beta kernel is chosen (each
 *                          glm_logpost_grad_multi call; a server's data set
 *                          when it is added).
 * Errors: GLM_EINVAL (NULL ctx or value pointer, unknown option, value out of
 * range). */
enum {
    GLM_OPT_BLOCKS_PER_CU = 1,
    GLM_OPT_INTERLEAVE = 2,
    GLM_OPT_MATRIX_CORES = 3
};
glm_status glm_set_option(glm_ctx* ctx, int32_t option, int64_t value);
glm_status glm_get_option(glm_ctx* ctx, int32_t option, int64_t* value);

/* Message for the last error raised on the calling thread ("" if none). */
const char* glm_last_error(void);

/* --------------------------------------------------------------- data sets */

/* Validates desc, picks the launch plan (kernel instance from dtype, K and
 * alignment; grid size from the device's compute-unit count and the tuning
 * cache) and returns an id.  The data are not read here.  Errors: GLM_EINVAL
 * (N < 0, K out of range, ldx < K, NULL X or y with N > 0, X not 16-byte
 * aligned or ldx * sizeof(dtype) not a multiple of 16, col_scale missing
 * for FP8 or present otherwise), GLM_EDTYPE. */
glm_status glm_dataset_register(glm_ctx* ctx, const glm_dataset_desc* desc,
                                glm_dataset_id* out);

/* Forgets a data set.  Calls already enqueued on a stream still read the
 * caller's buffers, so synchronise before freeing them.  GLM_ENOTFOUND. */
glm_status glm_dataset_unregister(glm_ctx* ctx, glm_dataset_id id);

/* ------------------------------------------------------------ plain call */

/* f and g at one beta (Sec. 4.2): one fused kernel launch streams X once,
 * computes u, the transcendental map and the X^t contribution per row tile,
 * and its last block to finish adds the partial sums of all blocks in a fixed
 * order and the prior.
 *   beta   device, K doubles
 *   prior  host struct; prior->mean is a device pointer (K doubles) or NULL
 *   out    device, 1 + K doubles: out[0] = f, out[1 + k] = g_k
 *   stream hipStream_t or NULL
 * Calls on one stream run one after another; concurrent calls on different
 * streams are safe (each stream has its own scratch).  A NaN or Inf in beta
 * propagates into the result.  Errors: GLM_EINVAL, GLM_ENOTFOUND, GLM_EHIP,
 * GLM_ENOMEM (scratch growth). */
glm_status glm_logpost_grad(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                            const glm_prior* prior, double* out, void* stream);

/* The plain call for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, kernel, launch shape and result bits as
 * glm_logpost_grad, but the block partials and tickets live in a static
 * device array of 4 MiB per GPU (1,024 tickets; held until the process
 * ends), set up once per device by glm_create, so this call allocates and
 * frees nothing.  The array's tickets are zero between calls (each launch
 * resets them); its partials keep the last call's values.
 *   The launch needs 4 KiB + 8 (nblocks + ngroups)(1 + K) bytes, where
 *   nblocks is at most one block per compute unit (256) and ngroups about
 *   sqrt(nblocks): every K up to 1,900 fits at any N, wider rows only at
 *   small N.  Larger needs return GLM_EINVAL (use glm_logpost_grad).
 * Every such call on one GPU shares the one array: calls that may overlap
 * on the device (different streams, or different contexts on the same GPU)
 * race and give wrong results; serialise them on one stream.
 * Errors: GLM_EINVAL, GLM_ENOTFOUND, GLM_EHIP. */
glm_status glm_logpost_grad_noalloc(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                                    const glm_prior* prior, double* out, void* stream);

/* Several coefficient vectors on one data set (e.g. many MCMC chains): f and
 * g for each of betas[0..nb-1], with X streamed once per pass of up to 8
 * vectors (the pass width is the largest of 8, 4, 2 that the instance's
 * register budget allows for this K and dtype; larger nb runs several passes).
 * For BF16 storage with 65 <= K <= 512 and nb >= 3 a pass holds 4 vectors and
 * their linear predictors X beta run on the matrix cores, with each beta
 * split into four BF16 pieces (about 32 significant bits); the result has the
 * accuracy of the other storage forms' FP32 hi/lo split.
 *   betas  device, nb x K doubles
 *   prior  host struct; prior->mean NULL (zero) or device nb x K doubles
 *          (row b is the mean for betas row b); prec shared
 *   out    device, nb x (1 + K) doubles, row b = [f_b, g_b]
 * A vector's result does not depend on the other vectors of its pass.
 * Errors: as glm_logpost_grad. */
glm_status glm_logpost_grad_multi(glm_ctx* ctx, glm_dataset_id id, const double* betas,
                                  int32_t nb, const glm_prior* prior, double* out, void* stream);

/* Host-buffer form mirroring the paper's routine: copies beta (and the
 * prior mean, if any) to the device, launches and waits; the kernel writes f
 * and g straight into the context's coherent pinned staging memory, from
 * which they are copied to f and g_host (no device-to-host copy).
 *   beta_host  K doubles;  prior->mean host K doubles or NULL
 *   f          host double;  g_host  host K doubles (may be NULL)
 * Uses the context's own stream.  Same errors as glm_logpost_grad. */
glm_status glm_logpost_grad_host(glm_ctx* ctx, glm_dataset_id id,
                                 const double* beta_host, const glm_prior* prior,
                                 double* f, double* g_host);

/* ------------------------------------------------------- batched (groups) */

/* Hierarchical model (Sec. 4.1): G groups, each with its own rows of one
 * stacked data set and its own coefficient vector beta_g; group g's
 * log-likelihood is the plain one over rows offsets[g] .. offsets[g+1]-1.
 * The groups are conditionally independent given the shared prior
 * parameters (Sec. 2.3, Theorem 2.1), so one launch evaluates all of them. */
typedef struct glm_groupset glm_groupset;

typedef struct {
    int64_t tile_rows;   /* groups longer than this are split into tiles        */
    int32_t blocks;      /* grid size of the persistent launch                   */
    int32_t waves;       /* waves that share the static work schedule            */
    int32_t items;       /* scheduled work items (whole groups + tiles)          */
    int32_t split_tiles; /* tiles of split groups (partials merged in-kernel)    */
    double tuned_us;     /* measured time of the chosen shape (0 if not tuned)   */
} glm_groupset_info;

/* Builds the static schedule of a group set.  concat describes the stacked
 * data (same rules as glm_dataset_register; the caller owns the buffers and
 * keeps them alive until the group set is destroyed).  offsets_host: G + 1
 * host int64, offsets[0] = 0, non-decreasing, offsets[G] = concat->N (empty
 * groups allowed: their result is the prior alone).  tune != 0 times the
 * candidate tile lengths and grid sizes on this group set at beta = 0 and
 * keeps the fastest (the choice is cached per shape for the process, and in
 * the file named by GLM_TUNE_CACHE if set); tune == 0 uses the default.
 * Synchronises the device.  Errors: GLM_EINVAL, GLM_EDTYPE, GLM_ENOMEM,
 * GLM_EHIP. */
glm_status glm_groupset_create(glm_ctx* ctx, const glm_dataset_desc* concat,
                               const int64_t* offsets_host, int32_t G, int32_t tune,
                               glm_groupset** out);

/* Frees the group set's device memory after synchronising the device. */
glm_status glm_groupset_destroy(glm_groupset* gs);

/* Shape of the schedule in use. */
glm_status glm_groupset_query(const glm_groupset* gs, glm_groupset_info* info);

/* f_g and g_g for every group in one launch.
 *   betas  device, G x K doubles (row g = beta_g)
 *   prior  host struct: prec, and mean = NULL (zero), K doubles (shared) or,
 *          with mean_per_group != 0, G x K doubles (device)
 *   out    device, G x (1 + K) doubles: row g = [f_g, g_g]
 * Calls on one group set share its scratch (tile partials and tickets), so
 * they must be ordered: issue them on one stream.  Errors: GLM_EINVAL,
 * GLM_EHIP. */
glm_status glm_logpost_grad_batched(glm_ctx* ctx, glm_groupset* gs, const double* betas,
                                    const glm_prior* prior, double* out, void* stream);

/* ----------------------------------------------------------------- server */

/* Request server for many concurrent MCMC chains.  Callers submit f + g
 * requests (one beta each) for registered data sets and collect results by
 * ticket.  A scheduler thread packs queued requests of one data set into a
 * single pass over X that evaluates up to max_beta_per_pass coefficient
 * vectors (glm_logpost_grad_multi's kernels), and keeps up to n_slots
 * launches in flight on n_streams streams: requests arriving while passes run
 * join the next free slot (continuous batching).  The passes of up to
 * max_sets_per_pass data sets that share a kernel geometry (storage type and
 * row width) and have requests queued go into one launch (a fleet launch):
 * small data sets are latency-bound, and one launch then pays that latency
 * for all of them.  A request's result does not depend on which other
 * requests share its pass or its launch (bitwise).
 *
 * Data sets given with host pointers are copied to device memory on first
 * use (admission) if they fit hbm_budget_bytes together with the resident
 * ones; otherwise the least recently used data sets with no pass in flight
 * are evicted first, and if that is not enough the requests wait until
 * passes finish.  Admission runs on a thread and a copy stream of its own
 * (pageable sources through pinned staging buffers, pinned sources
 * directly), so passes over resident data sets go on meanwhile; evicted
 * allocations are kept for reuse within the budget instead of freed.  The
 * latency quantiles come from a fixed histogram of 2 % buckets.  The offload
 * cost of one host round trip (Sec. 4.5) is paid per pass. */
typedef struct glm_server glm_server;

typedef struct {
    uint64_t hbm_budget_bytes;   /* device bytes the server may hold for data sets */
    int32_t max_beta_per_pass;   /* 1..8: coefficient vectors per pass over X       */
    int32_t n_streams;           /* device streams passes rotate over              */
    int32_t n_slots;             /* launches in flight at most                     */
    int32_t queue_capacity;      /* queued requests at most (submit: GLM_EAGAIN)    */
    int32_t max_sets_per_pass;   /* data sets per launch at most: 1 = one per
                                    launch; 0 = the default, 32; at most 256        */
} glm_server_config;

typedef struct {
    uint64_t submitted, completed, cancelled, failed;
    uint64_t passes;             /* passes launched (one data set each)             */
    uint64_t betas_in_passes;    /* requests served by them                         */
    uint64_t admissions, evictions;
    uint64_t resident_bytes;
    int32_t resident_datasets;
    int32_t queue_depth;
    uint64_t pass_width_hist[9]; /* [w] = passes that carried w requests (1..8)     */
    double latency_p50_us;       /* submit -> result ready, finished requests       */
    double latency_p99_us;
    double latency_mean_us;
    uint64_t launches;           /* kernel launches that carried the passes         */
    uint64_t bytes_streamed;     /* sum over passes of N (K size + 1): X and y read */
    uint64_t bytes_admitted;     /* data-set bytes copied to HBM by admissions      */
    double admit_seconds;        /* time the admission thread spent on them         */
    uint64_t cached_bytes;       /* evicted allocations kept for reuse (they count
                                    against the budget and are released as needed) */
    uint64_t bytes_staged;       /* of bytes_admitted, copied through the pinned
                                    staging buffers (pageable sources)              */
} glm_server_metrics;

/* Starts the scheduler thread.  Errors: GLM_EINVAL, GLM_EHIP. */
glm_status glm_server_create(glm_ctx* ctx, const glm_server_config* cfg, glm_server** out);

/* Registers a data set with the server.  on_device == 0: desc holds host
 * pointers (X, y, col_scale) that the caller keeps valid until the server is
 * destroyed; the server copies them to HBM when needed.  on_device != 0:
 * device pointers, always resident (counted in the budget, never evicted).
 * Errors: as glm_dataset_register; GLM_EBUDGET if the data set does not fit
 * the budget beside the device-resident data sets already added (then a
 * host-sourced one could never be admitted). */
glm_status glm_server_add_dataset(glm_server* srv, const glm_dataset_desc* desc, int32_t on_device,
                                  glm_dataset_id* out);

/* Queues one request; copies beta (K doubles, host) and the prior mean (K
 * doubles, host, or NULL for zero), so the caller may reuse its buffers.
 * Thread-safe.  Errors: GLM_ENOTFOUND (data set), GLM_EAGAIN (queue full),
 * GLM_ECANCELLED (server shutting down), GLM_EINVAL. */
glm_status glm_server_submit(glm_server* srv, glm_dataset_id ds, const double* beta_host,
                             double prec, const double* mean_host, uint64_t* ticket);

/* Queues n requests at once (all or none): request i is for data set ds[i]
 * with coefficient vector betas[i] (host, K doubles of that data set),
 * precision precs[i] and zero prior mean.  tickets: n entries out.
 * Errors: GLM_EAGAIN if the queue cannot take all n, else as
 * glm_server_submit. */
glm_status glm_server_submit_many(glm_server* srv, int32_t n, const glm_dataset_id* ds,
                                  const double* const* betas, const double* precs,
                                  uint64_t* tickets);

/* Waits for n tickets and retires them; f_out (n doubles, may be NULL)
 * receives f of each finished request (NaN for a cancelled or failed one).
 * Returns GLM_OK if all finished normally, else the first error met. */
glm_status glm_server_wait_many(glm_server* srv, int32_t n, const uint64_t* tickets, double* f_out);

/* Non-blocking: GLM_PENDING if not finished; GLM_OK copies f and g (K
 * doubles, host; either may be NULL) and retires the ticket; GLM_ECANCELLED
 * for a request dropped by shutdown (also retired); GLM_ENOTFOUND for an
 * unknown or retired ticket. */
glm_status glm_server_poll(glm_server* srv, uint64_t ticket, double* f, double* g_host);

/* As glm_server_poll but blocks until the request is finished. */
glm_status glm_server_wait(glm_server* srv, uint64_t ticket, double* f, double* g_host);

glm_status glm_server_stats(glm_server* srv, glm_server_metrics* out);

/* Clears the counters and latency record (not the queue). */
glm_status glm_server_reset_stats(glm_server* srv);

/* Stops accepting requests, cancels queued ones and waits for passes in
 * flight; results of finished requests stay available to poll. */
glm_status glm_server_shutdown(glm_server* srv);

/* Shuts down (if needed) and frees the server and its device copies. */
glm_status glm_server_destroy(glm_server* srv);

/* --------------------------------------------------------------- Hessian */

/* f, g and the Hessian H = -X^t W X - prec I at one beta (the paper names the
 * Hessian as the next derivative to fuse, Sec. 5.2), W = diag(w_n) with
 * w_n = sigmoid(u_n)(1 - sigmoid(u_n)) for GLM_LOGISTIC and exp(u_n) for
 * GLM_POISSON.  Device pointers: beta (K), prior mean as for
 * glm_logpost_grad, out (1 + K: f then g, as glm_logpost_grad), H (K x K
 * doubles, row-major, symmetric).  H is computed on the matrix cores in FP64
 * (products and sums) from each row's w_n, which the fused f+g pass writes;
 * the library keeps per-stream buffers of N + O(K^2) doubles for that.
 * Async on `stream`; bitwise reproducible.  Errors: GLM_EINVAL,
 * GLM_ENOTFOUND, GLM_ENOMEM, GLM_EHIP. */
glm_status glm_logpost_grad_hess(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                                 const glm_prior* prior, double* out, double* H, void* stream);

/* ----------------------------------------------- differential update */

/* One-coefficient-at-a-time samplers (slice sampling or Gibbs over the
 * coordinates of beta) change a single beta_k per step.  With u = X beta kept
 * on the device, f(beta + delta e_k) needs column k of X, u and y only:
 * u' = u + delta X_k (Sec. 3.4.4, the differential update).  The calls below
 * work on a column-major copy of X (a column set) so that column k is one
 * contiguous stream: N (sizeof(dtype) + 8 + 1) bytes per evaluation instead
 * of N (K sizeof(dtype) + 1).
 *
 * Column set: element (n, k) at Xt[k*ldt + n]; ldt >= N; Xt aligned to its
 * element; the other fields as in glm_dataset_desc.  All pointers are device
 * pointers owned by the caller and kept alive until unregistered. */
typedef struct {
    const void* Xt;
    int64_t ldt;
    int32_t dtype;
    const float* col_scale;
    const uint8_t* y;
    int64_t N;
    int32_t K;
    int32_t family;
} glm_colset_desc;

/* Writes the column-major copy of a row-major data set's X into Xt (device,
 * K*ldt elements of the same dtype, caller-owned; ldt >= N), bit for bit.
 * Async on `stream`.  Errors: GLM_EINVAL (as glm_dataset_register, or
 * ldt < N, Xt NULL/misaligned), GLM_EDTYPE, GLM_EHIP. */
glm_status glm_transpose(glm_ctx* ctx, const glm_dataset_desc* rows, void* Xt, int64_t ldt,
                         void* stream);

/* Registers a column set (FP8: the K scales are read once, here).  Errors:
 * GLM_EINVAL (N < 0, K out of range, ldt < N, NULL/misaligned Xt or y with
 * N > 0, col_scale missing for FP8 or present otherwise), GLM_EDTYPE,
 * GLM_EHIP. */
glm_status glm_colset_register(glm_ctx* ctx, const glm_colset_desc* desc, glm_dataset_id* out);
glm_status glm_colset_unregister(glm_ctx* ctx, glm_dataset_id id);

/* u = X beta (device: beta K doubles in, u N doubles out), FP64 products
 * and sums in column order.  Async.  Errors: GLM_EINVAL, GLM_ENOTFOUND,
 * GLM_EHIP. */
glm_status glm_linpred(glm_ctx* ctx, glm_dataset_id colset, const double* beta, double* u,
                       void* stream);

/* f(beta + delta_j e_k) for j < nd (Sec. 3.4.4 with the log-posterior of
 * Sec. 3.1.1): device u = X beta (N doubles), beta (K doubles), deltas (nd
 * doubles) and f_out (nd doubles).  Each pass reads column k, u and y once
 * for up to 16 step sizes.  Per-row terms and all sums in FP64; the prior is
 * evaluated at beta + delta_j e_k.  Async; bitwise reproducible.  Errors:
 * GLM_EINVAL (NULL, nd < 1, k outside [0, K), prec < 0), GLM_ENOTFOUND,
 * GLM_ENOMEM, GLM_EHIP. */
glm_status glm_diff_logpost(glm_ctx* ctx, glm_dataset_id colset, const double* u,
                            const double* beta, int32_t k, const double* deltas, int32_t nd,
                            const glm_prior* prior, double* f_out, void* stream);

/* Commits a step: u += delta X_k and, when beta is not NULL, beta_k += delta
 * (device pointers; delta is one device double, so a device-side sampler can
 * produce it without a host round trip).  The new u equals, bit for bit, the
 * u' that glm_diff_logpost evaluated for the same delta.  Async.  Errors:
 * GLM_EINVAL, GLM_ENOTFOUND, GLM_EHIP. */
glm_status glm_diff_commit(glm_ctx* ctx, glm_dataset_id colset, double* u, double* beta,
                           int32_t k, const double* delta, void* stream);

/* ------------------------------------------------ on-device sampler loop */

/* Runs n_steps of random-walk Metropolis on the device without host
 * round trips (Sec. 4.5 measures the round trip that this removes; the
 * accept rule is the Metropolis step of Sec. 2.2):
 *   beta' = beta + incs[t*K .. t*K+K-1];  accept iff logu[t] < f(beta') - f(beta)
 * All pointers are device pointers.  beta (K doubles) is the starting point
 * on entry and the chain's last state on return; fg (1 + K doubles) receives
 * f and g at the last state.  incs (n_steps x K) and logu (n_steps) are the
 * proposal increments and log-uniforms, drawn by the caller.  accepted
 * (n_steps bytes, 0/1) and f_trace (n_steps doubles: f of the state after
 * step t) may be NULL.  Async on `stream`; the kernels run in stream order,
 * one fused evaluation per step.  Chains on different streams are
 * independent; two calls on one stream must not overlap in time from
 * different host threads.  Errors: GLM_EINVAL, GLM_ENOTFOUND, GLM_ENOMEM,
 * GLM_EHIP. */
glm_status glm_mh_run(glm_ctx* ctx, glm_dataset_id id, double* beta, double* fg,
                      const double* incs, const double* logu, int32_t n_steps,
                      const glm_prior* prior, uint8_t* accepted, double* f_trace, void* stream);

/* Runs n_iter iterations of Hamiltonian Monte Carlo on the device (Sec. 4.2
 * names HMC among the samplers that consume the gradient; the leapfrog
 * integrator and the Metropolis correction are the standard ones, R. M. Neal,
 * "MCMC using Hamiltonian dynamics", 2011).  Each iteration draws momenta
 * p ~ N(0, I), takes n_leap leapfrog steps of size eps on
 * H = -f(beta) + |p|^2 / 2 (one fused f + g evaluation per step, whose last
 * block moves momenta and position) and accepts iff
 * log U < H(start) - H(end).  Momenta and U come from the counter-based
 * streams of glm_rng_fill with key (seed, chain): iteration t's momenta are
 * the normals of purpose 16, stream t; its U is word 0 of the block at
 * counter (0, 0, 17, t); so the chain is reproducible off the device.  The
 * iterations are t = iter0 .. iter0 + n_iter - 1: a chain run in pieces
 * (iter0 = the iterations already run, beta = its state) is the same chain.
 *   beta   device, K doubles: the start on entry, the last state on return
 *   fg     device, 1 + K doubles: f and g at the last state
 *   accepted (n_iter bytes) and f_trace (n_iter doubles: f of the state
 *   after iteration t): device, may be NULL
 * Async on `stream`, n_iter * n_leap + 1 fused launches and no host round
 * trip.  Errors: GLM_EINVAL (n_leap < 1, eps not > 0, iter0 + n_iter >= 2^32,
 * ...), GLM_ENOTFOUND,
 * GLM_ENOMEM, GLM_EHIP. */
glm_status glm_hmc_run(glm_ctx* ctx, glm_dataset_id id, double* beta, double* fg, int32_t n_iter,
                       int32_t n_leap, double eps, uint64_t seed, uint64_t chain, uint32_t iter0,
                       const glm_prior* prior, uint8_t* accepted, double* f_trace, void* stream);

/* ------------------------------------------------------- random numbers */

/* Batch generation of random deviates on the device (the paper's batch RNG,
 * Sec. 4.4 and Sec. 5.2, with the buffers filled by the GPU): values
 * offset .. offset + n - 1 of one stream of the counter-based generator
 * Philox4x64-10 (Salmon et al., SC'11) under key (seed, chain):
 *   GLM_RNG_UNIFORM      U_i = ((w >> 12) + 1/2) 2^-52 in (0, 1), w = word
 *                        i mod 4 of the block at counter (i / 4, 0, 1, stream_id)
 *   GLM_RNG_LOG_UNIFORM  log U_i of the same U_i (e.g. Metropolis accept tests)
 *   GLM_RNG_NORMAL       scale * z_i, standard normals by Marsaglia's polar
 *                        method: pair p tries blocks at counter
 *                        (p, a / 2, 2, stream_id), words 2 (a mod 2) and
 *                        2 (a mod 2) + 1, as u, v = 2 U - 1, until
 *                        0 < s = fma(u, u, v v) < 1; then z = (u, v) c with
 *                        c = sqrt(-2 log(s) / s)
 * (UNIFORM and LOG_UNIFORM values are scaled by 1, not by scale.)  Any value
 * depends only on its index, so fills of adjacent ranges join seamlessly.
 *   out  device, n doubles.  Async on `stream`.
 * Errors: GLM_EINVAL (unknown kind, n < 0, offset + n >= 2^63), GLM_EHIP. */
#define GLM_RNG_UNIFORM      1
#define GLM_RNG_NORMAL       2
#define GLM_RNG_LOG_UNIFORM  3
glm_status glm_rng_fill(glm_ctx* ctx, int32_t kind, uint64_t seed, uint64_t chain,
                        uint64_t stream_id, uint64_t offset, int64_t n, double scale, double* out,
                        void* stream);

/* -------------------------------------------------------- boundary probe */

/* The offload round trip the paper measures on its GPU (Sec. 4.5): copy K
 * doubles host -> device, launch an empty kernel, copy one double back and
 * wait, `iters` times on the context's stream with pinned host buffers.
 * Writes the mean microseconds per round trip to *us.  This is the latency
 * floor of any host-driven evaluation (glm_logpost_grad_host).  Errors:
 * GLM_EINVAL (K < 1, iters < 1, NULL us), GLM_EHIP. */
glm_status glm_probe_roundtrip(glm_ctx* ctx, int32_t K, int32_t iters, double* us);

/* The measured read ceiling that the fused kernels' bandwidth is compared
 * with: a plain streaming read of `bytes` (rounded down to 16) at device
 * address buf (16-byte aligned, caller-owned, only read), by
 * num_CU * blocks_per_cu blocks of 256 lanes with 16-byte nontemporal loads.
 * One untimed pass, then `iters` passes timed with events on the context's
 * stream; writes the achieved GB/s (1e9 bytes/s) to *gbps.  Blocks until done.
 * Errors: GLM_EINVAL (NULL, bytes < 16, misaligned, blocks_per_cu outside
 * [1, 16], iters < 1), GLM_ENOMEM, GLM_EHIP. */
glm_status glm_probe_read_bandwidth(glm_ctx* ctx, const void* buf, int64_t bytes,
                                    int32_t blocks_per_cu, int32_t iters, double* gbps);

/* The measured ceiling that the Hessian's matrix-core rate is compared with:
 * 2 blocks per compute unit of 4 waves, each wave issuing `iters` rounds of
 * 16 independent FP64 16x16x4 matrix instructions (no memory traffic), timed
 * with events on the context's stream after one short untimed launch.  Writes
 * the achieved TFLOP/s to *tflops.  Blocks until done.  Errors: GLM_EINVAL
 * (NULL, iters < 1), GLM_ENOMEM, GLM_EHIP. */
glm_status glm_probe_mfma_f64(glm_ctx* ctx, int32_t iters, double* tflops);

/* The measured floor that the differential-update evaluation (Sec. 3.4.4) is
 * compared with: its per-row term t(u) = y u - b(u) for the response family
 * (GLM_LOGISTIC or GLM_POISSON) over n synthetic rows (u spread over
 * [-2, 2.1) by the row index, y from the row index), on the evaluation's
 * grid and block size, with no memory traffic.  One untimed launch, then
 * `iters` launches back to back timed with events on the context's stream;
 * writes the mean microseconds per launch to *us.  Blocks until done.
 * Errors: GLM_EINVAL (NULL, n < 0, iters < 1, unknown family), GLM_ENOMEM,
 * GLM_EHIP. */
glm_status glm_probe_diff_map(glm_ctx* ctx, int64_t n, int32_t family, int32_t iters, double* us);

/* ----------------------------------------------------- storage conversions */

/* BF16 copy of an FP32 matrix, round to nearest even (NaN stays NaN).
 *   X device N x K FP32 (leading dim ldx); Q device N x K uint16 (leading dim ldq).
 * Errors: GLM_EINVAL, GLM_EHIP. */
glm_status glm_quantize_bf16(glm_ctx* ctx, const float* X, int64_t N, int32_t K,
                             int64_t ldx, uint16_t* Q, int64_t ldq, void* stream);

/* Per-column FP8 scales s_k = max_n |x_nk| / 448 in FP32 (1 for an all-zero
 * column), so that the largest magnitude of each column maps to the largest
 * finite E4M3FN value.  X device N x K FP32; scale device K floats. */
glm_status glm_fp8_col_scales(glm_ctx* ctx, const float* X, int64_t N, int32_t K,
                              int64_t ldx, float* scale, void* stream);

/* FP8 E4M3FN codes of x_nk / s_k (FP32 division), round to nearest even,
 * saturating at +-448.  Q device N x K bytes (leading dim ldq). */
glm_status glm_quantize_fp8(glm_ctx* ctx, const float* X, int64_t N, int32_t K,
                            int64_t ldx, const float* scale, uint8_t* Q, int64_t ldq,
                            void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GLM_H */
