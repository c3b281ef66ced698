/*
 * cholmod_mi355x.h -- C ABI of a rank-k Cholesky modification library for
 * AMD Instinct MI355X (gfx950).
 *
 * Operation (Walder 2010, "Rank k Cholesky Up/Down-dating on the GPU",
 * Section 1): given an upper-triangular L with A = L^T L, an n x k matrix V
 * and sigma = +1 (update) or -1 (downdate), overwrite L with the upper
 * triangular L~ (positive diagonal) such that
 *        L~^T L~ = A + sigma V V^T,
 * in O(k n^2) work, using the hyperbolic Compute/Apply rotations of
 * Algorithm 1 (CholeskyModifyB): for every row i in order, Compute the k
 * rotation pairs (c, s) of row i against the k columns of V, then Apply
 * them to the rest of row i of L and to the rows j > i of (a private copy
 * of) V.
 *
 * Layout of every entry point:
 *   L   device pointer, row-major, leading dimension ldl >= max(1, n);
 *       element (i, j), j >= i, lives at L[i*ldl + j].  Only the upper
 *       triangle (j >= i, j < n) is read or written; the strictly lower part
 *       and the padding columns n..ldl-1 are never touched.
 *   V   device pointer, row-major n x k, element (j, m) at V[j*k + m]
 *       (a contiguous (n, k) tensor).  Read only: the library works on a
 *       private copy in the workspace.
 *   Columns of V are processed in ascending order within each row.
 *
 * Ownership: the caller owns L, V, the workspace and the info word; the
 * library keeps no pointer after a call returns (the sync entry points use
 * a library-owned workspace that grows on demand and is kept per device).
 *
 * Errors.  Argument errors are detected on the host before any HIP call
 * and return CHOLMOD_ERR_ARG.  Numerical failures are detected on the
 * device: a Compute step whose old diagonal is not > 0 (BAD_DIAG) or whose
 * radicand L_ii^2 + sigma V_i^2 is not > 0 (NOT_PD: the modified matrix is
 * not positive definite; this includes a zero radicand and NaN).  The first
 * failure in (row, then column) order is reported with its index
 * r*k + m; after a failure the contents of L are unspecified (rows before r
 * are final).  n == 0 or k == 0 is a successful no-op.
 *
 * Modes (flags):
 *   CHOLMOD_FLAG_EXACT: every Compute and Apply is evaluated exactly as
 *     written in Algorithm 1 with IEEE-754 binary64 operations (correctly
 *     rounded sqrt and division, no fused multiply-add).  Slow; intended to
 *     reproduce a serial reference bit for bit.
 *   default (fast): the same rotations, evaluated with reciprocal square
 *     roots refined by a third-order step, multiplication by 1/c instead of
 *     division, and fused multiply-adds; results agree with the exact
 *     evaluation to a relative residual far below 1e-12.  The fast mode runs
 *     one persistent launch per modification (all 16-column passes of V);
 *     its workgroups wait for rotation records and block maps that earlier
 *     workgroups publish; such a wait is bounded, and a launch whose wait ran
 *     out (not expected while the GPU runs the launch) reports
 *     CHOLMOD_ERR_HIP.  A workgroup applies a block four or more blocks
 *     before its own by the block's map -- the block's rotations multiplied
 *     out into one 80 x 80 matrix, applied on the FP64 matrix cores -- which
 *     equals the rotation-by-rotation Apply up to rounding (maps whose
 *     entries exceed 2 in magnitude, as in a downdate close to
 *     indefiniteness, are not used; the last six blocks of a factor have no
 *     maps).
 *   CHOLMOD_FLAG_ROTATIONS: the fast mode with every block applied by its
 *     rotations, which is bit for bit the per-row fast schedule's result.
 */
#ifndef CHOLMOD_MI355X_H
#define CHOLMOD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (return values). */
#define CHOLMOD_OK 0
#define CHOLMOD_ERR_ARG (-1)      /* bad argument, detected on the host */
#define CHOLMOD_ERR_NOT_PD (-2)   /* A + sigma V V^T is not positive definite */
#define CHOLMOD_ERR_BAD_DIAG (-3) /* an input diagonal entry is not > 0 */
#define CHOLMOD_ERR_HIP (-4)      /* HIP runtime error */

/* Flags for the _ex entry points. */
#define CHOLMOD_FLAG_EXACT 1u     /* IEEE evaluation exactly as Algorithm 1 */
#define CHOLMOD_FLAG_BLOCKED 2u   /* force the host-driven per-block schedule */
#define CHOLMOD_FLAG_ROTATIONS 4u /* fast mode: every block by its rotations, no block maps */

/* Storage types for workspace sizing. */
#define CHOLMOD_F64 0
#define CHOLMOD_F32S 1            /* L and V stored in binary32 */

/* Raw value of an info word when no failure occurred. */
#define CHOLMOD_INFO_NONE INT64_MAX

typedef void *cholmod_stream_t;   /* a hipStream_t (NULL = default stream) */

/*
 * Library version, as major*10000 + minor*100 + patch.
 */
int cholmod_version(void);

/* Human-readable text for a status code (static storage). */
const char *cholmod_status_string(int status);

/*
 * Decode a raw device info word (as left in *d_info by an _async call).
 * Returns CHOLMOD_OK, CHOLMOD_ERR_NOT_PD or CHOLMOD_ERR_BAD_DIAG; when a
 * failure is recorded, *row and *col (if non-NULL) receive r and m of the
 * first failing Compute step (r = index / k, m = index % k), else -1.
 */
int cholmod_decode_info(int64_t info, int64_t k, int64_t *row, int64_t *col);

/*
 * Bytes of device workspace needed by the _async/_ex entry points for an
 * n x k problem with the given storage type (CHOLMOD_F64 or CHOLMOD_F32S).
 * Returns 0 for invalid sizes.  The workspace holds the private copy of V,
 * the per-row rotation coefficients and the block maps (38,912 bytes per
 * 64-row block and 16-column pass), and with CHOLMOD_F32S and k > 16 the
 * binary64 values of V that a 16-column pass leaves for the next one (128
 * bytes per row and pair of passes); it needs 256-byte alignment.
 */
size_t cholmod_workspace_bytes(int64_t n, int64_t k, int dtype);

/*
 * Synchronous rank-k modification in FP64 (the headline entry point).
 * Enqueues the whole modification on `stream`, waits for it, and returns
 * the status.  Uses a library-owned workspace (grown with hipMalloc on
 * demand, one per device).  Not safe to call concurrently from several
 * host threads on the same device.
 *   L      device double*, (n, ldl) row-major, modified in place
 *   V      device const double*, (n, k) row-major, unchanged
 *   sigma  +1 update, -1 downdate
 */
int cholmod_update(double *L, const double *V, int64_t n, int64_t k, int64_t ldl,
                   int sigma, cholmod_stream_t stream);

/*
 * Asynchronous form: enqueues the modification on `stream` and returns
 * without waiting.  No allocation; the caller provides the workspace
 * (>= cholmod_workspace_bytes(n, k, CHOLMOD_F64) bytes of device memory,
 * 256-byte aligned) and a device int64 `d_info` that receives the raw info
 * word (decode with cholmod_decode_info after the stream completes).
 * Returns CHOLMOD_OK if the work was enqueued, CHOLMOD_ERR_ARG for bad
 * arguments (nothing enqueued), or CHOLMOD_ERR_HIP.
 */
int cholmod_update_async(double *L, const double *V, int64_t n, int64_t k, int64_t ldl,
                         int sigma, void *ws, size_t ws_bytes, int64_t *d_info,
                         cholmod_stream_t stream);

/* As cholmod_update_async, with CHOLMOD_FLAG_* flags. */
int cholmod_update_ex(double *L, const double *V, int64_t n, int64_t k, int64_t ldl,
                      int sigma, unsigned flags, void *ws, size_t ws_bytes,
                      int64_t *d_info, cholmod_stream_t stream);

/*
 * Allocation-free form of cholmod_update_async, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  The same modification and kernels as
 * cholmod_update_async, bit for bit the same result, but the workspace is a
 * fixed device array inside the library (cholmod_noalloc_max_bytes() bytes,
 * 32 MiB), one copy per device, held until the process ends; the call
 * allocates nothing.  The caller passes L, V, the device info word d_info
 * (raw info word, decode with cholmod_decode_info) and the stream.
 *   Limit: cholmod_workspace_bytes(n, k, CHOLMOD_F64) must not exceed
 *   cholmod_noalloc_max_bytes() (n = 5000, k = 16 needs 3.2 MB; at k = 16,
 *   n up to about 52000); larger problems return CHOLMOD_ERR_ARG before
 *   any HIP call.
 * Every call on one device shares that device's array: calls that overlap
 * in time on one device (different streams, or host threads) race and
 * give undefined results; calls ordered on one stream are safe.  Each call
 * re-initialises every part of the array it uses.
 * Returns CHOLMOD_OK if enqueued, CHOLMOD_ERR_ARG, or CHOLMOD_ERR_HIP.
 */
size_t cholmod_noalloc_max_bytes(void);
int cholmod_update_noalloc(double *L, const double *V, int64_t n, int64_t k, int64_t ldl,
                           int sigma, int64_t *d_info, cholmod_stream_t stream);

/*
 * FP32-storage mode: the same modification (Algorithm 1) with L and V
 * stored in binary32.  The rows of each 64-row diagonal block -- every
 * Compute (w, c, s, 1/c) and the Apply inside the block -- are evaluated in
 * binary64 from the stored values and rounded to binary32 when stored; the
 * Apply of a block's rotations to the columns right of the block runs in
 * binary32 with the coefficients rounded to binary32, or, by the block's
 * map, in binary64 rounded to binary32 when stored.  Accuracy: the
 * relative Frobenius distance to the binary64 factor of the same (binary32)
 * inputs is about 1e-6 (bound tested: 1e-5).  Halves the memory traffic;
 * the serial chain is unchanged.  Layout, ownership and error reporting are
 * those of the FP64 entry points with float in place of double; there is no
 * EXACT mode.
 *   cholmod_update_f32s: synchronous, library-owned workspace.
 *   cholmod_update_f32s_async: caller workspace of at least
 *     cholmod_workspace_bytes(n, k, CHOLMOD_F32S) bytes, device info word.
 */
int cholmod_update_f32s(float *L, const float *V, int64_t n, int64_t k, int64_t ldl,
                        int sigma, cholmod_stream_t stream);
int cholmod_update_f32s_async(float *L, const float *V, int64_t n, int64_t k, int64_t ldl,
                              int sigma, void *ws, size_t ws_bytes, int64_t *d_info,
                              cholmod_stream_t stream);
/* As cholmod_update_f32s_async with flags: 0 or CHOLMOD_FLAG_ROTATIONS. */
int cholmod_update_f32s_ex(float *L, const float *V, int64_t n, int64_t k, int64_t ldl,
                           int sigma, unsigned flags, void *ws, size_t ws_bytes,
                           int64_t *d_info, cholmod_stream_t stream);

/*
 * Batched modification of many independent factors (uneven n, k, sigma and
 * storage type) on one stream.  Each factor is modified exactly as by the
 * single-factor entry point of its storage type (same blocking, same
 * operations), so its result is bit for bit the one it gets alone (with the
 * default flags, or with CHOLMOD_FLAG_ROTATIONS under a plan without block
 * maps).  By default the batch runs as one preparation launch and one
 * persistent launch whose workgroups take the factors' owner items longest
 * factor first (see the launch plans below); the blocks of different
 * factors run concurrently.
 *   descs     HOST array of `count` descriptors (read during the call only);
 *             the factors must not overlap in memory
 *   count     0 .. 65535 (0 is a no-op)
 *   ws        device workspace of at least
 *             cholmod_workspace_bytes_batched(descs, count) bytes, 256-byte
 *             aligned, not used by other work until the stream has passed
 *             this batch
 *   d_info    device int64[count]: raw info word of each factor (decode with
 *             cholmod_decode_info and that factor's k); a failure in one
 *             factor leaves the others unaffected
 * Returns CHOLMOD_OK when enqueued, CHOLMOD_ERR_ARG (nothing enqueued) if any
 * descriptor is invalid, or CHOLMOD_ERR_HIP.  Does not wait for the work; the
 * library keeps a pinned staging buffer per device for the batch tables.
 */
typedef struct cholmod_desc {
  void *L;          /* device double* (CHOLMOD_F64) or float* (CHOLMOD_F32S) */
  const void *V;    /* device, (n, k) row-major, unchanged */
  int64_t n, k, ldl;
  int32_t sigma;    /* +1 update, -1 downdate */
  int32_t dtype;    /* CHOLMOD_F64 or CHOLMOD_F32S */
} cholmod_desc;

/* Workspace bytes of a batch under any launch plan (0 if any descriptor is
 * invalid). */
size_t cholmod_workspace_bytes_batched(const cholmod_desc *descs, int64_t count);

int cholmod_update_batched(const cholmod_desc *descs, int64_t count, void *ws, size_t ws_bytes,
                           int64_t *d_info, cholmod_stream_t stream);

/*
 * Launch plans of batches.  A batch runs under one of two schedules (every
 * result is bit for bit the single-factor one: with block maps as the
 * default single-factor call, without as CHOLMOD_FLAG_ROTATIONS):
 *   CHOLMOD_SCHED_QUEUED   one preparation launch and one persistent launch
 *                          whose workgroups take owner items (the columns
 *                          of block j of factor f, every 16-column pass)
 *                          from a counter;
 *   CHOLMOD_SCHED_STEPPED  one preparation launch and one launch per block
 *                          step (block b of every factor that has one).
 * The queued launch has `grid` workgroups (0 = one per compute unit), takes
 * the items block-major (all factors' block 0, then block 1, ...) or
 * factor-major (every block of the longest factor, then the next), and
 * owners far from the chain sleep 64 x {1, 20, 100} cycles between polls
 * (poll = 0, 1, 2).
 * cholmod_update_batched takes the plan from a table indexed by the batch's
 * dominant (storage type, n bucket, k bucket) -- the bucket with most of
 * the batch's work, n^2 k summed over its factors; n buckets end at 256,
 * 1024, 4096, 16384 (bucket 4: larger), k buckets at 16, 32, 64 (bucket 3:
 * larger).  The table starts with {QUEUED, 0, BLOCK, 2, maps 1} everywhere and is
 * filled by cholmod_set_plan, normally from the plan cache of the
 * library's autotuner (paper_1011_1173_amd/tune.py), which times the
 * candidate plans of each bucket on the GPU.  The served mode uses the
 * table's grid, order and poll with the queued schedule.
 */
#define CHOLMOD_SCHED_QUEUED 0
#define CHOLMOD_SCHED_STEPPED 1
#define CHOLMOD_ORDER_BLOCK 0
#define CHOLMOD_ORDER_FACTOR 1

typedef struct cholmod_plan {
  int32_t schedule;  /* CHOLMOD_SCHED_* */
  int32_t grid;      /* queued: persistent workgroups, 0 = one per compute unit (<= 65536) */
  int32_t order;     /* queued: CHOLMOD_ORDER_* */
  int32_t poll;      /* queued: 0, 1 or 2 */
  int32_t maps;      /* queued: 1 = far blocks by their block maps, 0 = every block by its
                        rotations (the stepped schedule always uses rotations) */
} cholmod_plan;

/* cholmod_update_batched with an explicit plan (NULL: the table's plan).
 * CHOLMOD_ERR_ARG for an invalid plan, otherwise as cholmod_update_batched. */
int cholmod_update_batched_plan(const cholmod_desc *descs, int64_t count,
                                const cholmod_plan *plan, void *ws, size_t ws_bytes,
                                int64_t *d_info, cholmod_stream_t stream);

/* Plan table entries (thread-safe; CHOLMOD_ERR_ARG for a bad index or plan). */
int cholmod_set_plan(int dtype, int n_bucket, int k_bucket, const cholmod_plan *plan);
int cholmod_get_plan(int dtype, int n_bucket, int k_bucket, cholmod_plan *plan);

/* The table buckets of a factor of size n with k columns of V. */
int cholmod_plan_bucket(int64_t n, int64_t k, int *n_bucket, int *k_bucket);

/* Compute units of the current device (0 on error): the grid of a full
 * queued launch. */
int cholmod_compute_units(void);

/*
 * A batch captured once as a HIP graph and replayed: for a fixed set of
 * factors (the same descriptors, pointers and sizes) modified again and
 * again, e.g. serving slots whose L and V contents change between calls.
 * cholmod_batch_graph_create plans the batch, uploads its tables to `ws`
 * (synchronously) and captures the preparation launch and the per-step
 * launches of cholmod_update_batched; cholmod_batch_graph_launch enqueues
 * one replay on `stream`, which modifies every factor by its V and sigma as
 * cholmod_update_batched would (bit for bit the same result), reading the
 * current contents of L and V.  The graph holds kernel launches only.
 *   descs, count, ws, d_info  as for cholmod_update_batched (count >= 1);
 *           the graph keeps ws, d_info and every factor's L and V pointer:
 *           they must stay valid until cholmod_batch_graph_destroy
 * Replays of one graph share its workspace: replays that overlap in time
 * (on different streams) race; replays on one stream are ordered.
 * Returns CHOLMOD_OK, CHOLMOD_ERR_ARG (nothing created or enqueued) or
 * CHOLMOD_ERR_HIP.
 */
typedef struct cholmod_batch_graph cholmod_batch_graph;
int cholmod_batch_graph_create(const cholmod_desc *descs, int64_t count, void *ws,
                               size_t ws_bytes, int64_t *d_info, cholmod_batch_graph **out);
int cholmod_batch_graph_launch(cholmod_batch_graph *g, cholmod_stream_t stream);
int cholmod_batch_graph_destroy(cholmod_batch_graph *g);

/*
 * Out-of-core modification of a factor held in HOST memory (the paper keeps
 * only O(n) of L on the GPU, Section 4; here for factors larger than HBM).
 * L is streamed through the device in row panels of 64 rows: panel b
 * (rows 64b .. 64b+63, columns 64b .. n-1) is copied in before the block
 * step that factors block b and copied back after the next step has applied
 * block b to the columns right of block b+1.  The arithmetic is that of the
 * batched schedule, so the result is bit for bit the one the device entry
 * point of the same storage type gives.  Synchronous: returns when L in
 * host memory holds the result.
 *   L_host  HOST double* (CHOLMOD_F64) or float* (CHOLMOD_F32S), (n, ldl)
 *           row-major upper triangle, modified in place.  Pinned memory
 *           (hipHostMalloc) is copied directly.  Pageable memory goes
 *           through four pinned host buffers of 64 x n elements that the
 *           call allocates and frees, packed and unpacked by host threads
 *   V       DEVICE, (n, k) row-major in the storage type, unchanged
 *   ws      device workspace of at least cholmod_workspace_bytes_ooc(n, k,
 *           dtype) bytes, 256-byte aligned; NULL: the call allocates and
 *           frees it.  Device memory used: 6 panels of 64 x n elements plus
 *           V's copy and the rotation records, O(n (64 + k)).
 *   info    HOST int64* (may be NULL): the raw info word
 * Returns CHOLMOD_OK, CHOLMOD_ERR_NOT_PD / CHOLMOD_ERR_BAD_DIAG (L's rows at
 * and after the failing row are unspecified), CHOLMOD_ERR_ARG before any
 * HIP call for bad arguments, or CHOLMOD_ERR_HIP.
 */
size_t cholmod_workspace_bytes_ooc(int64_t n, int64_t k, int dtype);
int cholmod_update_ooc(void *L_host, const void *V, int64_t n, int64_t k, int64_t ldl,
                       int sigma, int dtype, void *ws, size_t ws_bytes, int64_t *info,
                       cholmod_stream_t stream);

/*
 * Served mode: factors registered once, then a stream of requests (one
 * update or downdate of one factor by a caller-owned V) batched
 * continuously onto one GPU by a library worker thread.
 *   Admission by HBM footprint: the server owns a device arena of
 *   cfg->ws_bytes bytes (its HBM budget besides the factors); a waiting
 *   request joins the next batch when its workspace (cholmod_workspace_bytes
 *   of its n, k and storage type, plus a few hundred bytes of tables) fits
 *   into the arena's free part.  A request that cannot fit into the whole
 *   arena fails with CHOLMOD_ERR_ARG.
 *   Overlap: up to cfg->streams batches are in flight at once, each on its
 *   own non-blocking stream; a batch formed while others run is launched at
 *   once and shares the GPU with them.
 *   Order: requests of one factor run in submission order (a factor's next
 *   request waits for the previous one); requests of different factors run
 *   concurrently, oldest first.  Each batch is cholmod_update_batched's
 *   schedule, so each result is bit for bit the single-factor result.
 *   Completion: a request completes as soon as its factor is finished in
 *   its batch (the device writes the factor's status into host-mapped
 *   memory), not when the whole batch ends.
 * The arena, streams and pinned memory are allocated by
 * cholmod_server_create.
 */
typedef struct cholmod_server cholmod_server;

typedef struct cholmod_server_cfg {
  size_t ws_bytes;    /* HBM budget of the work in flight (>= 4096): one device
                         arena that the batches in flight share; a request is
                         admitted when its workspace fits into the free part */
  int32_t max_batch;  /* most requests per batch (0 = 256, at most 65535) */
  int32_t device;     /* HIP device of the factors */
  int32_t streams;    /* batches in flight at once, each on its own stream
                         (0 = 4, at most 16) */
  int32_t reserved;   /* 0 */
} cholmod_server_cfg;

/* Create a server and start its worker.  CHOLMOD_ERR_ARG for a bad cfg. */
int cholmod_server_create(const cholmod_server_cfg *cfg, cholmod_server **out);

/*
 * Register a device factor (caller-owned, stays valid until the server is
 * destroyed; only the server modifies it meanwhile).  *id receives its index.
 * CHOLMOD_ERR_ARG for a bad size or dtype, including an n * ldl whose byte
 * count does not fit in int64.
 */
int cholmod_server_add_factor(cholmod_server *srv, void *L, int64_t n, int64_t ldl, int dtype,
                              int32_t *id);

/*
 * Queue the modification of factor `id` by V (device, (n, k) row-major, in
 * the factor's storage type; caller-owned and unchanged until the request
 * completes).  *ticket identifies the request.  Never blocks on the GPU.
 * CHOLMOD_ERR_ARG (nothing queued) for an unknown id, a bad k or sigma, a
 * null V, or an n * k whose workspace size does not fit in int64.
 * The server works on its own stream, which waits for no other stream: any
 * GPU work that writes V or the factor must have completed before the call.
 */
int cholmod_server_submit(cholmod_server *srv, int32_t id, const void *V, int64_t k, int sigma,
                          uint64_t *ticket);

/*
 * Non-blocking: returns 1 while the request is pending; 0 once it has
 * completed, with *status its result (CHOLMOD_OK, CHOLMOD_ERR_NOT_PD, ...;
 * CHOLMOD_ERR_ARG if it could not fit the workspace) and *latency_s the
 * host time from submission to completion; the ticket is then released.
 * CHOLMOD_ERR_ARG for an unknown ticket.
 */
int cholmod_server_poll(cholmod_server *srv, uint64_t ticket, int *status, double *latency_s);

/* Wait until every submitted request has completed. */
int cholmod_server_drain(cholmod_server *srv);

/* Drain, stop the worker and free the server's resources. */
int cholmod_server_destroy(cholmod_server *srv);

/*
 * Measurement entry point (not part of a modification): the two latencies
 * that bound the time of one factor, whose rows form a serial chain
 * (Algorithm 1: row i's Compute needs V_i after the Apply of rows < i).
 *   out4[0]  ns per step of the chain of a 64-row block with k columns of V
 *            (one step: Compute of one row for every column, the Apply of
 *            two rows to the next column, one workgroup barrier); a block
 *            takes 64 + k - 1 steps
 *   out4[1]  ns per 64-row block's chain
 *   out4[2]  ns per one-way hand-off of a flag between workgroups on two
 *            different XCDs (device-scope store, polling device-scope load)
 *   out4[3]  the same between two workgroups on one XCD
 * k in 1..16; `blocks` chains (1..100000) and `rounds` round trips
 * (1..1000000) are averaged.  Runs synthetic inputs held in LDS, allocates
 * 4 KB of device memory for the call, and waits for `stream`.  Returns
 * CHOLMOD_OK, CHOLMOD_ERR_ARG, or CHOLMOD_ERR_HIP (also if a bounded wait
 * of the hand-off ran out).
 */
int cholmod_probe_latency(int k, int blocks, int rounds, double *out4, cholmod_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CHOLMOD_MI355X_H */
