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
 *     roots refined by Newton steps, multiplication by 1/c instead of
 *     division, and fused multiply-adds; results agree with the exact
 *     evaluation to a relative residual far below 1e-12.
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
 * Returns 0 for invalid sizes.  The workspace holds the private copy of V
 * and the per-row rotation coefficients; it needs 256-byte alignment.
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

#ifdef __cplusplus
}
#endif

#endif /* CHOLMOD_MI355X_H */
