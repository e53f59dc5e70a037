/*
 * shiftsolve -- many shifted linear systems on one MI355X (gfx950).
 *
 * The library solves, for thousands of complex shifts sigma_j,
 *
 *     (A - sigma_j I) X_j = B,      G_j = C X_j = C (A - sigma_j I)^{-1} B,
 *
 * following Bosner, Bujanovic and Drmac, "Parallel solver for shifted
 * systems in a hybrid CPU-GPU framework" (arXiv 1708.06290):
 *
 *   1. once per system, an orthogonal reduction to controller-Hessenberg
 *      form (Algorithm 1, Section 2): H = Q^T A Q is m-Hessenberg
 *      (H(i,j) = 0 for i > j + m), R = Q^T B is upper triangular with only
 *      its first m rows nonzero, Ct = C Q;
 *   2. per shift, an RQ factorisation H - sigma I = R_sigma Q_sigma computed
 *      from the last column to the first with an (m+1)-column sliding window
 *      (Section 3.1), of which only R_sigma(1:m,1:m) is kept: the
 *      back-substitution Y_j = R_sigma(1:m,1:m)^{-1} R(1:m,:) is fused into
 *      the last m steps, then X_j = Q_sigma^*(:,1:m) Y_j (Section 3, items 1-3
 *      of the introduction to that section, and the per-shift right-hand-side
 *      variant of Section 3.3) and G_j = Ct X_j.
 *
 * Sign convention: the paper's transfer function is C (sigma I - A)^{-1} B;
 * this library returns G_j = C (A - sigma_j I)^{-1} B, i.e. minus that value.
 *
 * Data conventions used by every entry point:
 *   - matrices are column-major; "ld" arguments are leading dimensions in
 *     elements (ld >= number of rows);
 *   - complex arrays are interleaved (re, im) double pairs, the layout of C99
 *     `double _Complex` and of torch.complex128;
 *   - pointers documented as "device" must point to memory of the GPU that
 *     is current when the call is made; the library never takes ownership of
 *     caller memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls documented as asynchronous enqueue work on it and return.
 *
 * Error convention: 0 on success; a negative value -i means argument i
 * (1-based) is invalid; positive values are SHS_ERR_* codes.  No exception
 * crosses this interface.  shs_strerror() turns any code into text.
 */
#ifndef SHIFTSOLVE_H
#define SHIFTSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHS_ABI_VERSION 2

/* return codes (positive) */
#define SHS_ERR_NOMEM        1  /* device allocation failed or budget exceeded */
#define SHS_ERR_HIP          2  /* a HIP runtime call failed */
#define SHS_ERR_UNSUPPORTED  3  /* shape outside what the kernels support */
#define SHS_ERR_BUSY         4  /* resource in use (serving: queue full) */
#define SHS_ERR_NOTFOUND     5  /* unknown id (serving) */
#define SHS_ERR_TIMEOUT      6  /* wait timed out (serving) */
#define SHS_ERR_CANCELLED    7  /* the request was cancelled (serving) */
#define SHS_ERR_STATE        8  /* the request is not in a state that allows the call (serving) */
#define SHS_ERR_SCRATCH      9  /* the solve needs more than shs_solve_noalloc's static scratch */

/* bytes of the static per-GPU scratch of shs_solve_noalloc */
#define SHS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* per-shift status codes written by shs_solve */
#define SHS_STATUS_OK             0
#define SHS_STATUS_SINGULAR       1  /* a diagonal entry of R_sigma is exactly 0 */
#define SHS_STATUS_NONFINITE      2  /* a NaN or Inf appeared in the result */
#define SHS_STATUS_FALLBACK       3  /* mixed precision did not converge; FP64 result meets tol */
#define SHS_STATUS_NOT_CONVERGED  4  /* mixed precision: even the FP64 result is above tol */

/* solve modes */
#define SHS_MODE_FP64         0  /* FP64 sweep */
#define SHS_MODE_FP32_REFINE  1  /* complex FP32 sweep + FP64 iterative refinement */

/* output selection bits */
#define SHS_OUT_X    1  /* write X (reduced coordinates) */
#define SHS_OUT_G    2  /* write G */
#define SHS_OUT_ETA  4  /* compute the FP64 backward error of every shift */

/* largest supported m (number of inputs, columns of B) */
#define SHS_MAX_M 16

typedef struct shs_handle shs_handle;

typedef struct shs_config {
    int32_t abi_version;   /* must be SHS_ABI_VERSION */
    int32_t flags;         /* reserved, 0 */
    int64_t reserved[6];   /* 0 */
} shs_config;

typedef struct shs_info_t {
    int64_t n, m, p;
    double  reduce_ms;       /* device time of shs_reduce (HIP events) */
    size_t  resident_bytes;  /* device memory the handle owns */
} shs_info_t;

/*
 * Controller-Hessenberg reduction (Algorithm 1, Section 2; the reflector
 * sequence of Section 2.1).
 *
 *   n, m, p   sizes: A is n x n, B is n x m, C is p x n; need 1 <= m <= SHS_MAX_M,
 *             m < n, p >= 0.
 *   A, B, C   column-major FP64 device arrays with leading dimensions lda >= n,
 *             ldb >= n, ldc >= max(1, p); read only; C may be NULL if p == 0.
 *   cfg       NULL for defaults, else abi_version must equal SHS_ABI_VERSION.
 *   stream    HIP stream the reduction runs on.
 *   out       receives a new handle.
 *
 * The call is synchronous with respect to `stream` (it returns after the
 * reduction has finished).  The handle owns device copies of H, R, Ct, the
 * Householder vectors of Q, an FP32 copy of H and the off-diagonal row sums
 * of H; release it with shs_destroy.  The reduced form is sign-normalised:
 * R(i,i) >= 0 and H(j+m, j) >= 0.  Errors: -1..-13 for bad arguments,
 * SHS_ERR_NOMEM, SHS_ERR_HIP.
 */
int shs_reduce(int64_t n, int64_t m, int64_t p,
               const double *A, int64_t lda,
               const double *B, int64_t ldb,
               const double *C, int64_t ldc,
               const shs_config *cfg, void *stream, shs_handle **out);

/*
 * Host-only check of the blocked reduction's launch plan for an n x n system
 * with m inputs and p outputs (the GEMM updates of Algorithms 2-3): the
 * sequence of launches shs_reduce would make is generated without a GPU, and
 * every GEMM's grid, split-K partials and operand extents are checked
 * against the allocations shs_reduce makes.  Returns the number of
 * violations (0: every launch stays inside its buffers), negative for bad
 * arguments; *launches (nullable) receives the number of GEMM launches and
 * msg (msg_len bytes, nullable) the first violation, if any.  Touches no
 * device.
 */
int shs_reduce_check_plan(int64_t n, int64_t m, int64_t p, int64_t *launches, char *msg, int64_t msg_len);

/*
 * Exact number of bytes of device workspace shs_solve needs for `s` shifts
 * with the given mode and outputs (per-shift reflector store, the carried
 * columns and block transforms of the blocked FP64 sweep, the FP32 buffers
 * of the mixed path, the packed copy of the solutions the residual GEMM
 * reads, the residual and bookkeeping).  The serving layer admits work by
 * this figure.
 */
int shs_solve_workspace(const shs_handle *h, int64_t s, int mode, int outputs,
                        size_t *bytes);

/*
 * Solve (H - sigma_j I) X_j = R and form G_j = Ct X_j for j = 0..s-1.
 *
 *   shifts     device, s complex values (interleaved re, im).
 *   mode       SHS_MODE_FP64 or SHS_MODE_FP32_REFINE.
 *   outputs    OR of SHS_OUT_X, SHS_OUT_G, SHS_OUT_ETA (at least X or G).
 *   tol        backward-error target of the mixed mode (e.g. 1e-13); ignored
 *              by SHS_MODE_FP64.
 *   max_iter   refinement iterations before falling back to FP64 (mixed mode).
 *   work       device workspace of work_bytes >= shs_solve_workspace(...), or
 *              NULL to let the library allocate it on `stream` (stream-ordered).
 *   X, ldx     device, n x (s*m) complex, X(:, j*m:(j+1)*m) = X_j in reduced
 *              coordinates (multiply by Q, shs_apply_q, for A's coordinates);
 *              required when SHS_OUT_X is set, else may be NULL.
 *   G, ldg     device, p x (s*m) complex, G(:, j*m:(j+1)*m) = G_j; required
 *              when SHS_OUT_G is set and p > 0.
 *   eta        device, s doubles, the normwise backward error
 *              max_c ||r_c||_inf / (||H - sigma I||_inf ||x_c||_inf + ||R(:,c)||_inf)
 *              with r = R - (H X_j - sigma_j X_j) evaluated in FP64; required
 *              when SHS_OUT_ETA is set or the mode is mixed.
 *   status     device, s int32 SHS_STATUS_* codes, always written.  A bad
 *              shift never fails the call; its outputs are NaN.
 *
 * Mixed mode: the FP32 sweep result is refined until eta <= tol, a shift
 * at a time; a shift whose eta is NaN, does not at least halve per round, or
 * is still above tol after max_iter corrections is recomputed by the FP64
 * sweep (status FALLBACK, or NOT_CONVERGED if that result is above tol as
 * well).  max_iter = 0 sends every shift to the FP64 sweep.
 *
 * Asynchronous on `stream` in both modes: the host never waits inside the
 * call (mixed mode keeps its per-shift lists on the device).  One solve per
 * handle at a time per stream.  s = 0 returns 0 at once, without looking at
 * the output pointers.
 */
int shs_solve(shs_handle *h, int64_t s, const double *shifts,
              int mode, int outputs, double tol, int max_iter,
              void *work, size_t work_bytes,
              double *X, int64_t ldx, double *G, int64_t ldg,
              double *eta, int32_t *status, void *stream);

/*
 * shs_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, arguments and results as shs_solve, with its workspace taken
 * from a static per-GPU array of SHS_NOALLOC_SCRATCH_BYTES (128 MiB) inside
 * the library instead of `work`.  The call makes no hipMalloc, hipFree or
 * other allocation; the array exists on every GPU the library is used on
 * until the process ends (its address is looked up on the first call on a
 * device).
 *
 *   Requests whose shs_solve_workspace bytes exceed SHS_NOALLOC_SCRATCH_BYTES
 *   fail with SHS_ERR_SCRATCH before any work is queued.  The handle's device
 *   must be current (else SHS_ERR_STATE), and phase timing must be off
 *   (shs_set_timing(h, 0), else SHS_ERR_STATE).
 *
 *   All calls on one GPU share that GPU's array: calls whose work can
 *   overlap on the device (different streams, or threads) race and must be
 *   serialised by the caller, e.g. by issuing them on one stream.  The array
 *   keeps the last call's contents; every call clears what it needs cleared.
 */
int shs_solve_noalloc(shs_handle *h, int64_t s, const double *shifts, int mode, int outputs, double tol,
                      int max_iter, double *X, int64_t ldx, double *G, int64_t ldg, double *eta,
                      int32_t *status, void *stream);

/*
 * Transposed systems with unstructured right-hand sides (Section 3.3, the
 * second family of systems of the interpolation method; Algorithm 11 and its
 * continuation): solve
 *
 *     (H - sigma_j I)^T Y_j = D_j,   j = 0 .. s-1,
 *
 * in reduced coordinates (for (A - sigma I)^T x = c take D = Q^T c, e.g.
 * D = Ct^T c_hat for c = C^T c_hat; then x = Q Y, shs_apply_q).  The
 * transpose is the plain one, not the conjugate transpose.  The matrix
 * (H - sigma I)^T is lower m-Hessenberg; it is factored top-down,
 * (H - sigma I)^T = L Q_sigma, with the forward substitution for L fused
 * into the factorisation, and Y = Q_sigma^* (L^{-1} D) formed afterwards
 * from the stored reflectors.  The library carries this out as the
 * bottom-up RQ sweep of J H^T J - sigma I (J the order-reversing permutation;
 * J H^T J is upper m-Hessenberg) on the reversed right-hand sides, which is
 * the same factorisation in reversed index order; J H^T J is built on the
 * first transposed solve and kept by the handle (n^2 doubles).
 *
 *   shifts   device, s complex.
 *   r        right-hand sides per shift, r >= 1 (processed in groups of m).
 *   D, ldd   device, n x (s*r) complex, D(:, j*r:(j+1)*r) = D_j; read only.
 *   outputs  SHS_OUT_X and/or SHS_OUT_ETA.
 *   work     device workspace of shs_solve_transposed_workspace(h, s, r)
 *            bytes, or NULL (allocated on the stream).
 *   X, ldx   device, n x (s*r) complex, laid out as D (with SHS_OUT_X).
 *   eta      device, s doubles (with SHS_OUT_ETA): the normwise backward
 *            error of the transposed system, max over the shift's columns of
 *            ||r_c||_inf / (||(H - sigma I)^T||_inf ||y_c||_inf + ||d_c||_inf),
 *            r = D_j - (H - sigma_j I)^T Y_j in FP64.
 *   status   device, s int32 SHS_STATUS_* (OK, SINGULAR, NONFINITE).
 *
 * FP64 throughout.  Asynchronous on `stream` (the first call on a handle
 * allocates J H^T J with hipMalloc).  Errors as shs_solve.
 */
int shs_solve_transposed_workspace(const shs_handle *h, int64_t s, int64_t r, size_t *bytes);
int shs_solve_transposed(shs_handle *h, int64_t s, const double *shifts, int64_t r,
                         const double *D, int64_t ldd, int outputs, void *work, size_t work_bytes,
                         double *X, int64_t ldx, double *eta, int32_t *status, void *stream);

/*
 * Systems with a direction of their own per shift (Section 3.3, the systems
 * of the interpolation method; Section 2 shows why only m entries of the
 * right-hand side are nontrivial after the reduction): for j = 0 .. s-1,
 *
 *     shs_solve_vec:            (H - sigma_j I) x_j = R b_j,
 *     shs_solve_transposed_vec: (H - sigma_j I)^T w_j = Ct^T c_j,
 *
 * i.e. (A - sigma_j I) Q x_j = B b_j and (A - sigma_j I)^T Q w_j = C^T c_j in
 * A's coordinates (Q x_j, Q w_j via shs_apply_q).  shs_solve_vec runs the
 * FP64 structured sweep and ends it as the paper's modification lists:
 * y_j = R_sigma(1:m,1:m)^{-1} R(1:m,1:m) b_j, x_j = Q_sigma^*(:,1:m) y_j.
 * shs_solve_transposed_vec forms Ct^T c_j on the device and runs
 * shs_solve_transposed with one right-hand side per shift.
 *
 *   shifts     device, s complex.
 *   bhat, ldb  device, m x s complex (column j = b_j), ldb >= m; read only.
 *   chat, ldc  device, p x s complex (column j = c_j), ldc >= max(1, p);
 *              may be NULL when p == 0.
 *   outputs    SHS_OUT_X and/or SHS_OUT_ETA.
 *   work       device workspace of the matching *_workspace bytes, or NULL
 *              (allocated on the stream).
 *   X, ldx     device, n x s complex, column j = x_j (resp. w_j).  shs_solve_vec
 *              needs X even without SHS_OUT_X (the residual reads it).
 *   eta        device, s doubles (with SHS_OUT_ETA): normwise backward error
 *              of each shift's system, in FP64, defined as for shs_solve and
 *              shs_solve_transposed with the shift's own right-hand side.
 *   status     device, s int32 SHS_STATUS_* (OK, SINGULAR, NONFINITE).
 *
 * FP64.  Asynchronous on `stream`.  Errors as shs_solve (-i for argument i).
 */
int shs_solve_vec_workspace(const shs_handle *h, int64_t s, size_t *bytes);
int shs_solve_vec(shs_handle *h, int64_t s, const double *shifts, const double *bhat, int64_t ldb, int outputs,
                  void *work, size_t work_bytes, double *X, int64_t ldx, double *eta, int32_t *status,
                  void *stream);
int shs_solve_transposed_vec_workspace(const shs_handle *h, int64_t s, size_t *bytes);
int shs_solve_transposed_vec(shs_handle *h, int64_t s, const double *shifts, const double *chat, int64_t ldc,
                             int outputs, void *work, size_t work_bytes, double *X, int64_t ldx, double *eta,
                             int32_t *status, void *stream);

/*
 * Petrov-Galerkin projection for the interpolation method (Section 1, the
 * spaces V_k, W_k; Section 2: in reduced coordinates W^T A V - lambda W^T V =
 * What^T H Vhat - lambda What^T Vhat, and orthogonalising Vhat, What is the
 * same as orthogonalising V_k, W_k).  From complex bases V, W (n x r each,
 * e.g. the outputs of shs_solve_vec and shs_solve_transposed_vec) the call
 *
 *   1. forms real bases: column k of Vr is the real part (sel[k] even) or the
 *      imaginary part (sel[k] odd) of column sel[k] / 2 of V, likewise Wr
 *      (a conjugate pair of points contributes the real and the imaginary
 *      part of one of its columns);
 *   2. orthonormalises Vr and Wr (Gram-Schmidt with reorthogonalisation);
 *   3. writes Ar = Wr^T H Vr, Er = Wr^T Vr (r x r), Br = Wr^T R (r x m) and
 *      Cr = Ct Vr (p x r), column-major with leading dimensions r, r, r, p.
 *
 *   V, ldv / W, ldw  device, n x r complex, ld >= n; read only.
 *   sel              device, r int32 (0 <= sel[k] < 2r).
 *   work             device workspace of shs_project_workspace(h, r) bytes,
 *                    or NULL (allocated on the stream).
 *   Ar, Er, Br, Cr   device outputs (Cr may be NULL when p == 0).
 *   rank_def         device, one int32: set to 1 if a basis column vanished
 *                    in the orthogonalisation (it is then zero), else 0.
 *
 * FP64, asynchronous on `stream`.  Errors: -i for argument i, SHS_ERR_NOMEM,
 * SHS_ERR_HIP.
 */
int shs_project_workspace(const shs_handle *h, int64_t r, size_t *bytes);
int shs_project(shs_handle *h, int64_t r, const double *V, int64_t ldv, const double *W, int64_t ldw,
                const int32_t *sel, void *work, size_t work_bytes, double *Ar, double *Er, double *Br, double *Cr,
                int32_t *rank_def, void *stream);

/*
 * Structured pseudospectrum (Section 1, the structured epsilon-pseudospectrum
 * of (A, B, C): the points z with ||C (zI - A)^{-1} B||_2 >= 1/epsilon):
 *
 *     norms[j] = ||G_j||_2,   G_j = G(:, j*m : (j+1)*m),  j = 0 .. s-1,
 *
 * the largest singular value of each p x m block, e.g. of shs_solve's G at
 * the points of a grid (the sign of G does not change the norm).  Computed in
 * FP64 from the Hermitian Gram matrix of the smaller side by Jacobi sweeps;
 * relative error a few units of rounding.
 *
 *   s, p, m   blocks, rows, columns per block (1 <= m <= SHS_MAX_M, p >= 0;
 *             p == 0 gives zeros and G may then be NULL).
 *   G, ldg    device, p x (s*m) complex (interleaved), ldg >= max(1, p); read only.
 *   norms     device, s doubles; NaN for a block holding a NaN or infinity.
 *   stream    asynchronous on this stream.
 *
 * Errors: -1..-6 for bad arguments, SHS_ERR_HIP.  Needs no handle.
 */
int shs_transfer_norm2(int64_t s, int64_t p, int64_t m, const double *G, int64_t ldg, double *norms,
                       void *stream);

/*
 * X_orig = Q X_red: maps ncols reduced-coordinate columns (complex, device,
 * n x ncols, leading dimension ld) to A's coordinates (device, ldo), where
 * X_orig = (A - sigma I)^{-1} B for a solution X_red of the reduced system
 * (Section 2: the change of coordinates is orthogonal).  Xred and Xorig may
 * be the same array when ld == ldo.  Asynchronous on `stream`.
 */
int shs_apply_q(const shs_handle *h, int64_t ncols,
                const double *Xred, int64_t ld, double *Xorig, int64_t ldo,
                void *stream);

/*
 * Copy the reduced form to caller device arrays (column-major FP64):
 * H n x n (ldh >= n), R n x m (ldr >= n; rows >= m are zero), Ct p x n
 * (ldct >= max(1,p)); any pointer may be NULL to skip it.  Asynchronous.
 */
int shs_get_reduced(const shs_handle *h, double *H, int64_t ldh,
                    double *R, int64_t ldr, double *Ct, int64_t ldct,
                    void *stream);

/* Sizes, reduction time and resident bytes of a handle. */
int shs_info(const shs_handle *h, shs_info_t *info);

/*
 * Phase timing of the most recent shs_solve on a handle.  When enabled with
 * shs_set_timing(h, 1), shs_solve records HIP events on its stream around
 * every kernel phase; shs_last_timings waits for the last of them and sums
 * the elapsed device time per phase (milliseconds).  Calls per phase are
 * counted in the *_calls fields.  Disabled by default (no events recorded).
 */
typedef struct shs_timings_t {
    double sweep_ms;          /* FP64 sweep (structured right-hand side) */
    double qstar_ms;          /* Q* passes (all precisions) */
    double residual_ms;       /* FP64 residual GEMM + backward error */
    double sweep32_ms;        /* FP32 sweep, structured right-hand side */
    double sweep32_dense_ms;  /* FP32 correction sweeps (dense right-hand side) */
    double other_ms;          /* G evaluation, scaling, bookkeeping */
    int64_t sweep_calls, qstar_calls, residual_calls, sweep32_calls, sweep32_dense_calls, other_calls;
    int64_t sweep_shifts;     /* shifts processed by FP64 sweeps */
    int64_t sweep32_shifts;   /* shifts processed by FP32 structured sweeps */
    int64_t sweep32_dense_shifts; /* shift-solves processed by FP32 dense sweeps */
    int64_t refine_iterations;    /* correction rounds run by the mixed mode */
    int64_t fallback_shifts;      /* shifts the mixed mode recomputed in FP64 */
    /* The FP64 sweep of shs_solve runs blocked by row tiles (Section 3.1,
     * Step 2 revisited): per tile, one kernel makes the reflectors and the
     * block transform of every shift, one GEMM updates all rows above for all
     * shifts.  Both are part of sweep_ms; these split it. */
    double sweep_tile_ms;         /* per-shift row-tile kernels */
    double sweep_update_ms;       /* all-shift update GEMMs */
    int64_t sweep_tile_calls, sweep_update_calls;
    /* Algorithmic flops of those launches (2 per multiply-add): tile steps
     * (16m+4 per row above each pivot), block transforms and group products;
     * update GEMMs (H block times 2m real columns per shift, carried columns
     * times 2m x 2m). */
    double sweep_tile_flops, sweep_update_flops;
} shs_timings_t;

int shs_set_timing(shs_handle *h, int enable);
int shs_last_timings(const shs_handle *h, shs_timings_t *out);

/* ------------------------------------------------------------------------ */
/* Serving: resident systems, continuous batching of shift requests.         */
/* ------------------------------------------------------------------------ */
/*
 * A server keeps reduced systems (handles) resident on the current GPU and
 * runs shift requests from many clients.  Worker threads, one per HIP stream,
 * take work as soon as they are free: FP64 requests that are waiting are
 * batched into one launch of the work-item kernel (shifts of different
 * systems, with different n and m, in the same launch), unless one shift is
 * too much work for one wavefront (see blocked_flops): such a request, like
 * a mixed-precision one, runs as one shs_solve on its worker's stream.  A
 * request's route depends only on its system and mode, so its results are
 * the same alone or in any mix.  A request is
 * admitted only when its workspace (shs_solve_workspace bytes) fits in what
 * is left of the device-memory budget; requests that arrive while others
 * run are admitted as workers and memory free up, so their work overlaps on
 * the device.  Latency is stamped at submit and at completion.
 *
 * A request on the solve route (mixed mode, or FP64 above blocked_flops)
 * is batched with the other waiting requests of the same system, mode and
 * outputs into one shs_solve over all their shifts.  Every kernel computes
 * each shift independently of the other shifts in its launch, so a result
 * is bitwise the same alone and in any batch.  Latency runs from the
 * request's arrival (given by the caller, else the submit call) to the end
 * of its batch.
 *
 * Thread-safe: any thread may submit, poll, wait and cancel.  The server
 * never owns the handles it serves; destroy the server before them.  Do not
 * enable phase timing (shs_set_timing) on a handle a server uses.
 */
typedef struct shs_server shs_server;

typedef struct shs_server_config {
    int32_t abi_version;    /* must be SHS_ABI_VERSION */
    int32_t streams;        /* worker threads / HIP streams (>= 1) */
    int64_t budget_bytes;   /* device-memory budget for request workspaces */
    int32_t max_batch;      /* most requests per FP64 batch (>= 1) */
    int32_t flags;          /* reserved, 0 */
    /* FP64 requests whose per-shift sweep work (8m+2) n^2 flops exceeds this
     * run alone through shs_solve's blocked sweep instead of the work-item
     * kernel (0: the default, 7.7e8 flops, about 20 ms of one wavefront);
     * negative: never. */
    double blocked_flops;
    int64_t reserved[3];
} shs_server_config;

/* request states (shs_server_poll) */
#define SHS_REQ_QUEUED     0
#define SHS_REQ_RUNNING    1
#define SHS_REQ_DONE       2
#define SHS_REQ_FAILED     3
#define SHS_REQ_CANCELLED  4

typedef struct shs_server_stats_t {
    int64_t submitted, completed, failed, cancelled, queued, running;
    int64_t solves;              /* shifts completed */
    int64_t batches;             /* launches of batched requests (both routes) */
    int64_t max_batch_systems;   /* most distinct systems in one batch */
    int64_t max_batch_requests;  /* most requests in one batch */
    double  p50_ms, p99_ms, max_ms, mean_ms;   /* arrival -> completion of completed requests */
    double  busy_s;              /* wall time from the first arrival to the last completion */
    int64_t peak_bytes;          /* largest admitted workspace total */
} shs_server_stats_t;

/* Options of one request (shs_server_submit_ex). */
typedef struct shs_request_opts {
    int32_t abi_version;   /* must be SHS_ABI_VERSION */
    int32_t order_after;   /* 1: the request's work starts after all work queued on after_stream
                              before the submit call (e.g. the allocation of its outputs); 0: no ordering */
    void   *after_stream;  /* hipStream_t (NULL = the null stream), used when order_after = 1 */
    double  arrival_s;     /* arrival time on the shs_server_clock() clock; <= 0 or later than
                              the submit call: the submit call's time */
    int64_t reserved[4];   /* 0 */
} shs_request_opts;

int shs_server_create(const shs_server_config *cfg, shs_server **out);

/* Make a handle servable; *sys_id receives its id.  The handle must belong
 * to the server's device. */
int shs_server_register(shs_server *srv, shs_handle *h, int32_t *sys_id);

/*
 * Queue a request: s shifts (host array, copied before return) on system
 * sys_id with mode/outputs as for shs_solve.  X, G, eta, status are device
 * arrays laid out as in shs_solve; they must stay valid until the request
 * completes.  *req_id receives the request id.  Returns SHS_ERR_NOMEM if the
 * request alone exceeds the budget, SHS_ERR_NOTFOUND for an unknown system.
 */
int shs_server_submit(shs_server *srv, int32_t sys_id, int64_t s, const double *shifts_host,
                      int mode, int outputs, double *X, int64_t ldx, double *G, int64_t ldg,
                      double *eta, int32_t *status, int64_t *req_id);

/* As shs_server_submit, with options (NULL: none): ordering after the
 * caller's stream and the request's arrival time.  -13 for a bad opts. */
int shs_server_submit_ex(shs_server *srv, int32_t sys_id, int64_t s, const double *shifts_host,
                         int mode, int outputs, double *X, int64_t ldx, double *G, int64_t ldg,
                         double *eta, int32_t *status, const shs_request_opts *opts,
                         int64_t *req_id);

/* The server's clock (steady, seconds) for arrival times. */
double shs_server_clock(void);

/* *state: one of SHS_REQ_*. */
int shs_server_poll(shs_server *srv, int64_t req_id, int *state);

/* Wait until the request completes (timeout_ms < 0: no limit).  Returns 0,
 * SHS_ERR_TIMEOUT, SHS_ERR_CANCELLED, or the error the request failed with. */
int shs_server_wait(shs_server *srv, int64_t req_id, double timeout_ms);

/* Cancel a request.  A queued request is removed from the queue (its outputs
 * are not touched) and is cancelled at once; a running one completes (its
 * outputs may be written) and is then marked cancelled; either way it does
 * not count as completed.  SHS_ERR_STATE if it already finished. */
int shs_server_cancel(shs_server *srv, int64_t req_id);

/* Hold (paused = 1) or release (0) the workers: while held, they start no
 * new batch (running batches finish); requests queue up and are batched
 * together on release. */
int shs_server_pause(shs_server *srv, int paused);

/* Arrival -> completion latency of a completed request, milliseconds;
 * SHS_ERR_STATE if it has not completed. */
int shs_server_latency(shs_server *srv, int64_t req_id, double *ms);

int shs_server_stats(shs_server *srv, shs_server_stats_t *out);

/* Waits for all requests, stops the workers and frees the server. */
void shs_server_destroy(shs_server *srv);

/* Release a handle and all device memory it owns (synchronises its device). */
void shs_destroy(shs_handle *h);

/* Static text for any return code of this library. */
const char *shs_strerror(int code);

/* ABI version compiled into the library (SHS_ABI_VERSION). */
int shs_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHIFTSOLVE_H */
