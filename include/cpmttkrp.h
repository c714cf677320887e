/*
 * cpmttkrp -- dense MTTKRP, CP-ALS sweep and CP least-squares gradient on
 * AMD Instinct MI355X (gfx950).
 *
 * Operations follow Hayashi, Ballard, Jiang, Tobia, "Shared-Memory
 * Parallelization of MTTKRP for Dense Tensors" (2018):
 *
 *   MTTKRP (Section 2.2, first of the three CP-ALS operations):
 *     M = X_(n) (U_{N-1} kr ... kr U_{n+1} kr U_{n-1} kr ... kr U_0),
 *     i.e. M(i_n, c) = sum over the entries with mode-n index i_n of
 *          X(i_0..i_{N-1}) * prod_{k != n} U_k(i_k, c).
 *   CP-ALS factor update (Section 2.2): M as above, H = Hadamard product of
 *     the Grams U_k^T U_k over k != n, U_n = M H^-1.
 *   CP gradient (Section 2.2 notes MTTKRP is part of the gradient): for
 *     f = 1/2 ||X - [[U_0..U_{N-1}]]||_F^2, df/dU_n = U_n H_n - MTTKRP_n.
 *
 * Layout conventions shared by every entry point
 *   - dims[0..N-1] are I_0..I_{N-1}; X is stored in the natural
 *     linearisation of Section 2.1, l = sum_n i_n prod_{k<n} I_k, so mode 0
 *     is the stride-1 index.  (A C-contiguous array of shape
 *     (I_{N-1}, ..., I_0) has exactly this layout.)  The tensor is never
 *     permuted or copied.
 *   - factors[k] is an I_k x R matrix, row-major (R contiguous).
 *   - MTTKRP outputs and gradients are I_n x R, row-major, fully overwritten.
 *   - Element types by cpm_dtype:
 *       CPM_F32    : X float32, factors/outputs float32.
 *       CPM_F64    : X float64, factors/outputs float64.
 *       CPM_BF16X2 : X is 2*I bfloat16 values (uint16 bit patterns): the hi
 *                    plane (I values) followed by the lo plane; an entry's
 *                    value is hi + lo.  Factors/outputs float32.  The
 *                    contraction runs on bf16 MFMA with float32 accumulation
 *                    using hi*hi + hi*lo + lo*hi products of the split tensor
 *                    and of the split Khatri-Rao rows.
 *
 * Ownership: every pointer named "device" is caller-owned device memory on
 * the current HIP device; pointer arrays (factors, grads) and dims are host
 * memory read during the call only.  The library allocates no memory and
 * keeps no state between calls apart from the thread-local error message.
 * Workspaces are caller-provided; query their size with the *_workspace_bytes
 * functions (0 is a valid size; a null workspace is then accepted).
 *
 * Errors: every call returns a cpm_status.  All argument validation happens
 * before any HIP call, so invalid arguments never launch work.  A HIP
 * runtime failure returns CPM_EHIP.  cpm_last_error() gives a message for
 * the last non-OK status returned on the calling thread.
 *
 * Ordering: work is enqueued on `stream` and calls return without waiting,
 * except cp_als_step, which waits once for the stream to learn whether every
 * Cholesky factorisation succeeded (and to return the fit when asked).
 *
 * Limits: 2 <= N <= 12 (N outside gives CPM_EINVAL), every dim >= 1,
 * prod(dims) < 2^62, 1 <= R <= 256 (R <= 128 for cp_als_step, whose
 * float64 Cholesky factorisation keeps the R x R matrix in one work-group's
 * LDS, and for cpm_residual2).  Every factor that a call reads must span
 * fewer than 2^32 - 256 bytes (I_k * R * element size), the reach of one
 * buffer resource; larger factors give CPM_EUNSUPPORTED.  Larger R gives
 * CPM_EUNSUPPORTED.
 */
#ifndef CPMTTKRP_H
#define CPMTTKRP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CPM_OK = 0,
    CPM_EINVAL = 1,       /* bad argument: null pointer, bad dims/mode/R */
    CPM_EUNSUPPORTED = 2, /* valid but outside the library's limits */
    CPM_ENOTPD = 3,       /* cp_als_step: Hadamard-of-Grams not positive definite */
    CPM_EHIP = 4,         /* HIP runtime error (launch or synchronisation) */
    CPM_EWORKSPACE = 5    /* workspace null or smaller than the queried size */
} cpm_status;

/* The two range markers are not types: they make every int value a valid
 * cpm_dtype object, so a caller's out-of-range code is well defined and is
 * rejected with CPM_EINVAL. */
typedef enum {
    CPM_F32 = 0,
    CPM_F64 = 1,
    CPM_BF16X2 = 2,
    CPM_DTYPE_RANGE_MIN_ = -2147483647 - 1,
    CPM_DTYPE_RANGE_MAX_ = 2147483647
} cpm_dtype;

#define CPM_MAX_MODES 12
#define CPM_MAX_RANK 256
#define CPM_MAX_RANK_SOLVE 128

/* Library version: major * 10000 + minor * 100 + patch. */
int cpm_version(void);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *cpm_last_error(void);

/*
 * Bytes of workspace `mttkrp` needs for this shape, mode, rank and type.
 * Returns 0 for invalid arguments too (the call itself then reports them).
 */
size_t cpm_mttkrp_workspace_bytes(const int64_t *dims, int N, int R, int mode, cpm_dtype dt);

/*
 * Mode-`mode` MTTKRP (Section 2.2).  X: device tensor; factors: host array
 * of N device pointers (factors[mode] is not read and may be null); out:
 * device I_mode x R.  Internal modes fuse the partial MTTKRP against the
 * left Khatri-Rao product with the multi-TTV against the right one (the
 * 2-step scheme of Section 4.3); Khatri-Rao rows are formed on the fly
 * (the row-wise product with reuse of Section 4.1) and never stored.
 * The result is bitwise reproducible run to run.
 */
cpm_status mttkrp(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                  int mode, void *out, cpm_dtype dt, void *workspace, size_t ws_bytes,
                  hipStream_t stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): `mttkrp` without
 * a workspace argument.  The split-K partial results go to a fixed device
 * array of CPM_SCRATCH_BYTES bytes inside the library (one per GPU, held
 * until the process ends), so the call allocates nothing and launches the
 * same kernels with the same tiling as `mttkrp` -- the result is bitwise
 * equal to mttkrp's.  Arguments as for `mttkrp`.  Shapes whose partial
 * results exceed CPM_SCRATCH_BYTES (cpm_mttkrp_workspace_bytes tells)
 * return CPM_EUNSUPPORTED before any launch.  Every call on one GPU uses
 * the same array: calls that overlap on one GPU (concurrent streams or
 * threads) race and give wrong results; serialise them.  Nothing in the
 * array needs clearing between calls (every partial read is written first
 * by the same call).  The first call on a device looks up the array's
 * device address (hipGetSymbolAddress) with that device current.
 */
#define CPM_SCRATCH_BYTES (64u << 20)
cpm_status mttkrp_scratch(const void *X, const int64_t *dims, int N, const void *const *factors, int R, int mode,
                          void *out, cpm_dtype dt, hipStream_t stream);

/*
 * Diagnostics: writes into buf (at most len bytes, NUL-terminated) the
 * kernel and launch shape `mttkrp` would use for this shape, mode, rank and
 * type -- the contraction kernel with its template parameters, its grid,
 * LDS bytes, Khatri-Rao chunk, inner/outer split (Section 4.1's reuse at
 * tile level), split-K count and whether the fixed-order reduction runs.
 * X is used only for its address alignment (never dereferenced; null
 * counts as aligned, like any multiple of 16).  Host only, launches
 * nothing.  Returns
 * a cpm_status (CPM_EINVAL for bad arguments or an empty buffer).
 */
int cpm_mttkrp_describe(const int64_t *dims, int N, int R, int mode, cpm_dtype dt, const void *X, char *buf,
                        size_t len);

/*
 * Bytes of workspace `mttkrp_all` needs (0 for invalid arguments).
 */
size_t cpm_mttkrp_all_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt);

/*
 * The MTTKRPs of several modes with the same factors (Section 2.2's
 * definition for every requested mode), with the reuse of partial results
 * across modes that the Conclusion names as the next step (after Phan et
 * al.).  X, dims, factors, R, dt as for `mttkrp`, except that every factor
 * is read.  outs: host array of N device pointers, outs[n] an I_n x R
 * output or null to skip mode n.  When three or more modes are requested,
 * the modes are split into a left group [0, s) and a right group [s, N):
 * one pass over X contracts the right group and one the left, each leaving
 * an intermediate of (entries of its group) x R values in the workspace,
 * and every requested mode then follows from its group's intermediate --
 * two passes over X instead of one per mode.  From N = 4 on the split is
 * chosen so that the intermediates move fewer entries than one pass over X.
 * For N = 3 the split is {0, 1} | {2}, used under the same rule and only
 * where the pass over the (I_0 I_1, I_2) view runs as fast as a single-mode
 * call (float32, I_0 I_1 of about 131072 or more, I_2 up to 512; the query
 * `cpm_mttkrp_all_workspace_bytes` reserves room for it exactly then).
 * Otherwise (and for N = 2) each mode is an ordinary `mttkrp`.  The result
 * agrees with `mttkrp` to rounding (a different summation order) and is
 * bitwise reproducible run to run.  Stream-ordered, no synchronisation.
 */
cpm_status mttkrp_all(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                      void *const *outs, cpm_dtype dt, void *workspace, size_t ws_bytes,
                      hipStream_t stream);

/*
 * The straightforward MTTKRP the paper measures against (Section 2.3; its
 * Section 5.3 also times one matrix multiplication of the same shape as a
 * lower bound): X_(n) formed explicitly by reordering the entries (internal
 * modes; X_(0) and X_(N-1) are already column- and row-major matrices in
 * the natural layout, as the paper notes, and are used in place), the full
 * Khatri-Rao product U_{N-1} kr ... kr U_{n+1} kr U_{n-1} kr ... kr U_0
 * formed explicitly (I / I_n rows of R values), then one hipBLASLt GEMM
 * M = X_(n) K.  Provided to measure the fused kernels against it; it moves
 * the tensor up to three times (read, reordered copy written and read) plus
 * the Khatri-Rao product.  Arguments as for `mttkrp`; CPM_F32 or CPM_F64
 * (CPM_BF16X2 gives CPM_EUNSUPPORTED).  The workspace holds the reordered
 * tensor (internal modes), the Khatri-Rao product and 32 MiB for the GEMM.
 * The first call on a device creates a hipBLASLt handle (which allocates);
 * the algorithm for each GEMM shape is chosen once and kept.  A shape for
 * which hipBLASLt offers no algorithm (float64 with R = 1 or I_n = 1 on
 * gfx950) gives CPM_EUNSUPPORTED; the reordering and the Khatri-Rao product
 * have then been enqueued into the workspace but nothing is written to out.
 */
size_t cpm_explicit_workspace_bytes(const int64_t *dims, int N, int R, int mode, cpm_dtype dt);
cpm_status mttkrp_explicit(const void *X, const int64_t *dims, int N, const void *const *factors, int R, int mode,
                           void *out, cpm_dtype dt, void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Symmetric-pair packed storage (Section 5.3.3 stores the symmetric
 * region-by-region pair of its fMRI tensor as one linearised triangle).
 * A tensor with I_0 = I_1 = n and X(i, j, rest) = X(j, i, rest) is held as
 * its triangle i <= j: pair index p = j (j + 1) / 2 + i (i fastest, then j),
 * followed by modes 2..N-1 in natural order, P = n (n + 1) / 2 pairs, so
 * about half the entries.  The diagonal is kept, so the packed tensor
 * stands for the whole symmetric tensor: a packed entry is the value of
 * (i, j, rest) and, when i != j, of (j, i, rest).  For CPM_BF16X2 the
 * packed tensor is two planes (hi then lo) of P * I_2 * ... entries.
 * dims are the full tensor's; N >= 3; dims[0] == dims[1] (else
 * CPM_EINVAL).
 */
size_t cpm_sympair_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt);

/*
 * MTTKRPs (Section 2.2) of the full symmetric tensor held packed in Xp, for
 * every mode n with outs[n] non-null (device I_n x R; null skips the mode);
 * results equal `mttkrp` of the unpacked tensor to rounding while X is read
 * at about half the bytes.  Modes 2..N-1 are MTTKRPs of the packed view
 * (P, I_2, ...) with the pair factor W(p, :) = U_0(i) * U_1(j) + U_0(j) *
 * U_1(i) (i < j; U_0(i) * U_1(i) on the diagonal) built on the fly per
 * call; the two pair modes share one pass, the view's mode-0 MTTKRP T
 * (P x R), and then M_0(a, :) = sum_j T(pair(a, j), :) * U_1(j, :) and
 * M_1(b, :) = sum_i T(pair(i, b), :) * U_0(i, :).  Every factor is read.
 * Stream-ordered; bitwise reproducible run to run.
 */
cpm_status mttkrp_sympair(const void *Xp, const int64_t *dims, int N, const void *const *factors, int R,
                          void *const *outs, cpm_dtype dt, void *workspace, size_t ws_bytes,
                          hipStream_t stream);

/*
 * Packs a full tensor symmetric in modes 0 and 1 (device X, natural order)
 * into the triangle layout above (device Xp, P * I_2 * ... entries, or two
 * planes of them for CPM_BF16X2).  Only entries i <= j of X are read; the
 * symmetry itself is not checked.  Pure data movement.
 */
cpm_status cpm_pack_sympair(const void *X, const int64_t *dims, int N, cpm_dtype dt, void *Xp,
                            hipStream_t stream);

/*
 * Bytes of workspace `cpm_residual2` needs (0 for invalid arguments).
 */
size_t cpm_residual2_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt);

/*
 * *out_dev = ||X - [[U_0..U_{N-1}]]||_F^2 (device double), with every model
 * entry sum_c prod_k U_k(i_k, c) (the CP model of Section 2.2) recomputed on
 * the fly while X streams past once; nothing of the residual is stored.
 * The Conclusion names this computation as the next bottleneck once MTTKRP
 * is fast.  Unlike the identity ||X||^2 - 2 <M, U> + sum(Hadamard of
 * Grams), it does not lose digits to cancellation when the model fits well:
 * model entries are float32 sums of float32 products, differences and
 * squares are summed in float64.  dt: CPM_F32 or CPM_BF16X2 (CPM_F64 gives
 * CPM_EUNSUPPORTED).  factors: every entry read.  R <= 128.  The sum runs
 * in a fixed order (bitwise reproducible).  Stream-ordered.
 */
cpm_status cpm_residual2(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                         cpm_dtype dt, double *out_dev, void *workspace, size_t ws_bytes,
                         hipStream_t stream);

/* Bytes of workspace for cp_als_step / cp_grad. */
size_t cpm_cp_als_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt);
size_t cpm_cp_grad_workspace_bytes(const int64_t *dims, int N, int R, cpm_dtype dt);

/*
 * One CP-ALS sweep (Section 2.2): for n = 0..N-1 in order, M = MTTKRP_n with
 * the current factors, H = Hadamard product of the other Grams (float64),
 * Cholesky H = L L^T (float64), U_n = M H^-1 (float64, stored in the
 * factor type).  factors: host array of N device pointers, updated in
 * place.  If any H is not positive definite, every factor is restored to
 * its input value and CPM_ENOTPD is returned.  xnorm2: ||X||_F^2 if known,
 * or negative to have it computed (only needed when fit_out is non-null).
 * fit_out: host pointer, may be null; receives 1 - ||X - Y|| / ||X|| of the
 * updated model (from ||X||^2 - 2 <M_{N-1}, U_{N-1}> + sum(Hadamard of all
 * Grams), accumulated in float64).  Waits for the stream once (and once
 * more to restore the factors when it fails).
 * Where `mttkrp_all` would split the modes, the MTTKRPs come from its two
 * passes: the
 * left group's intermediate depends only on factors not yet updated when
 * it is formed, and the right group's is formed after the left group's
 * updates, so the sweep is the same Gauss-Seidel order.
 * R <= 128.
 */
cpm_status cp_als_step(const void *X, const int64_t *dims, int N, void *const *factors, int R,
                       cpm_dtype dt, double xnorm2, double *fit_out, void *workspace,
                       size_t ws_bytes, hipStream_t stream);

/*
 * Gradient of f = 1/2 ||X - [[U_0..U_{N-1}]]||_F^2 for every factor:
 * grads[n] = U_n H_n - MTTKRP_n (device I_n x R each; grads may be null to
 * compute only the loss, and single entries may be null to skip a mode).
 * loss_dev: device double, may be null; receives f evaluated as
 * 1/2 (||X||^2 - 2 <MTTKRP_{N-1}, U_{N-1}> + sum(Hadamard of all Grams)),
 * accumulated in float64, the residual itself never being formed.
 * xnorm2: ||X||_F^2 if known, negative to compute it on the device.
 * The MTTKRPs are formed as by `mttkrp_all` (two passes over X where it
 * splits the modes).
 * R <= 256: the gradient needs no factorisation.
 */
cpm_status cp_grad(const void *X, const int64_t *dims, int N, const void *const *factors, int R,
                   void *const *grads, double xnorm2, double *loss_dev, cpm_dtype dt,
                   void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * ||X||_F^2 accumulated in float64 into *out_dev (device double).
 * Workspace: cpm_xnorm2_workspace_bytes().
 */
size_t cpm_xnorm2_workspace_bytes(const int64_t *dims, int N, cpm_dtype dt);
cpm_status cpm_xnorm2(const void *X, const int64_t *dims, int N, cpm_dtype dt, double *out_dev,
                      void *workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Split `count` float32 values into bfloat16 planes: hi = RNE(x) and
 * lo = RNE(x - hi) (x - hi is exact in float32).  planes: device, 2*count
 * uint16 values, hi plane first -- the CPM_BF16X2 tensor format.
 */
cpm_status cpm_split_bf16(const float *x, int64_t count, uint16_t *planes, hipStream_t stream);

/*
 * Rows [j0, j0 + nrows) of the Khatri-Rao product mats[0] kr ... kr
 * mats[Z-1] (Section 2.1: the last matrix's row index varies fastest),
 * formed on the device row by row, each row's multi-index stepped with
 * carries and the slow partial Hadamard product reused across consecutive
 * rows (Section 4.1).
 * mats: host array of Z device pointers to J_z x R row-major matrices
 * (float32 for CPM_F32, float64 for CPM_F64); out: device nrows x R.
 * 1 <= Z <= 12.
 */
cpm_status cpm_krp_rows(const void *const *mats, const int64_t *J, int Z, int R, int64_t j0,
                        int64_t nrows, void *out, cpm_dtype dt, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CPMTTKRP_H */
