/*
 * mxs.h -- C ABI of libmxs, an MI355X (gfx950) library for sparse
 * matrix-vector multiplication y = A*x over the COO, CSR and DIA storage
 * formats and the conjugate-gradient loop that calls it, after
 * "Morpheus unleashed: Fast cross-platform SpMV on emerging architectures"
 * (arXiv 2304.09511).
 *
 * General conventions
 *   - Every call returns an mxs_status; no C++ exception crosses the ABI.
 *   - Pointers to matrix arrays and vectors are DEVICE pointers unless the
 *     argument description says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked [async] only enqueue work on `stream`; calls marked
 *     [syncs] wait for `stream` before returning because they hand a value
 *     back to the host.  Device faults surface as MXS_ERR_HIP at the next
 *     call that synchronises.
 *   - Indices are int32 and 0-based; ranges are half-open, as in the loops
 *     of Algorithms 1-3 (Section III-B).  Counts of entries or slots are
 *     int64.
 *   - Values are FP64 (double) or FP32 (float), fixed per matrix by its
 *     mxs_dtype; vectors passed with a matrix have that matrix's dtype.
 *   - A call that fails validation leaves its outputs untouched.
 *   - Memory: the library allocates device memory only for the arrays a
 *     handle owns (copies made without MXS_BORROW) and for temporaries of
 *     conversions, checks, plan sizing and feature extraction; all of it is
 *     freed by mxs_destroy or before the call returns.  Execution plans,
 *     outputs and CG workspaces are allocated by the caller.
 */
#ifndef MXS_H
#define MXS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MXS_OK = 0,
    MXS_NOT_CONVERGED = 1,       /* iteration cap reached; the result is valid */
    MXS_ERR_INVALID_ARG = -1,    /* null pointer, negative size, aliasing, bad enum */
    MXS_ERR_INDEX_RANGE = -2,    /* an index outside its dimension, bad row pointers */
    MXS_ERR_UNSORTED = -3,       /* order required and not met (borrowed arrays, DIA offsets) */
    MXS_ERR_DUPLICATE = -4,      /* the same (row, col) stored twice */
    MXS_ERR_DIA_TOO_SPARSE = -5, /* DIA would store more than 8 slots per non-zero */
    MXS_ERR_OUT_OF_MEMORY = -6,
    MXS_ERR_HIP = -7,            /* a HIP runtime error, including device faults */
    MXS_ERR_BREAKDOWN = -8,      /* CG: p.Ap <= 0 or not finite (A not SPD) */
    MXS_ERR_NONFINITE = -9,      /* NaN or Inf in a CG right-hand side or start vector */
    MXS_ERR_UNSUPPORTED = -10,   /* operation not defined for this format/dtype/shape */
    MXS_ERR_NO_PLAN = -11        /* the handle has no plan: call mxs_optimize first */
} mxs_status;

typedef enum {
    MXS_COO = 0, MXS_CSR = 1, MXS_DIA = 2, MXS_HDC = 3, MXS_ELL = 4, MXS_SELL = 5, MXS_HYB = 6
} mxs_format;
typedef enum { MXS_F64 = 0, MXS_F32 = 1 } mxs_dtype;

/* Opaque host-side handle of a sparse matrix in one storage format. */
typedef struct mxs_mat_s *mxs_mat;
typedef struct mxs_mg_s *mxs_mg; /* multigrid hierarchy of the HPCG problem */

/* Creation flags. */
#define MXS_BORROW 1u /* reference the caller's arrays instead of copying them;
                         they must stay alive and unchanged until mxs_destroy */

/* Human-readable name of a status code (static string, never NULL). */
const char *mxs_status_string(mxs_status s);

/* Library version as major*10000 + minor*100 + patch. */
int32_t mxs_version(void);

/* Detail of the last HIP failure seen by this thread (HIP error name and
 * message, the failing call and, if one was pending, the error another
 * library left in HIP's per-thread error slot, which every entry point
 * clears on entry), or of the last size a fixed scratch array refused.
 * Empty if none; valid until the thread's next failure. */
const char *mxs_last_error(void);

/* ------------------------------------------------------------------------
 * Containers (Section III-B: COO, CSR, DIA; typed for double and float as
 * in Section VI-A's containers).  All three validate their input on the
 * device and therefore [syncs].
 * --------------------------------------------------------------------- */

/* COO (Section III-B): entry k is (ai[k], aj[k], av[k]), k in [0, nnz).
 * The paper's COO imposes no order.  The handle holds the canonical form:
 * sorted by (row, col), which the COO kernel requires.  Unsorted input is
 * sorted on the device into the handle's own copy; with MXS_BORROW it is
 * refused with MXS_ERR_UNSORTED.  Errors: MXS_ERR_INDEX_RANGE for an index
 * outside [0,nrows) x [0,ncols), MXS_ERR_DUPLICATE for a repeated
 * (row, col).  nnz = 0 is legal (A = 0). */
mxs_status mxs_coo_create(mxs_mat *out, int32_t nrows, int32_t ncols, int64_t nnz,
                          const int32_t *ai, const int32_t *aj, const void *av,
                          mxs_dtype dtype, unsigned flags, void *stream);

/* CSR (Section III-B): irp[nrows+1] row pointers with irp[0] = 0 and
 * irp[nrows] = nnz, non-decreasing; aj[nnz], av[nnz].  The paper imposes
 * no order within a row; this library requires strictly ascending columns
 * within a row (MXS_ERR_UNSORTED otherwise, MXS_ERR_DUPLICATE for a
 * repeat), which makes conversions exact.  Bad row pointers or columns:
 * MXS_ERR_INDEX_RANGE. */
mxs_status mxs_csr_create(mxs_mat *out, int32_t nrows, int32_t ncols, int64_t nnz,
                          const int32_t *irp, const int32_t *aj, const void *av,
                          mxs_dtype dtype, unsigned flags, void *stream);

/* DIA (Section III-B, Algorithm 3): ndiag offsets doff[d] (strictly
 * ascending, each in [-(nrows-1), ncols-1]) and values stored
 * DIAGONAL-MAJOR: av[d*nrows + i] multiplies x[i + doff[d]] in row i
 * (row-aligned, as av(i,j) in Algorithm 3; the paper keeps av(i,j)
 * row-major, this layout transposes it so that consecutive rows are
 * consecutive in memory).  Slots with i + doff[d] outside [0, ncols) are
 * never read.  Errors: MXS_ERR_INDEX_RANGE (offset out of range),
 * MXS_ERR_UNSORTED (offsets not strictly ascending). */
mxs_status mxs_dia_create(mxs_mat *out, int32_t nrows, int32_t ncols, int32_t ndiag,
                          const int32_t *doff, const void *av, mxs_dtype dtype,
                          unsigned flags, void *stream);

/* Frees what the handle owns (waits for its pending work first).  A NULL
 * handle is accepted. */
mxs_status mxs_destroy(mxs_mat A);

/* Host copies of a handle's shape.  Any output pointer may be NULL.  nnz is
 * the stored-entry count (COO, CSR) or the in-range slot count (DIA). */
mxs_status mxs_info(mxs_mat A, mxs_format *fmt, mxs_dtype *dtype, int32_t *nrows,
                    int32_t *ncols, int64_t *nnz, int32_t *ndiag);

/* Device pointers of the canonical arrays (owned by the handle or borrowed):
 * COO (ai, aj, av); CSR (irp, aj, av); DIA (doff, NULL, av).  Read-only. */
mxs_status mxs_arrays(mxs_mat A, const int32_t **idx0, const int32_t **idx1,
                      const void **vals);

/* ------------------------------------------------------------------------
 * Format conversion (the runtime switching of Sections I-II)
 * --------------------------------------------------------------------- */

/* Sizes of the arrays mxs_convert will write for `dst` [syncs]:
 *   dst COO/CSR: *count = number of entries (for DIA sources, the in-range
 *                slots whose value is not +0.0 or -0.0); *ndiag = 0.
 *   dst DIA:     *ndiag = number of distinct offsets j - i, *count =
 *                ndiag*nrows (length of av).  Refused with
 *                MXS_ERR_DIA_TOO_SPARSE when ndiag*nrows > 8*nnz.
 *   dst ELL:     (sources COO, CSR, ELL) *ndiag = K, the longest row's
 *                length, *count = K*nrows.  Refused with
 *                MXS_ERR_DIA_TOO_SPARSE when K*nrows > 8*nnz.
 * ELL and SELL sources convert to COO and CSR only, SELL is reached
 * through mxs_to_sell (MXS_ERR_UNSUPPORTED otherwise).
 * count or ndiag may be NULL. */
mxs_status mxs_convert_size(mxs_mat src, mxs_format dst, int64_t *count, int32_t *ndiag,
                            void *stream);

/* Writes `src` in format `dst` into caller-allocated device arrays and
 * returns a new handle that BORROWS them [syncs]:
 *   dst COO: idx0 = ai[count], idx1 = aj[count], vals = av[count]
 *   dst CSR: idx0 = irp[nrows+1], idx1 = aj[count], vals = av[count]
 *   dst DIA: idx0 = doff[ndiag], idx1 unused (may be NULL), vals = av[count]
 *   dst ELL: idx0 = col[K*nrows], idx1 unused, vals = val[K*nrows]: ELL
 *            (Section IX's further formats), column-major: slot k of row i
 *            at k*nrows + i holds the row's k-th entry; slots past the row's
 *            length hold column -1 and +0.0.  mxs_info reports K as ndiag.
 * with sizes from mxs_convert_size.  Output is canonical: rows ascending,
 * columns ascending within a row, DIA offsets ascending with +0.0 in slots
 * that hold no entry.  Values are moved, never recomputed: bit-exact. */
mxs_status mxs_convert(mxs_mat src, mxs_format dst, int32_t *idx0, int32_t *idx1, void *vals,
                       mxs_mat *out, void *stream);

/* SELL-C-sigma (Section IX's further formats; Kreutzer et al., 2014) with
 * C = 64, one wavefront per slice, from a COO or CSR source.  Rows are sorted
 * by descending length, stably, inside windows of `sigma` >= 1 consecutive
 * rows: perm[p] = row at sorted position p.  Slice s (positions
 * [64s, 64s+64)) is as wide as its longest row and starts at cs[s]
 * (cs[s+1] = cs[s] + 64*width_s); slot k of position p in slice s is at
 * cs[s] + 64k + (p - 64s), padded as ELL (positions past the last row too).
 * mxs_sell_size [syncs]: *slots = cs[nslices], *nslices = ceil(nrows/64);
 *   refused with MXS_ERR_DIA_TOO_SPARSE when slots > 8*nnz.
 * mxs_to_sell [syncs]: writes perm[nrows], cs[nslices+1], col[slots],
 *   vals[slots] (caller-allocated) and returns a handle that borrows them;
 *   mxs_info reports the slice count as ndiag.  Values are moved
 *   (bit-exact).  SpMV, CG (FP64, also as the FP32 operand of mixed
 *   solves after mxs_cast), conversion to COO/CSR and cast accept ELL and
 *   SELL handles; features and splits do not (MXS_ERR_UNSUPPORTED). */
mxs_status mxs_sell_size(mxs_mat A, int32_t sigma, int64_t *slots, int32_t *nslices, void *stream);
mxs_status mxs_to_sell(mxs_mat A, int32_t sigma, int32_t *perm, int64_t *cs, int32_t *col,
                       void *vals, mxs_mat *out, void *stream);

/* Same structure, values rounded to nearest (even) in `dtype` into
 * caller-allocated `vals` (as many values as src stores) [async].  The new handle borrows src's
 * index arrays and `vals`: destroy it before src. */
mxs_status mxs_cast(mxs_mat src, mxs_dtype dtype, void *vals, mxs_mat *out, void *stream);

/* ------------------------------------------------------------------------
 * SpMV (Algorithms 1-3)
 * --------------------------------------------------------------------- */

/* Execution plans (the optimize stage of Section VI-A's Table I: create,
 * optimize, execute, destroy).  A plan lives in device memory the CALLER
 * allocates and keeps alive, unchanged, until mxs_destroy or the next
 * mxs_optimize of the handle; the library allocates none of it.  It holds:
 *   COO, CSR: tiles of a fixed number of entries with their first rows and
 *     flags, and the carries mxs_spmv puts the partial sums of rows that span
 *     tiles in;
 *   CSR: an ELL copy when rows have near-equal lengths (at most 5% padding
 *     slots; skipped with MXS_PLAN_NO_ELL);
 *   COO, CSR: column blocks when x is large and the entries scattered
 *     (see implementation CSR 4 below; skipped with MXS_PLAN_NO_COLBLK);
 *   DIA: a row-blocked copy of the values, only with MXS_PLAN_DIA_BLOCKED
 *     (measured within 3% of the diagonal-major kernel on the stencil);
 *   split and HYB handles: their two parts' plans; ELL, SELL: nothing. */
#define MXS_PLAN_NO_ELL 1u      /* CSR: no ELL copy (implementation 3 not applicable) */
#define MXS_PLAN_NO_COLBLK 2u   /* COO, CSR: no column blocks */
#define MXS_PLAN_DIA_BLOCKED 4u /* DIA: make the row-blocked copy (implementations 0, 1) */

/* Bytes of workspace mxs_optimize(A, opts, ...) needs [syncs].  It measures
 * what the layout depends on (longest row, scattered entries, entries per
 * column block) on the device with a 4 KiB temporary it frees before
 * returning.  The bytes include temporaries used only while the plan is
 * built.  Parts of split matrices and column blocks are planned with their
 * parent: MXS_ERR_INVALID_ARG for them, and for unknown option bits. */
mxs_status mxs_plan_size(mxs_mat A, unsigned opts, size_t *bytes, void *stream);

/* Builds A's plan in workspace[bytes] (device memory, 256-byte aligned,
 * bytes >= mxs_plan_size(A, opts)) [syncs]; allocates nothing.  A plan built
 * earlier is dropped first (its memory may be reused as this workspace, or
 * freed once this returns); no other call on A may be in flight meanwhile.
 * MXS_ERR_INVALID_ARG for a workspace that is too small or misaligned; on
 * any failure A is left without a plan.
 * Every call below that runs SpMV kernels on A returns MXS_ERR_NO_PLAN until
 * A has a plan: mxs_spmv, mxs_spmv_ws, mxs_set_impl, mxs_get_impl,
 * mxs_tune, mxs_cg_solve (A and A32), mxs_pcg_solve. */
mxs_status mxs_optimize(mxs_mat A, unsigned opts, void *workspace, size_t bytes, void *stream);

/* Whether A has a plan, and its options [host only]; either pointer may be NULL. */
mxs_status mxs_plan_info(mxs_mat A, int32_t *optimized, unsigned *opts);

/* SpMV implementations (Section III keeps one kernel per format; no single
 * kernel wins on every matrix, so each format here has several, all giving
 * the same sums within rounding):
 *   COO  0: row tiles (the CSR tiling rebuilt from the row ids; applicable
 *           when no tile owns more than 512 rows)
 *        1: segmented-scan tiles (always applicable)
 *        2: column blocks, as CSR's 4 below, each block a COO matrix
 *   CSR  0: tiles of a fixed number of entries   1: a thread per row
 *        2: entry tiles, columns and values staged in LDS, x gathered per
 *           row   3: a lane per row over an ELL copy made by mxs_optimize
 *           (applicable when that copy adds at most 5% slots)
 *        4: column blocks: mxs_optimize splits the entries by column range
 *           into K full-height CSR blocks whose part of x about fits one
 *           XCD's 4 MiB L2 (K = ceil(x bytes / 6 MiB), at most 32) and runs them
 *           in turn, the first writing y and the others adding to it
 *           (applicable when x is at least 8 MiB, the rows hold at least
 *           three entries on average, and at least half of the
 *           entries lie half a block or more from the diagonal and read x
 *           from another 128-byte line than the row's previous entry; the copy
 *           takes as much memory as the entries, plus K row-pointer arrays
 *           for CSR)   5: a wavefront per row (lanes stride over the row)
 *   DIA  0: row-blocked values, one x load per run of three consecutive
 *           offsets (needs the row-blocked copy and offsets in such runs)
 *        1: row-blocked values (needs the copy)
 *        2: diagonal-major values as stored (always applicable)
 * After mxs_optimize the default is: COO 2 where applicable, else 0 where
 * applicable, else 1; CSR 4
 * where applicable, else 3 where applicable, else 1 when nrows > 2*nnz,
 * else 0; DIA the lowest
 * applicable id; ELL and SELL have one implementation, 0.
 * mxs_impl_count: number of ids of A's format (0 for split matrices).
 * mxs_set_impl [host only]: MXS_ERR_UNSUPPORTED for an id that is not
 *   applicable to A or a split matrix.
 * mxs_get_impl [host only]: the active id.
 * mxs_tune [syncs]: runs every applicable implementation (3 untimed calls,
 *   then `reps` >= 1 timed calls y = A*x each), keeps the one with the
 *   smallest median time and returns its id; ms[mxs_impl_count] (may be
 *   NULL) receives each median in milliseconds, -1 where not applicable.
 *   y is overwritten with A*x.  Split matrices: MXS_ERR_UNSUPPORTED.
 * Changing the implementation must not overlap other calls on the handle. */
int32_t mxs_impl_count(mxs_mat A);
mxs_status mxs_set_impl(mxs_mat A, int32_t impl, void *stream);
mxs_status mxs_get_impl(mxs_mat A, int32_t *impl, void *stream);
mxs_status mxs_tune(mxs_mat A, const void *x, void *y, int32_t reps, int32_t *impl,
                    double *ms, void *stream);

/* y = A*x, overwriting y[nrows]; x has ncols entries [async].  Entry-wise
 * the result is sum over stored (i, j, v) of v*x[j] (Algorithm 1 with y
 * cleared first, which is what Algorithms 2 and 3 compute).  Summation
 * order differs from a sequential loop; results are deterministic (no
 * floating-point atomics).  x and y must not overlap (MXS_ERR_INVALID_ARG).
 * Rows without entries get 0.  Never builds a plan (MXS_ERR_NO_PLAN without
 * one) and allocates nothing.  The plan's carries (partial sums of rows that
 * span tiles) are shared by every mxs_spmv on the handle: calls on one
 * handle issued to different streams must not overlap (use mxs_spmv_ws);
 * calls on one stream are ordered. */
mxs_status mxs_spmv(mxs_mat A, const void *x, void *y, void *stream);

/* Bytes of scratch mxs_spmv_ws needs for A's carries (0 when none) [host
 * only; MXS_ERR_NO_PLAN without a plan]. */
mxs_status mxs_spmv_scratch_size(mxs_mat A, size_t *bytes);

/* mxs_spmv with the carries in the caller's scratch[bytes] (device, not
 * overlapping x or y; may be NULL when mxs_spmv_scratch_size gives 0)
 * instead of the plan's [async].  Calls on one handle from different streams
 * may overlap when each has its own scratch; the results equal mxs_spmv's
 * bit for bit. */
mxs_status mxs_spmv_ws(mxs_mat A, const void *x, void *y, void *scratch, size_t bytes,
                       void *stream);

/* Dot product a.b of n values of `dtype`, accumulated in FP64, written to
 * the device double *result [async].  Deterministic. */
mxs_status mxs_dot(int64_t n, mxs_dtype dtype, const void *a, const void *b, double *result,
                   void *stream);

/* mxs_dot without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc) [async].  Same arguments, kernels and result, bit for bit, as
 * mxs_dot; the workgroup partials go to a fixed array of 8,192 FP64 values
 * (64 KiB) that the library keeps on each GPU it runs on until the process
 * ends, instead of a buffer allocated per call.  A call that would need more
 * partials than the array holds is refused with MXS_ERR_UNSUPPORTED (detail
 * in mxs_last_error); the grid is capped at the array's size, so no n is
 * refused today.  Calls that overlap on one GPU (different streams, or threads
 * without ordering) share the array and race; calls on one stream are
 * ordered.  The first call on a device looks up the array's address there. */
mxs_status mxs_dot_noalloc(int64_t n, mxs_dtype dtype, const void *a, const void *b,
                           double *result, void *stream);

/* y = alpha*x + beta*y over n values of `dtype` [async]. */
mxs_status mxs_axpby(int64_t n, mxs_dtype dtype, double alpha, const void *x, double beta,
                     void *y, void *stream);

/* ------------------------------------------------------------------------
 * Conjugate gradients: HPCG's solver with the preconditioner disabled
 * (Section VII-D), and an FP32-inner / FP64-outer refinement built on it.
 * --------------------------------------------------------------------- */

typedef struct {
    double rtol;         /* FP64 CG: stop when ||r_k|| <= rtol*||r_0|| (recursive r).
                            Mixed: stop when ||b - A x|| <= rtol*||b|| (FP64). */
    int64_t maxit;       /* FP64 CG and mixed = 2: iteration cap.  mixed = 1: cap per
                            inner solve. */
    int32_t mixed;       /* 0: FP64 CG on A.
                            1: iterative refinement: r = b - A x in FP64, an FP32 CG on
                               A32 solves for the correction from zero, x += correction;
                               repeated until converged or max_outer corrections.
                            2: reliable updates: one FP32 CG on A32 whose accumulated
                               correction is added to x in FP64, and whose residual is
                               replaced by b - A x (FP64), whenever its recursive
                               residual falls to ru_delta times its largest value since
                               the last update, or to rtol*||b||; the search direction
                               is kept (van der Vorst and Ye's residual replacement). */
    int32_t max_outer;   /* mixed = 1: at most this many corrections */
    double inner_rtol;   /* mixed = 1: inner solves stop at ||r|| <= inner_rtol*||r_0|| */
    int32_t check_every; /* host reads the device convergence flag every this many
                            iterations (>= 1); iterations past convergence are no-ops.
                            mixed = 2 without timing: the host also enqueues a residual
                            replacement when it reads that one is pending (the steps
                            after the one that asked for it return at entry until
                            then); the result does not depend on check_every */
    int32_t timing;      /* 1: time SpMV, dot and vector-update kernels with events
                            (mixed = 2 counts its FP64 updates as vector updates) */
    double ru_delta;     /* mixed = 2: update factor in [0, 1] */
} mxs_cg_opts;

typedef struct {
    int64_t iters;         /* FP64: CG iterations (loop SpMVs).  Mixed: FP32 iterations */
    int64_t outer_iters;   /* mixed = 1: corrections applied; mixed = 2: reliable updates
                              triggered; FP64: 0 */
    double rel_resid;      /* FP64: ||r_k||/||r_0|| (recursive).  Mixed: ||b-Ax||/||b|| */
    double true_rel_resid; /* ||b - A x||/||b|| from an FP64 SpMV at exit */
    double t_spmv_ms;      /* timing = 1: summed kernel times per class; else 0 */
    double t_dot_ms;
    double t_axpy_ms;
    double t_precond_ms;   /* PCG with timing = 1: the preconditioner's time; else 0 */
} mxs_cg_result;

/* Bytes of device workspace mxs_cg_solve needs for A (n = nrows). */
mxs_status mxs_cg_workspace_size(mxs_mat A, int32_t mixed, size_t *bytes);

/* Solves A x = b (A square, symmetric positive definite, FP64) [syncs].
 * x holds x0 on entry and the solution on exit; b and x are FP64 device
 * vectors of nrows entries.  With opts->mixed = 1 or 2, A32 must be an FP32
 * handle of the same matrix (e.g. from mxs_cast) used by the FP32 recurrences.
 * Returns MXS_OK on convergence, MXS_NOT_CONVERGED at the cap (x valid),
 * MXS_ERR_BREAKDOWN when p.Ap <= 0 (x holds the last iterate),
 * MXS_ERR_NONFINITE for NaN/Inf in b or x0, MXS_ERR_INVALID_ARG for a
 * non-square A or a workspace smaller than mxs_cg_workspace_size. */
mxs_status mxs_cg_solve(mxs_mat A, mxs_mat A32, const double *b, double *x,
                        const mxs_cg_opts *opts, mxs_cg_result *res, void *workspace,
                        size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Split matrices (MXS_HDC): a DIA band plus a remainder.  The hybrid
 * DIA/CSR format is among the further formats of Section IX; the
 * distributed HPCG runs of Section VII-D split each process's matrix into a
 * local part and a remote part with separate formats (Table III).
 * --------------------------------------------------------------------- */

/* Sizes of the split of A (COO or CSR) [syncs]: the band is the diagonals
 * that hold at least one entry and at least min_fill times as many entries
 * as they have slots inside the matrix (compared in FP64); *band_ndiag gets
 * their number and *rest_nnz the number of entries off them. */
mxs_status mxs_split_size(mxs_mat A, double min_fill, int32_t *band_ndiag, int64_t *rest_nnz,
                          void *stream);

/* Splits A (COO or CSR) [syncs] into caller-allocated arrays: the band as
 * DIA (band_doff[band_ndiag] ascending, band_vals[band_ndiag*nrows]
 * diagonal-major with +0.0 in empty slots) and the remaining entries in
 * rest_format, MXS_COO (rest_idx0 = row ids [rest_nnz]) or MXS_CSR
 * (rest_idx0 = row pointers [nrows+1]), with rest_idx1 = columns and
 * rest_vals = values [rest_nnz], in canonical order.  *out is an MXS_HDC
 * handle that borrows all of these arrays (nnz = band in-range slots plus
 * remainder entries; ndiag = band diagonals); mxs_spmv on it computes y = A x
 * as the band's product plus the remainder's, and mxs_cg_solve accepts it
 * (FP64, mixed = 0).  Conversion, cast and features of an MXS_HDC handle
 * return MXS_ERR_UNSUPPORTED. */
mxs_status mxs_split(mxs_mat A, double min_fill, mxs_format rest_format, int32_t *band_doff,
                     void *band_vals, int32_t *rest_idx0, int32_t *rest_idx1, void *rest_vals,
                     mxs_mat *out, void *stream);

/* HYB (Section IX's hybrid formats; Bell and Garland, 2009): each row's
 * first K entries in ELL (column-major, padding column -1 and +0.0), the
 * rest in COO (canonical order).  K < 0 asks for the width rule: the
 * largest k such that at least max(4096, nrows/3) rows (all rows when
 * fewer) hold k or more entries.
 * mxs_hyb_size [syncs]: *K_out, and *rest_nnz entries past the K-th of
 *   their row; refused with MXS_ERR_DIA_TOO_SPARSE when K*nrows > 8*nnz.
 * mxs_to_hyb [syncs]: writes ell_col, ell_val [K*nrows] and rest_ai,
 *   rest_aj, rest_av [rest_nnz] (caller-allocated) and returns an MXS_HYB
 *   handle that borrows them (ndiag = K); SpMV and FP64 CG accept it, and
 *   mxs_split_parts gives its ELL and COO parts; conversion, cast, features
 *   and mixed solves do not (MXS_ERR_UNSUPPORTED).  A is COO or CSR. */
mxs_status mxs_hyb_size(mxs_mat A, int32_t K, int32_t *K_out, int64_t *rest_nnz, void *stream);
mxs_status mxs_to_hyb(mxs_mat A, int32_t K, int32_t *ell_col, void *ell_val, int32_t *rest_ai,
                      int32_t *rest_aj, void *rest_av, mxs_mat *out, void *stream);

/* The two parts of a split or HYB matrix H as handles of their own [host
 * only]: *band (MXS_DIA for a split, MXS_ELL for HYB) and *rest (MXS_COO or
 * MXS_CSR), either pointer may be NULL.  They stay valid until H is destroyed and belong to H: mxs_destroy
 * on a part returns MXS_ERR_INVALID_ARG.  Every other call accepts them, so
 * each part's implementation can be chosen (mxs_set_impl, mxs_tune); the
 * choice holds for H's product.  MXS_ERR_UNSUPPORTED if H is neither MXS_HDC nor MXS_HYB. */
mxs_status mxs_split_parts(mxs_mat H, mxs_mat *band, mxs_mat *rest);

/* ------------------------------------------------------------------------
 * HPCG's preconditioner (Section VII-D: CG preconditioned by a multigrid
 * cycle with a symmetric Gauss-Seidel smoother; HPCG's cycle in full).
 *
 * Level l (0 finest) is the 27-point stencil (26 on the diagonal, -1 off it)
 * on the (n >> l)^3 grid, rows x-fastest.  The smoother is one symmetric
 * Gauss-Seidel sweep in multicolour order: the colour of a point is the
 * parity of its coordinates, c = (ix & 1) + 2 (iy & 1) + 4 (iz & 1); the
 * forward sweep visits colours 1, 2, ..., 7, 0 (ascending rows inside a
 * colour), the backward sweep the reverse; row i becomes
 * x_i = (r_i - sum_{j != i} a_ij x_j) / a_ii.  Points of one colour never
 * couple, so each colour updates in parallel and the sweep equals the
 * sequential one in that order.  The V-cycle: z = 0, one sweep, coarse
 * right-hand side r_c = (r - A z) at the points (2i, 2j, 2k) (injection),
 * the cycle on the next level from zero, z += its result at those points,
 * one more sweep; on the coarsest level one sweep from zero.
 * --------------------------------------------------------------------- */

/* Bytes of device workspace the hierarchy of mxs_mg_create(n, levels) needs
 * [host only]: each level's CSR operator, a copy of its off-diagonal entries
 * sliced for the smoother, its diagonal and colour order, two vectors per
 * coarse level, and temporaries used only while it is built.  Shape rules
 * as for mxs_mg_create. */
mxs_status mxs_mg_size(int32_t n, int32_t levels, size_t *bytes);

/* Builds the hierarchy [syncs] in the caller's workspace[bytes] (device,
 * 256-byte aligned, bytes >= mxs_mg_size; kept alive and unchanged until
 * mxs_mg_destroy); allocates no device memory.  n >= 1 divisible by
 * 2^(levels-1), levels in [1, 12] (MXS_ERR_INVALID_ARG otherwise, and for a
 * workspace that is too small); n^3 rows and (3n-2)^3 entries within int32
 * (else MXS_ERR_UNSUPPORTED).  Calls on one hierarchy must not overlap
 * (they share the coarse vectors). */
mxs_status mxs_mg_create(int32_t n, int32_t levels, void *workspace, size_t bytes, mxs_mg *out,
                         void *stream);
mxs_status mxs_mg_destroy(mxs_mg M);

/* Grid edge and operator (an MXS_CSR handle owned by M: mxs_destroy on it
 * returns MXS_ERR_INVALID_ARG) of level `level` [host only]. */
mxs_status mxs_mg_level(mxs_mg M, int32_t level, int32_t *n, mxs_mat *A);

/* One symmetric Gauss-Seidel sweep of level `level` on x in place, with
 * right-hand side r (FP64 device vectors of the level's rows; x and r must
 * not overlap) [async]. */
mxs_status mxs_symgs(mxs_mg M, int32_t level, const double *r, double *x, void *stream);

/* z = M^{-1} r, one V-cycle from the finest level (r, z FP64 device
 * vectors of n^3 entries, not overlapping) [async]. */
mxs_status mxs_mg_apply(mxs_mg M, const double *r, double *z, void *stream);

/* Bytes of device workspace mxs_pcg_solve needs. */
mxs_status mxs_pcg_workspace_size(mxs_mg M, size_t *bytes);

/* PCG on A x = b with z = M^{-1} r (HPCG's recurrences: beta = r.z over the
 * previous r.z, alpha = r.z / p.Ap; stop when ||r_k|| <= rtol ||r_0||)
 * [syncs].  A is the finest operator in any FP64 format (NULL: M's own CSR
 * operator from mxs_mg_level, which then needs a plan of its own); it must
 * be that matrix.  opts: rtol, maxit, check_every and
 * timing as for mxs_cg_solve; mixed must be 0.  Statuses as mxs_cg_solve,
 * and MXS_ERR_BREAKDOWN also when r.z <= 0. */
mxs_status mxs_pcg_solve(mxs_mg M, mxs_mat A, const double *b, double *x,
                         const mxs_cg_opts *opts, mxs_cg_result *res, void *workspace,
                         size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * HPCG problem setup (Section VII-D: Poisson on a regular 3-D grid)
 * --------------------------------------------------------------------- */

/* Number of stored entries of the n^3 stencil with `points` = 7 or 27. */
int64_t mxs_stencil_nnz(int32_t n, int32_t points);

/* Writes the n^3 stencil as canonical COO [async]: grid point (x,y,z) is
 * row x + n*y + n*n*z; an entry for every neighbour inside the grid
 * (27-point: all of {-1,0,1}^3; 7-point: the centre and the six faces),
 * `diag` on the diagonal and `offdiag` elsewhere.  ai, aj, av hold
 * mxs_stencil_nnz(n, points) entries; av has `dtype`. */
mxs_status mxs_stencil_coo(int32_t n, int32_t points, double diag, double offdiag,
                           int32_t *ai, int32_t *aj, void *av, mxs_dtype dtype, void *stream);

/* ------------------------------------------------------------------------
 * Format selection (the run-first tuner of Section VII-D and the dynamic
 * selection named as further work in Section IX): matrix features and a
 * small MLP 8-64-64-7 (FP32) with its training step.  Its outputs are the
 * label set's formats in this order: COO, CSR, DIA, ELL, SELL-64-1, HYB,
 * HDC (a DIA band of the diagonals at least half full plus a COO
 * remainder).
 * --------------------------------------------------------------------- */

#define MXS_NFEAT 8
#define MXS_NCLASS 7
#define MXS_MLP_NPARAM 5191

/* Eight features of A's stored entries into host out[8] [syncs]:
 *   0 rows, 1 nnz, 2 mean row length, 3 population variance of row lengths,
 *   4 max row length, 5 number of distinct diagonals j-i,
 *   6 DIA fill ratio nnz/(ndiag*rows), 7 max |j-i| / ncols.
 * For a DIA handle the features are those of its non-zero slots. */
mxs_status mxs_features(mxs_mat A, double out[8], void *stream);

/* Network input from raw features [async]: X[s][f] = (t(raw[s][f]) - mu[f]) / sd[f]
 * with t = log1p for features 0-5 and identity for 6-7.  raw is FP64
 * [n][8], X, mu and sd are FP32. */
mxs_status mxs_mlp_inputs(const double *raw, int32_t n, const float *mu, const float *sd,
                          float *X, void *stream);

/* Normalisation statistics of a training set [async]: mu[f], sd[f] are the
 * mean and population standard deviation over the n samples of t(raw[s][f])
 * (t as in mxs_mlp_inputs), accumulated in FP64; sd is replaced by 1 where
 * it is 0 or below 1e-6 |mu| (a constant feature up to rounding). */
mxs_status mxs_mlp_norm_stats(const double *raw, int32_t n, float *mu, float *sd,
                              void *stream);

/* Logits[n][MXS_NCLASS] of the MLP with parameters w[MXS_MLP_NPARAM] laid out as
 * W1[8][64], b1[64], W2[64][64], b2[64], W3[64][7], b3[7] (row-major,
 * input index first), ReLU hidden layers [async]. */
mxs_status mxs_mlp_forward(const float *w, const float *X, int32_t n, float *logits,
                           void *stream);

/* fmt_out[s] = argmax over formats f with feasible[s*MXS_NCLASS+f] != 0 of the
 * logits (feasible may be NULL: all allowed); -1 if none is feasible [async]. */
mxs_status mxs_mlp_predict(const float *w, const float *X, int32_t n, const uint8_t *feasible,
                           int32_t *fmt_out, void *stream);

/* Bytes of device workspace for mxs_mlp_grad / mxs_mlp_train_step with n
 * samples (per-sample activations and deltas, then the gradient). */
size_t mxs_mlp_workspace_size(int32_t n);

/* Mean softmax cross-entropy over n samples (labels in {0,...,MXS_NCLASS-1}) into the
 * device float *loss and its gradient grad[MXS_MLP_NPARAM] [async].
 * Deterministic. */
mxs_status mxs_mlp_grad(const float *w, const float *X, const int32_t *labels, int32_t n,
                        float *grad, float *loss, void *workspace, size_t bytes, void *stream);

/* One Adam step (Kingma and Ba 2015) at step t >= 1 on w, m, v [async]. */
mxs_status mxs_mlp_adam(float *w, float *m, float *v, const float *grad, float lr, int32_t t,
                        float beta1, float beta2, float eps, void *stream);

/* mxs_mlp_grad followed by mxs_mlp_adam (beta1 0.9, beta2 0.999, eps 1e-8) [async]. */
mxs_status mxs_mlp_train_step(float *w, float *m, float *v, const float *X,
                              const int32_t *labels, int32_t n, float lr, int32_t t,
                              float *loss, void *workspace, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MXS_H */
