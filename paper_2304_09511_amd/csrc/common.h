// Internal declarations of libmxs: the handle, device helpers and the
// launchers each translation unit provides.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "mxs.h"

namespace mxs {

constexpr int kWave = 64;  // CDNA wavefront width
constexpr int kNumXcd = 8; // MI355X: 8 accelerator complex dies, 32 CUs each

// ---------------------------------------------------------------------------
// Error plumbing
// ---------------------------------------------------------------------------
// Records a failed HIP call (error name, message and source position) for
// mxs_last_error(); returns the status it maps to.
mxs_status note_hip_error(hipError_t e, const char *where);
// The text mxs_last_error() returns (per thread).
extern thread_local char g_last_error[512];

#define MXS_STR2(x) #x
#define MXS_STR(x) MXS_STR2(x)
#define MXS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::mxs::note_hip_error(e_, #call " (" __FILE__ ":" MXS_STR(__LINE__) ")"); \
    } while (0)

inline mxs_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return MXS_OK;
    if (e == hipErrorOutOfMemory) return MXS_ERR_OUT_OF_MEMORY;
    return MXS_ERR_HIP;
}

// Checks the launch that was just enqueued.
inline mxs_status launch_status()
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MXS_OK : note_hip_error(e, "kernel launch");
}

// ---------------------------------------------------------------------------
// CG state kept in device memory (one per solve level)
// ---------------------------------------------------------------------------
struct CgState {
    double rho0;     // r0.r0
    double rho;      // r.r of the current iterate
    double sigma;    // p.Ap
    double alpha;    // rho / sigma
    double beta;     // rho_new / rho
    double rtol;     // stopping tolerance (relative to sqrt(rho0))
    double rr;       // last reduced value of an auxiliary dot (residual norms)
    long long iters; // loop SpMVs done
    long long maxit;
    int done;        // 1: every later CG kernel returns at entry
    int status;      // mxs_status of the solve
    int nonfinite;   // set when an input vector holds NaN or Inf
    int pad;
    // mixed CG with reliable updates
    double rmax;     // largest recursive residual norm since the last update
    double delta;    // update when the residual norm drops to delta * rmax
    double thresh;   // rtol * ||b||: stop on ||b - A x|| <= thresh
    double rtrue2;   // ||b - A x||^2 at the last update
    long long nupd;  // updates made
    int noupd;       // 0 only while an update is pending (update kernels run)
    int last;        // the pending update is the last allowed (iteration cap)
    // plain CG whose r.r is reduced inside the direction update
    // (cg_rho_p_kernel): that launch may not write rho while its workgroups
    // read it, so it leaves the new value here and the next finish of p.Ap
    // moves it into rho
    double rho_next;
    int rho_pend;    // 1: rho_next holds the new rho
    int rmax_pend;   // 1: rmax_next holds the new rmax (reliable updates, same reason)
    double rmax_next;
};

// Where a fused dot product of an SpMV epilogue goes: one partial per
// workgroup, then a finish kernel computes alpha = rho / (p.Ap) into st.
struct DotSink {
    double *partials;
    CgState *st;
};

// ---------------------------------------------------------------------------
// The matrix handle
// ---------------------------------------------------------------------------
}  // namespace mxs
struct mxs_mat_s;
namespace mxs {

struct CsrPlan {
    int32_t *tile_row = nullptr; // [ntiles+1] first row owned by each tile (sentinel nrows)
    int32_t *tile_info = nullptr; // [ntiles] overflow length and carry flags
    void *carry = nullptr;       // [2*ntiles] head / tail pieces of rows too long to finish
    int64_t ntiles = 0;
    int32_t tile = 0;            // entries per tile (256 threads x entries per thread)
    bool fixup = false;          // some row reaches past its owner's overflow window
    bool rowwise = false;        // a thread per row (default when rows outnumber entries 2:1)
    bool gx = false;             // entry tiles, x gathered per row from LDS-staged columns
    // ELL copy (implementation 3), made when it adds at most 5% slots:
    // K slots per row, column-major, padding column -1
    int32_t ell_k = 0;
    int32_t *ell_col = nullptr;
    void *ell_val = nullptr;
    bool ell = false;            // the active implementation reads it
    bool vec = false;            // a wavefront per row (implementation 5)
};

struct DiaPlan {
    void *blk = nullptr;     // values re-laid out by row block: [block][diagonal][row in block]
    int32_t *pos = nullptr;  // [ndiag] LDS position of each diagonal's x window start
    int32_t *runs = nullptr; // [3*nruns] first offset, length, LDS base of each x window
    int32_t nruns = 0;
    int32_t lds_elems = 0;   // x-window LDS per block in elements (0: windows off)
    int32_t first_off = 0, last_off = 0;
    int32_t triples = 0;     // 1: offsets form runs o, o+1, o+2 (ndiag a multiple of 3)
    bool use_blk = false;    // the active implementation reads the row-blocked copy
    bool use_share = false;  // ... and shares x loads over runs of three offsets
};

struct CooPlan {
    // the active implementation's tiles and carries
    bool rows = false;     // row tiles (else segmented-scan tiles)
    void *carry = nullptr; // [2*ntiles] values: head partial, tail partial
    int64_t ntiles = 0;
    // Row tiles (the CSR tiling; possible when no tile owns more rows than
    // fit in LDS): first owned row and extension/carry word per tile.
    bool rows_ok = false;
    int32_t *tile_row = nullptr; // [nt_rows + 1]
    int32_t *tile_info = nullptr; // [nt_rows]
    bool fixup = false;           // some row is longer than its owner's window
    int64_t nt_rows = 0, nt_seg = 0;
    int32_t seg_tile = 0;         // entries per segmented tile
    void *carry_rows = nullptr, *carry_seg = nullptr;
};

}  // namespace mxs

struct mxs_mat_s;
// a split (DIA band) or HYB (ELL part) handle: two parts, band then rest
inline bool is_split(const mxs_mat_s *A);

struct mxs_mat_s {
    mxs_format fmt = MXS_CSR;
    mxs_dtype dtype = MXS_F64;
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;     // COO/CSR: stored entries; DIA: in-range slots
    int32_t ndiag = 0;   // DIA only
    const int32_t *idx0 = nullptr; // COO ai | CSR irp | DIA doff
    const int32_t *idx1 = nullptr; // COO aj | CSR aj  | DIA unused
    const void *vals = nullptr;    // values
    std::vector<void *> owned;     // device allocations freed by mxs_destroy
    int device = 0;
    std::mutex mu;
    bool optimized = false;
    int32_t impl = -1; // active SpMV implementation (see mxs_set_impl)
    mxs::CsrPlan csr;
    mxs::CooPlan coo;
    mxs::DiaPlan dia;
    // COO and CSR column blocks (colblk.hip): the entries split by column
    // range into full-height part handles of the same format, run in turn
    std::vector<mxs_mat_s *> cblk;
    bool colblk = false;       // the active implementation runs them
    mxs_mat_s *band = nullptr; // HDC: the DIA band (owned by this handle)
    mxs_mat_s *rest = nullptr; // HDC: the COO or CSR remainder (owned)
    bool part = false;         // owned by another handle or a hierarchy (not destroyable)
    bool sub = false;          // a split's band or remainder, or a column block: its plan
                               // is laid out inside its parent's
    bool cblk_part = false;    // a column block (its columns scattered by construction)
    unsigned plan_opts = 0;    // options of the current plan (mxs_optimize)
    // ELL: ndiag = slots per row.  SELL: idx0 = columns, idx1 = perm,
    // sell_cs = slice offsets, slots = sell_cs[nslices], sigma = sort window.
    const int64_t *sell_cs = nullptr;
    int64_t slots = 0;
    int32_t sigma = 0;
};

inline bool is_split(const mxs_mat_s *A) { return A->fmt == MXS_HDC || A->fmt == MXS_HYB; }

namespace mxs {
// ---------------------------------------------------------------------------
// Plan memory (mxs_plan_size, mxs_optimize)
// ---------------------------------------------------------------------------
// A plan is laid out twice by the same code: a sizing pass, in which nothing
// is written and every take only counts bytes, and a build pass into the
// caller's workspace.  What the layout depends on (the longest row, the
// count of scattered entries, entries per column block) is measured in both
// passes with a few device counters (`tiny`), so both passes take the same
// arrays in the same order.  Workspace layout:
//   [arrays the plan keeps][tiny counters][temporaries of the build]
// The temporaries are dead once mxs_optimize returns.
constexpr size_t kPlanAlign = 256;
constexpr size_t kTinyBytes = 4096;

struct PlanCtx {
    unsigned opts = 0;
    bool build = false;        // false: the sizing pass (nothing is written)
    char *keep_base = nullptr; // build pass: where kept arrays go
    size_t keep_used = 0;
    char *tmp_base = nullptr;  // build pass: temporaries
    size_t tmp_used = 0, tmp_peak = 0;
    void *tiny = nullptr;      // kTinyBytes of device counters, both passes (nullptr: none)
    bool tiny_used = false;

    static size_t up(size_t b) { return (b + kPlanAlign - 1) / kPlanAlign * kPlanAlign; }
    // an array the plan keeps
    void *keep(size_t bytes)
    {
        keep_used = up(keep_used);
        void *p = build ? keep_base + keep_used : nullptr;
        keep_used += bytes;
        return p;
    }
    // a temporary, given back with release(mark())
    void *tmp(size_t bytes)
    {
        tmp_used = up(tmp_used);
        void *p = build ? tmp_base + tmp_used : nullptr;
        tmp_used += bytes;
        tmp_peak = tmp_used > tmp_peak ? tmp_used : tmp_peak;
        return p;
    }
    size_t mark() const { return tmp_used; }
    void release(size_t m) { tmp_used = m; }
    // device counters of a measurement taken in both passes (nullptr: the
    // caller's workspace is too small to hold them)
    void *counters()
    {
        tiny_used = true;
        return tiny;
    }
    // workspace bytes of the layout
    size_t total() const { return up(keep_used) + (tiny_used ? kTinyBytes : 0) + tmp_peak; }
};

// One grid of the multigrid hierarchy (mg.hip).
struct MgLevel {
    int32_t n = 0, rows = 0;  // grid edge, rows = n^3
    mxs_mat_s *A = nullptr;   // the level's CSR operator (owned by the hierarchy)
    int32_t coff[9] = {};     // colour c holds positions [coff[c], coff[c+1]) of order
    int32_t sfirst[9] = {};   // first slice of colour c (sfirst[8]: slice count)
    int32_t nslices = 0;
    int32_t *order = nullptr; // row id at each position (colour order)
    int64_t *soff = nullptr;  // [nslices+1] first entry of each 64-row slice
    int32_t *col = nullptr;   // off-diagonal columns, slice column-major, padded
    double *val = nullptr;    // their values (0 in padding)
    double *diag = nullptr;   // a_ii at each position
    double *r = nullptr, *z = nullptr; // right-hand side and correction (coarse levels)
};
}  // namespace mxs

struct mxs_mg_s {
    std::vector<mxs::MgLevel> lv; // finest first; arrays in the caller's workspace
    int device = 0;
};


namespace mxs {

inline size_t dsize(mxs_dtype t) { return t == MXS_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b % 8).  The remap gives each XCD a contiguous range of logical
// blocks, so rows that share x entries meet in the same L2.  The grid must
// be padded to a multiple of 8; logical ids >= the real count must exit.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t grid)
{
    const uint32_t per = grid / kNumXcd;
    return (bid % kNumXcd) * per + bid / kNumXcd;
}

inline uint32_t pad_grid(int64_t nblocks)
{
    return (uint32_t)(((nblocks + kNumXcd - 1) / kNumXcd) * kNumXcd);
}

// Butterfly sum over the 64 lanes: every lane ends with the same value,
// independent of scheduling.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over the workgroup (NT threads); the result is valid in thread 0.
// smem must hold NT/64 doubles.  Fixed combination order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *smem)
{
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (NT > kWave) {
        if (l == 0) smem[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NT / kWave; ++i) s += smem[i];
            v = s;
        }
        __syncthreads();
    }
    return v;
}

// Sum of n partials (one per workgroup of the producing kernel) in index
// order, run by a single workgroup of NT threads; valid in thread 0.  The
// producing kernel has finished (kernel boundary), so plain loads see every
// partial: no device-scope fences are needed.
template <int NT>
__device__ __forceinline__ double reduce_partials(const double *__restrict__ partials, int64_t n,
                                                  double *smem)
{
    // thread t sums partials t, t + NT, ... in eight interleaved accumulators,
    // eight loads in flight per round; the last round is masked, its loads
    // still issued together (a partial round summed one load at a time cost a
    // dependent round trip per partial), then the fixed combination below
    constexpr int U = 8;
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += (int64_t)U * NT) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i + (int64_t)u * NT < n ? partials[i + (int64_t)u * NT] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += v[u];
    }
    const double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    return block_sum<NT>(v, smem);
}

// Threads of the single-workgroup kernels that reduce partials.
constexpr int kFinNT = 1024;

// Finisher of the fused p.Ap: one loop SpMV done; alpha = rho / sigma, or a
// breakdown when sigma <= 0 or not finite.
__device__ __forceinline__ void cg_finish_sigma(CgState *st, double sigma)
{
    if (st->rho_pend) {
        st->rho = st->rho_next;
        st->rho_pend = 0;
    }
    if (st->rmax_pend) {
        st->rmax = st->rmax_next;
        st->rmax_pend = 0;
    }
    st->sigma = sigma;
    st->iters += 1;
    if (!(sigma > 0.0) || !__builtin_isfinite(sigma)) {
        st->status = (int)MXS_ERR_BREAKDOWN;
        st->alpha = 0.0;
        st->done = 1;
    } else {
        st->alpha = st->rho / sigma;
    }
}

// ---------------------------------------------------------------------------
// Launchers provided by the translation units
// ---------------------------------------------------------------------------

// spmv.hip.  `done` (nullable) makes every workgroup return at entry when
// *done != 0; `dot` (nullable, square A only) fuses sum_i y_i*x_i into the
// epilogue and launches the finish kernel that applies cg_finish_sigma.
mxs_status spmv_launch(const mxs_mat_s *A, const void *x, void *y, const int *done,
                       const DotSink *dot, hipStream_t s, void *carry = nullptr);
// `carry` (nullable): where the tile kernels put the partial sums of rows
// that span tiles, spmv_scratch_bytes(A) bytes; nullptr: the plan's own.
// p.Ap (n = nrows) reduced into `dot` as the COO path and the timed CG path do.
mxs_status dot_sigma_launch(int64_t n, mxs_dtype t, const void *a, const void *b, const int *done,
                            const DotSink *dot, hipStream_t s);
// Number of per-workgroup partials the fused dot of spmv_launch writes.
int64_t spmv_dot_parts(const mxs_mat_s *A);
// Capacity of every partials array (workgroups of any reducing launch).
constexpr int64_t kMaxParts = 1 << 18;
// Lays out (sizing pass) or builds (build pass) A's plan; see PlanCtx.
mxs_status plan_walk(mxs_mat_s *A, PlanCtx &c, hipStream_t s);
// Forgets A's plan (and its parts' and column blocks'); the memory is the caller's.
void plan_reset(mxs_mat_s *A);
// Bytes of the scratch mxs_spmv_ws takes for A's carries (0 when none).
size_t spmv_scratch_bytes(const mxs_mat_s *A);
// spmv.hip: the SpMV implementations of a format and the choice among them.
int32_t impl_count(const mxs_mat_s *A);
bool impl_ok(const mxs_mat_s *A, int32_t impl);
void set_impl(mxs_mat_s *A, int32_t impl); // impl_ok(A, impl) holds
mxs_status tune(mxs_mat_s *A, const void *x, void *y, int32_t reps, int32_t *impl_out,
                double *ms, hipStream_t s); // syncs
// spmv.hip: y += A x for a COO or CSR handle (the remainder of a split).
mxs_status spmv_acc_launch(const mxs_mat_s *A, const void *x, void *y, const int *done,
                           hipStream_t s, void *carry = nullptr);

// split.hip
mxs_status split_size(const mxs_mat_s *A, double min_fill, int32_t *band_ndiag, int64_t *rest_nnz,
                      hipStream_t s); // syncs
mxs_status split(const mxs_mat_s *A, double min_fill, mxs_format rest_fmt, int32_t *band_doff,
                 void *band_vals, int32_t *rest_idx0, int32_t *rest_idx1, void *rest_vals,
                 mxs_mat_s **out, hipStream_t s); // syncs

// scan.hip
// out[i] = sum_{k<i} in[k] for i in [0, n]; out has n+1 entries (the total
// last).  Fails with MXS_ERR_INDEX_RANGE if the total exceeds INT32_MAX.
mxs_status scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
// The same with its temporaries in the caller's ws[scan_ws_bytes(n)] (syncs).
size_t scan_ws_bytes(int64_t n);
mxs_status scan_i32_ws(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s);
mxs_status fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
mxs_status fill_bytes0(void *p, size_t bytes, hipStream_t s);

// convert.hip
mxs_status check_coo(const mxs_mat_s *A, hipStream_t s);  // syncs
mxs_status check_csr(const mxs_mat_s *A, hipStream_t s);  // syncs
mxs_status check_dia(const mxs_mat_s *A, hipStream_t s);  // syncs
mxs_status sort_coo(int32_t nrows, int32_t ncols, int64_t nnz, int32_t *ai, int32_t *aj,
                    void *av, mxs_dtype t, hipStream_t s);
mxs_status dia_slot_count(const mxs_mat_s *A, int64_t *slots, hipStream_t s); // syncs
mxs_status convert_size(const mxs_mat_s *A, mxs_format dst, int64_t *count, int32_t *ndiag,
                        hipStream_t s);
mxs_status convert(const mxs_mat_s *A, mxs_format dst, int32_t *idx0, int32_t *idx1,
                   void *vals, int64_t count, int32_t ndiag, hipStream_t s);
mxs_status cast_values(const void *src, mxs_dtype from, void *dst, mxs_dtype to, int64_t n,
                       hipStream_t s);
mxs_status csr_row_index(const int32_t *irp, int32_t nrows, int64_t nnz, int32_t *ai,
                         hipStream_t s);
// irp[nrows+1] of sorted row ids ai[nnz]
mxs_status coo_irp_launch(int64_t nnz, int32_t nrows, const int32_t *ai, int32_t *irp,
                          hipStream_t s);

// cg.hip
mxs_status dot_launch(int64_t n, mxs_dtype t, const void *a, const void *b, double *result,
                      hipStream_t s);
mxs_status dot_noalloc_launch(int64_t n, mxs_dtype t, const void *a, const void *b, double *result,
                              hipStream_t s);
mxs_status axpby_launch(int64_t n, mxs_dtype t, double alpha, const void *x, double beta,
                        void *y, hipStream_t s);
size_t cg_workspace_bytes(int64_t n, int32_t mixed, int64_t parts64, int64_t parts32);
mxs_status cg_solve(const mxs_mat_s *A, const mxs_mat_s *A32, const double *b, double *x,
                    const mxs_cg_opts *o, mxs_cg_result *r, void *ws, size_t bytes,
                    hipStream_t s);

// features.hip
mxs_status features(const mxs_mat_s *A, double out[8], hipStream_t s);

// ell.hip: ELL and SELL-C-sigma (C = 64).
mxs_status ell_width(const mxs_mat_s *A, int32_t *K, hipStream_t s); // syncs; refuses > 8 slots/entry
mxs_status ell_build(const mxs_mat_s *A, int32_t K, int32_t *col, void *vals, hipStream_t s);
mxs_status sell_size(const mxs_mat_s *A, int32_t sigma, int64_t *slots, hipStream_t s); // syncs
// HYB: *K < 0 on entry asks for the width rule; *rest = entries past the K-th
mxs_status hyb_size(const mxs_mat_s *A, int32_t *K, int64_t *rest, hipStream_t s); // syncs
mxs_status hyb_build(const mxs_mat_s *A, int32_t K, int32_t *ell_col, void *ell_val, int32_t *ri,
                     int32_t *rj, void *rv, hipStream_t s);
mxs_status sell_build(const mxs_mat_s *A, int32_t sigma, int32_t *perm, int64_t *cs, int32_t *col,
                      void *vals, hipStream_t s);
// ELL/SELL -> COO (idx0 = row ids) or CSR (idx0 = row pointers)
mxs_status padded_to_rows(const mxs_mat_s *A, mxs_format dst, int32_t *idx0, int32_t *idx1,
                          void *vals, hipStream_t s);
mxs_status padded_spmv(const mxs_mat_s *A, const void *x, void *y, const int *done, double *parts,
                       hipStream_t s);
int64_t padded_grid(const mxs_mat_s *A, bool dot);
// ELL kernel on raw arrays (the CSR plan's ELL copy)
mxs_status ell_launch(int32_t nrows, int32_t K, const int32_t *col, const void *vals, mxs_dtype t,
                      const void *x, void *y, const int *done, double *parts, hipStream_t s);
int64_t ell_grid(int32_t nrows, bool dot);

// Frees a handle, its parts and the device memory it owns (api.hip).
void release(mxs_mat_s *A);
// colblk.hip: COO and CSR column blocks (laid out by the plan when they apply);
// irp: A's row pointers (CSR: its own; COO: a build-pass temporary, else nullptr).
mxs_status colblk_plan(mxs_mat_s *A, const int32_t *irp, PlanCtx &c, hipStream_t s);

// ell.hip: longest row of row pointers irp into *K, with `counter` one device int.
mxs_status longest_row_with(int32_t nrows, const int32_t *irp, int *counter, int32_t *K,
                            hipStream_t s); // syncs

// mg.hip: HPCG's multigrid preconditioner.
size_t mg_bytes(int32_t n, int32_t levels); // workspace of the hierarchy (0: unsupported)
mxs_status mg_create(int32_t n, int32_t levels, void *ws, size_t bytes, mxs_mg_s **out,
                     hipStream_t s); // syncs
void mg_release(mxs_mg_s *M);
mxs_status symgs_launch(const mxs_mg_s *M, int32_t level, const double *r, double *x,
                        hipStream_t s);
// z = V-cycle(r) on the finest level; kernels return at entry when *done.
mxs_status mg_apply(const mxs_mg_s *M, const double *r, double *z, const int *done, hipStream_t s);
size_t pcg_workspace_bytes(int64_t n);
mxs_status pcg_solve(const mxs_mg_s *M, const mxs_mat_s *A, const double *b, double *x,
                     const mxs_cg_opts *o, mxs_cg_result *r, void *ws, size_t bytes,
                     hipStream_t s);

// gen.hip
mxs_status stencil_coo(int32_t n, int32_t points, double diag, double offdiag, int32_t *ai,
                       int32_t *aj, void *av, mxs_dtype t, hipStream_t s);
// The same with its temporaries in ws[stencil_ws_bytes(n)].
size_t stencil_ws_bytes(int32_t n);
mxs_status stencil_coo_ws(int32_t n, int32_t points, double diag, double offdiag, int32_t *ai,
                          int32_t *aj, void *av, mxs_dtype t, void *ws, hipStream_t s);

// mlp.hip
mxs_status mlp_inputs(const double *raw, int32_t n, const float *mu, const float *sd,
                      float *X, hipStream_t s);
mxs_status mlp_norm_stats(const double *raw, int32_t n, float *mu, float *sd, hipStream_t s);
mxs_status mlp_forward(const float *w, const float *X, int32_t n, float *logits, hipStream_t s);
mxs_status mlp_predict(const float *w, const float *X, int32_t n, const uint8_t *feasible,
                       int32_t *fmt, hipStream_t s);
size_t mlp_ws_bytes(int32_t n);
mxs_status mlp_grad(const float *w, const float *X, const int32_t *labels, int32_t n,
                    float *grad, float *loss, void *ws, hipStream_t s);
mxs_status mlp_adam(float *w, float *m, float *v, const float *g, float lr, int32_t t,
                    float b1, float b2, float eps, hipStream_t s);

}  // namespace mxs
