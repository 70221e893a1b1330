// HPCG's preconditioner (Section VII-D): a multigrid V-cycle on the
// 27-point stencil whose smoother is symmetric Gauss-Seidel.
//
// Gauss-Seidel is sequential in its row order; on the GPU the rows are
// ordered by colour instead: the 8 colours of the grid points' coordinate
// parities, c = (ix & 1) + 2 (iy & 1) + 4 (iz & 1).  No 27-point coupling
// joins two points of one colour, so all rows of a colour update at once,
// one launch per colour, and the sweep equals the sequential one in that
// order.  Colour 0 (the points the next coarser grid keeps) is swept last,
// so the forward sweep after prolongation reads the coarse correction before
// it recomputes those points.
//
// Storage of a level for the smoother: rows in colour order (colour-id
// order, ascending row id inside a colour), grouped 64 to a slice (one
// wavefront, a lane per row); a slice holds its rows' off-diagonal entries
// column-major, k-th entry of lane l at k*64 + l, padded to the slice's
// longest row with zero values, so each load of a slice is one contiguous
// 256-byte (columns) or 512-byte (values) access.  The diagonal is kept
// apart: a row's update is x_i = (r_i - sum_{j != i} a_ij x_j) / a_ii.
//
// Restriction is fused: the coarse right-hand side r_c = (r - A z) at the
// colour-0 rows is computed from the colour-0 slices and their diagonals,
// the only rows of A z it needs (1/8 of an SpMV).  Colour-0 rows in colour
// order are exactly the coarse rows in their natural order.
#include "common.h"

#include <algorithm>
#include <cstdio>

namespace mxs {

constexpr int kSlice = 64;
constexpr int kColours = 8;
constexpr int kMgNT = 256;
// Colour passes of a large level (at least kBigRows rows) are bandwidth
// bound: 256-thread workgroups, 16 entries a step, slice entries streamed
// with non-temporal loads.  Those of a smaller level are latency bound and
// its slices stay in cache between passes: 64-thread workgroups (more CUs
// for a few rows), 32 entries a step, cached loads.
constexpr int32_t kBigRows = 1 << 20;

template <bool STREAM, typename T>
__device__ __forceinline__ T ld_slice(const T *p)
{
    if constexpr (STREAM) return __builtin_nontemporal_load(p);
    else return *p;
}
// Workgroup index of the cycle's kernels: with a grid of a multiple of 8
// workgroups, XCD j (workgroups j, j + 8, ...) takes the j-th eighth of the
// rows in colour order, that is the same z-slab of the grid in every
// colour's pass, so the neighbour values a pass reads were mostly written by
// the previous pass through the same L2.
__device__ __forceinline__ int32_t mg_block()
{
    return gridDim.x % kNumXcd ? (int32_t)blockIdx.x : (int32_t)xcd_remap(blockIdx.x, gridDim.x);
}

// The cycle's kernels read their convergence flag from here when they are
// given none, so that the flag's load needs no test of the pointer first and
// goes out with the kernel's other first loads.
__device__ const int kNoFlag = 0;
__device__ __forceinline__ int flag_of(const int *done) { return *(done ? done : &kNoFlag); }

// sweep order of the colours: coarse points (colour 0) last
constexpr int kSweep[kColours] = {1, 2, 3, 4, 5, 6, 7, 0};

__device__ __forceinline__ int grid_colour(int64_t i, int32_t n)
{
    const int64_t ix = i % n, iy = (i / n) % n, iz = i / ((int64_t)n * n);
    return (int)((ix & 1) + 2 * (iy & 1) + 4 * (iz & 1));
}

// position of each row: order[pos[i]] = i (closed form: colour c holds the
// points with those parities, ordered by (iz, iy, ix)).
struct ColourGeom {
    int32_t n;
    int32_t coff[kColours + 1];
};

__global__ void mg_order_kernel(ColourGeom g, int32_t *__restrict__ order)
{
    const int64_t rows = (int64_t)g.n * g.n * g.n;
    const int32_t h[2] = {(g.n + 1) / 2, g.n / 2}; // points of parity 0 / 1 along an axis
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = i % g.n, iy = (i / g.n) % g.n, iz = i / ((int64_t)g.n * g.n);
        const int px = (int)(ix & 1), py = (int)(iy & 1), pz = (int)(iz & 1);
        const int c = px + 2 * py + 4 * pz;
        const int64_t rank = (iz >> 1) * (int64_t)h[py] * h[px] + (iy >> 1) * (int64_t)h[px] + (ix >> 1);
        order[g.coff[c] + rank] = (int32_t)i;
    }
}

// Off-diagonal count of each slice's longest row.
__global__ void mg_width_kernel(ColourGeom g, const int32_t *__restrict__ slice_colour_first,
                                const int32_t *__restrict__ order, const int32_t *__restrict__ irp,
                                int32_t nslices, int32_t *__restrict__ width)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    // colour of slice s: the last c with slice_colour_first[c] <= s
    int c = 0;
    for (int k = 1; k < kColours; ++k) c = s >= slice_colour_first[k] ? k : c;
    const int32_t p0 = g.coff[c] + (s - slice_colour_first[c]) * kSlice;
    const int32_t p1 = min(p0 + kSlice, g.coff[c + 1]);
    int32_t w = 0;
    for (int32_t p = p0; p < p1; ++p) {
        const int32_t i = order[p];
        w = max(w, irp[i + 1] - irp[i] - 1);
    }
    width[s] = max(w, 0);
}

__global__ void mg_slice_offsets_kernel(const int32_t *__restrict__ wscan, int32_t nslices,
                                        int64_t *__restrict__ soff)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s <= nslices) soff[s] = (int64_t)kSlice * wscan[s];
}

// Scatters row order[p]'s entries into its slice; flags a row without a
// nonzero diagonal (bit 0) or with a neighbour of its own colour (bit 1).
__global__ void mg_fill_kernel(ColourGeom g, const int32_t *__restrict__ slice_colour_first,
                               const int32_t *__restrict__ order, const int32_t *__restrict__ irp,
                               const int32_t *__restrict__ aj, const double *__restrict__ av,
                               const int64_t *__restrict__ soff, int32_t *__restrict__ col,
                               double *__restrict__ val, double *__restrict__ diag,
                               int *__restrict__ flags)
{
    const int64_t rows = (int64_t)g.n * g.n * g.n;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= rows) return;
    int c = 0;
    for (int k = 1; k < kColours; ++k) c = p >= g.coff[k] ? k : c;
    const int32_t local = (int32_t)p - g.coff[c];
    const int32_t s = slice_colour_first[c] + local / kSlice;
    const int lane = local % kSlice;
    const int64_t base = soff[s];
    const int32_t w = (int32_t)((soff[s + 1] - base) / kSlice);
    const int32_t i = order[p];
    double d = 0.0;
    int32_t k = 0;
    int bad = 0;
    for (int32_t e = irp[i]; e < irp[i + 1]; ++e) {
        const int32_t j = aj[e];
        if (j == i) {
            d = av[e];
        } else if (k < w) {
            if (grid_colour(j, g.n) == c) bad |= 2;
            col[base + (int64_t)k * kSlice + lane] = j;
            val[base + (int64_t)k * kSlice + lane] = av[e];
            ++k;
        }
    }
    for (; k < w; ++k) {
        col[base + (int64_t)k * kSlice + lane] = i;
        val[base + (int64_t)k * kSlice + lane] = 0.0;
    }
    diag[p] = d;
    if (d == 0.0) bad |= 1;
    if (bad) atomicOr(flags, bad);
}

// One colour of a Gauss-Seidel sweep: every row of the colour at once.
template <int U, bool STREAM>
__global__ __launch_bounds__(kMgNT) void symgs_colour_kernel(
    const int32_t *__restrict__ order, const int64_t *__restrict__ soff,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ diag, const double *__restrict__ r, double *__restrict__ x,
    int32_t p0, int32_t nrows_c, int32_t s0, const int *__restrict__ done)
{
    const int stop = flag_of(done);
    const int32_t t = mg_block() * blockDim.x + threadIdx.x;
    if (t >= nrows_c) return;
    const int32_t s = s0 + t / kSlice;
    const int lane = t % kSlice;
    const int32_t i = order[p0 + t];
    const int64_t base = soff[s];
    const int32_t w = (int32_t)((soff[s + 1] - base) / kSlice);
    const double dg = diag[p0 + t];
    // The convergence flag is tested with the loads above in flight (i and w
    // are never negative: testing them keeps those loads ahead of the
    // branch), so the flag costs the pass no round trip of its own.
    if (stop | (i < 0) | (w < 0)) return;
    double sum = r[i];
    {
        const int32_t *__restrict__ cs = col + base + lane;
        const double *__restrict__ vs = val + base + lane;
        // U entries per step, all loads of a step issued together; entries
        // past the slice width are skipped (column i, value 0: no load)
        for (int32_t k = 0; k < w; k += U) {
            int32_t cu[U];
            double vu[U], xu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = k + u < w;
                cu[u] = in ? ld_slice<STREAM>(&cs[(k + u) * kSlice]) : i;
                vu[u] = in ? ld_slice<STREAM>(&vs[(k + u) * kSlice]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xu[u] = x[cu[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) sum -= vu[u] * xu[u];
        }
    }
    x[i] = sum / dg;
}

// The first colour pass of a sweep from z = 0 with the zeroing folded in:
// rows of the first colour (positions [q0, q1)) get r_i / a_ii (their
// neighbours are all zero), every other row gets 0.
__global__ __launch_bounds__(kMgNT) void mg_start_kernel(const int32_t *__restrict__ order,
                                                         const double *__restrict__ diag,
                                                         const double *__restrict__ r,
                                                         double *__restrict__ z, int32_t rows,
                                                         int32_t q0, int32_t q1,
                                                         const int *__restrict__ done)
{
    const int stop = flag_of(done);
    for (int32_t p = mg_block() * blockDim.x + threadIdx.x; p < rows; p += gridDim.x * blockDim.x) {
        const int32_t i = order[p];
        const bool first = p >= q0 && p < q1;
        const double dg = first ? diag[p] : 1.0;
        // the flag with the row's loads in flight (i is never negative)
        if (stop | (i < 0)) return;
        z[i] = first ? r[i] / dg : 0.0;
    }
}

// r_c[ic] = r[i] - (A z)[i] for the colour-0 row i = order[ic].
__global__ __launch_bounds__(kMgNT) void mg_restrict_kernel(
    const int32_t *__restrict__ order, const int64_t *__restrict__ soff,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ diag, const double *__restrict__ r, const double *__restrict__ z,
    int32_t nc, double *__restrict__ rc, const int *__restrict__ done)
{
    const int stop = flag_of(done);
    const int32_t t = mg_block() * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    const int32_t s = t / kSlice;
    const int lane = t % kSlice;
    const int32_t i = order[t];
    const int64_t base = soff[s];
    const int32_t w = (int32_t)((soff[s + 1] - base) / kSlice);
    const double dg = diag[t];
    // the flag with the loads above in flight (i and w are never negative)
    if (stop | (i < 0) | (w < 0)) return;
    double az = dg * z[i];
    for (int32_t k = 0; k < w; ++k)
        az += val[base + (int64_t)k * kSlice + lane] * z[col[base + (int64_t)k * kSlice + lane]];
    rc[t] = r[i] - az;
}

// z[order[ic]] += zc[ic]
__global__ void mg_prolong_kernel(const int32_t *__restrict__ order, const double *__restrict__ zc,
                                  int32_t nc, double *__restrict__ z, const int *__restrict__ done)
{
    const int stop = flag_of(done);
    const int32_t t = mg_block() * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    const int32_t i = order[t];
    const double c = zc[t];
    // the flag with the loads above in flight (i is never negative)
    if (stop | (i < 0)) return;
    z[i] += c;
}

static uint32_t blocks(int64_t n, int nt = kMgNT) { return (uint32_t)std::max<int64_t>(1, (n + nt - 1) / nt); }
// grid of the cycle's kernels: a multiple of 8 workgroups (see mg_block)
static uint32_t xblocks(int64_t n, int nt) { return pad_grid(blocks(n, nt)); }

// ---------------------------------------------------------------------------
// Hierarchy: every array lives in the caller's workspace, laid out by a
// sizing pass (closed forms, no device work) and then built by the same code
// (see PlanCtx).
// ---------------------------------------------------------------------------
// Neighbours along one axis of coordinate t on an n-point edge, t included.
static int along(int32_t t, int32_t n) { return 1 + (t > 0 ? 1 : 0) + (t < n - 1 ? 1 : 0); }

// Sum over the slices of a level of their widths (the longest row's
// off-diagonal count, from the stencil's row lengths), in colour order.
static int64_t slice_total(int32_t n)
{
    int64_t total = 0;
    for (int c = 0; c < kColours; ++c) {
        const int px = c & 1, py = (c >> 1) & 1, pz = (c >> 2) & 1;
        int k = 0, w = 0;
        for (int32_t z = pz; z < n; z += 2)
            for (int32_t y = py; y < n; y += 2)
                for (int32_t x = px; x < n; x += 2) {
                    w = std::max(w, along(x, n) * along(y, n) * along(z, n) - 1);
                    if (++k == kSlice) {
                        total += w;
                        k = 0;
                        w = 0;
                    }
                }
        if (k > 0) total += w;
    }
    return total;
}

static mxs_status build_level(mxs_mg_s *M, MgLevel &L, int32_t n, bool vectors, PlanCtx &c,
                              hipStream_t s)
{
    L = MgLevel{};
    L.n = n;
    const int64_t rows64 = (int64_t)n * n * n;
    const int64_t nnz = (3 * (int64_t)n - 2) * (3 * (int64_t)n - 2) * (3 * (int64_t)n - 2);
    if (rows64 > INT32_MAX || nnz > INT32_MAX) return MXS_ERR_UNSUPPORTED;
    L.rows = (int32_t)rows64;
    // colour order (closed form) and slices
    ColourGeom g{};
    g.n = n;
    const int32_t h[2] = {(n + 1) / 2, n / 2};
    g.coff[0] = 0;
    for (int c2 = 0; c2 < kColours; ++c2)
        g.coff[c2 + 1] = g.coff[c2] + h[c2 & 1] * h[(c2 >> 1) & 1] * h[(c2 >> 2) & 1];
    std::copy(g.coff, g.coff + kColours + 1, L.coff);
    int32_t nsl = 0;
    for (int c2 = 0; c2 < kColours; ++c2) {
        L.sfirst[c2] = nsl;
        nsl += (L.coff[c2 + 1] - L.coff[c2] + kSlice - 1) / kSlice;
    }
    L.sfirst[kColours] = nsl;
    L.nslices = nsl;
    const int64_t total = slice_total(n);
    const size_t entries = (size_t)kSlice * (size_t)total;

    // kept: the operator in CSR, the colour order, the slices, the diagonal,
    // and on coarse levels their right-hand side and correction
    auto *irp = (int32_t *)c.keep(sizeof(int32_t) * ((size_t)L.rows + 1));
    auto *aj = (int32_t *)c.keep(sizeof(int32_t) * (size_t)nnz);
    auto *av = (double *)c.keep(sizeof(double) * (size_t)nnz);
    L.order = (int32_t *)c.keep(sizeof(int32_t) * (size_t)L.rows);
    L.soff = (int64_t *)c.keep(sizeof(int64_t) * ((size_t)nsl + 1));
    L.col = (int32_t *)c.keep(sizeof(int32_t) * entries);
    L.val = (double *)c.keep(sizeof(double) * entries);
    L.diag = (double *)c.keep(sizeof(double) * (size_t)L.rows);
    if (vectors) {
        L.r = (double *)c.keep(sizeof(double) * (size_t)L.rows);
        L.z = (double *)c.keep(sizeof(double) * (size_t)L.rows);
    }
    // temporaries: row ids, the generator's, slice widths and their scan, a
    // flag.  The next level's are taken only after this level's build has
    // synchronised, so the region is handed back at once.
    const size_t mark = c.mark();
    auto *ai = (int32_t *)c.tmp(sizeof(int32_t) * (size_t)nnz);
    void *gws = c.tmp(stencil_ws_bytes(n));
    auto *dev_sfirst = (int32_t *)c.tmp(sizeof(int32_t) * (kColours + 1));
    auto *width = (int32_t *)c.tmp(sizeof(int32_t) * ((size_t)nsl + 1));
    auto *wscan = (int32_t *)c.tmp(sizeof(int32_t) * ((size_t)nsl + 1));
    auto *flags = (int *)c.tmp(sizeof(int));
    void *sws = c.tmp(scan_ws_bytes(nsl));
    c.release(mark);
    if (!c.build) return MXS_OK;

    // the operator: 27-point stencil, 26 on the diagonal and -1 off it, in CSR
    mxs_status st = stencil_coo_ws(n, 27, 26.0, -1.0, ai, aj, av, MXS_F64, gws, s);
    if (st == MXS_OK) st = coo_irp_launch(nnz, L.rows, ai, irp, s);
    if (st != MXS_OK) return st;
    auto *A = new mxs_mat_s;
    A->fmt = MXS_CSR;
    A->dtype = MXS_F64;
    A->nrows = A->ncols = L.rows;
    A->nnz = nnz;
    A->idx0 = irp;
    A->idx1 = aj;
    A->vals = av;
    A->device = M->device;
    A->part = true;
    L.A = A;

    mg_order_kernel<<<std::min<uint32_t>(blocks(L.rows), 65536), kMgNT, 0, s>>>(g, L.order);
    if ((st = launch_status()) != MXS_OK) return st;
    MXS_HIP(hipMemcpyAsync(dev_sfirst, L.sfirst, sizeof(int32_t) * (kColours + 1),
                           hipMemcpyHostToDevice, s));
    mg_width_kernel<<<blocks(nsl), kMgNT, 0, s>>>(g, dev_sfirst, L.order, irp, nsl, width);
    st = launch_status();
    if (st == MXS_OK) st = scan_i32_ws(width, wscan, nsl, sws, s);
    if (st == MXS_OK) {
        mg_slice_offsets_kernel<<<blocks(nsl + 1), kMgNT, 0, s>>>(wscan, nsl, L.soff);
        st = launch_status();
    }
    int32_t dev_total = 0;
    if (st == MXS_OK && hipMemcpyAsync(&dev_total, wscan + nsl, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = MXS_ERR_HIP;
    if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;
    if (dev_total != total) { // the slices' size was laid out from the closed form
        snprintf(g_last_error, sizeof g_last_error,
                 "multigrid level %d: slice widths sum to %d on the device, %lld laid out", n,
                 dev_total, (long long)total);
        return MXS_ERR_HIP;
    }
    // lanes past a colour's last row are never read; zero them anyway
    st = fill_bytes0(L.col, sizeof(int32_t) * entries, s);
    if (st == MXS_OK) st = fill_bytes0(L.val, sizeof(double) * entries, s);
    if (st == MXS_OK) st = fill_bytes0(flags, sizeof(int), s);
    if (st == MXS_OK) {
        mg_fill_kernel<<<blocks(L.rows), kMgNT, 0, s>>>(g, dev_sfirst, L.order, irp, aj, av, L.soff,
                                                        L.col, L.val, L.diag, flags);
        st = launch_status();
    }
    int hf = 0;
    if (st == MXS_OK && hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = MXS_ERR_HIP;
    if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;
    if (hf) return MXS_ERR_INVALID_ARG; // no such row in the stencil: a build fault
    return MXS_OK;
}

void mg_release(mxs_mg_s *M)
{
    if (!M) return;
    // the level operators' arrays are in the caller's workspace; plans built
    // on them are the caller's too
    for (auto &L : M->lv) release(L.A);
    delete M;
}

static mxs_status mg_walk(mxs_mg_s *M, int32_t n, int32_t levels, PlanCtx &c, hipStream_t s)
{
    M->lv.resize((size_t)levels);
    for (int32_t l = 0; l < levels; ++l) {
        const mxs_status st = build_level(M, M->lv[(size_t)l], n >> l, l > 0, c, s);
        if (st != MXS_OK) return st;
    }
    return MXS_OK;
}

size_t mg_bytes(int32_t n, int32_t levels)
{
    mxs_mg_s M;
    PlanCtx c;
    if (mg_walk(&M, n, levels, c, nullptr) != MXS_OK) return 0;
    return c.total();
}

mxs_status mg_create(int32_t n, int32_t levels, void *ws, size_t bytes, mxs_mg_s **out, hipStream_t s)
{
    PlanCtx z;
    {
        mxs_mg_s sizing;
        const mxs_status st = mg_walk(&sizing, n, levels, z, s);
        if (st != MXS_OK) return st;
    }
    if (bytes < z.total()) return MXS_ERR_INVALID_ARG;
    auto *M = new mxs_mg_s;
    (void)hipGetDevice(&M->device);
    PlanCtx c;
    c.build = true;
    c.keep_base = (char *)ws;
    c.tmp_base = (char *)ws + PlanCtx::up(z.keep_used);
    mxs_status st = mg_walk(M, n, levels, c, s);
    if (st != MXS_OK) {
        (void)hipStreamSynchronize(s);
        mg_release(M);
        return st;
    }
    *out = M;
    return MXS_OK;
}

// ---------------------------------------------------------------------------
// Sweeps and the cycle
// ---------------------------------------------------------------------------
static void colour_pass(const MgLevel &L, int c, const double *r, double *x,
                        const int *done, hipStream_t s)
{
    const int32_t p0 = L.coff[c], nr = L.coff[c + 1] - L.coff[c];
    if (nr == 0) return;
    const bool big = L.rows >= kBigRows;
    const int nt = big ? 256 : 64;
    auto kern = big ? symgs_colour_kernel<16, true> : symgs_colour_kernel<32, false>;
    kern<<<xblocks(nr, nt), nt, 0, s>>>(L.order, L.soff, L.col, L.val, L.diag, r, x, p0, nr,
                                       L.sfirst[c], done);
}

// Forward over kSweep, backward over its reverse.  The backward sweep's
// first colour would recompute the forward sweep's last one from the same
// neighbour values (no colour reads itself): the same numbers, so it is
// not launched.  zero_start: x is set to zero first (folded into the first
// colour's pass, whose rows then read only zeros).
static mxs_status symgs_level(const MgLevel &L, const double *r, double *x, bool zero_start,
                              const int *done, hipStream_t s)
{
    if (zero_start) {
        const int c = kSweep[0];
        mg_start_kernel<<<std::min<uint32_t>(xblocks(L.rows, 256), 8192), 256, 0, s>>>(
            L.order, L.diag, r, x, L.rows, L.coff[c], L.coff[c + 1], done);
    }
    for (int k = zero_start ? 1 : 0; k < kColours; ++k) colour_pass(L, kSweep[k], r, x, done, s);
    for (int k = kColours - 2; k >= 0; --k) colour_pass(L, kSweep[k], r, x, done, s);
    return launch_status();
}

mxs_status symgs_launch(const mxs_mg_s *M, int32_t level, const double *r, double *x,
                        hipStream_t s)
{
    return symgs_level(M->lv[(size_t)level], r, x, false, nullptr, s);
}

static mxs_status vcycle(const mxs_mg_s *M, size_t l, const double *r, double *z, const int *done,
                         hipStream_t s)
{
    const MgLevel &L = M->lv[l];
    mxs_status st = symgs_level(L, r, z, true, done, s);
    if (st != MXS_OK || l + 1 == M->lv.size()) return st;
    const MgLevel &C = M->lv[l + 1];
    const int32_t nc = L.coff[1]; // colour-0 rows = coarse rows
    const int nt = L.rows >= kBigRows ? 256 : 64;
    mg_restrict_kernel<<<xblocks(nc, nt), nt, 0, s>>>(L.order, L.soff, L.col, L.val, L.diag, r, z, nc,
                                                     C.r, done);
    if ((st = launch_status()) != MXS_OK) return st;
    if ((st = vcycle(M, l + 1, C.r, C.z, done, s)) != MXS_OK) return st;
    mg_prolong_kernel<<<xblocks(nc, nt), nt, 0, s>>>(L.order, C.z, nc, z, done);
    if ((st = launch_status()) != MXS_OK) return st;
    return symgs_level(L, r, z, false, done, s);
}

mxs_status mg_apply(const mxs_mg_s *M, const double *r, double *z, const int *done, hipStream_t s)
{
    return vcycle(M, 0, r, z, done, s);
}

}  // namespace mxs
