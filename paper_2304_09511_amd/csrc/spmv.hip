// SpMV kernels for gfx950: y = A*x in CSR, DIA and COO (Algorithms 2, 3, 1
// of Section III-B), plus the analysis that builds each format's plan.
//
// All three are HBM-bound streams (0.12-0.23 flop/byte in FP64), so the
// design goals are wide coalesced loads of the matrix arrays, x gathers that
// hit in L2, deterministic reductions without floating-point atomics, and
// enough bytes in flight per CU.  No MFMA: SpMV is not a dense contraction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace mxs {

// ===========================================================================
// CSR (Algorithm 2): row blocks of bounded non-zero count, products staged in
// LDS, rows reduced by lane groups sized to the block's row count.
// ===========================================================================
template <typename T>
struct CsrCfg;
template <>
struct CsrCfg<double> {
    static constexpr int NT = 256;     // threads per workgroup
    static constexpr int BUCKET = 1024; // target non-zeros per row block
    static constexpr int TMAX = 2048;  // LDS capacity (a block holds < 2*BUCKET)
    static constexpr int RMAX = 256;   // rows per block at most
};
template <>
struct CsrCfg<float> {
    static constexpr int NT = 256;
    static constexpr int BUCKET = 2048;
    static constexpr int TMAX = 4096;
    static constexpr int RMAX = 256;
};

// Row-block boundaries.  Row r starts a block when its first entry falls in
// another BUCKET-sized slice of the entry range than row r-1's, when either
// row is longer than BUCKET, or every RMAX rows.  Rows of one block then
// start within one slice and none is long, so a block holds fewer than
// 2*BUCKET entries; a long row is a block of its own.
template <int BUCKET, int RMAX>
__global__ void csr_block_flags(const int32_t *__restrict__ irp, int32_t nrows,
                                int32_t *__restrict__ flag)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    int f = 1;
    if (r > 0) {
        const int32_t a = irp[r - 1], b = irp[r], c = irp[r + 1];
        f = (a / BUCKET != b / BUCKET) || (b - a > BUCKET) || (c - b > BUCKET) ||
            (r % RMAX == 0);
    }
    flag[r] = f;
}

__global__ void csr_block_scatter(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                                  int32_t nrows, int32_t *__restrict__ blk_row)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrows && flag[r]) blk_row[pos[r]] = (int32_t)r;
    if (r == 0) blk_row[pos[nrows]] = nrows;
}

template <typename T, bool DOT>
__global__ __launch_bounds__(256) void csr_spmv_kernel(
    const int32_t *__restrict__ irp, const int32_t *__restrict__ aj, const T *__restrict__ av,
    const T *__restrict__ x, T *__restrict__ y, const int32_t *__restrict__ blk_row,
    int64_t nblk, int64_t per, const int *__restrict__ done, DotSink dot)
{
    using C = CsrCfg<T>;
    constexpr int NT = C::NT;
    constexpr int U = C::TMAX / NT; // entries per thread when a block is full
    __shared__ T prod[C::TMAX];
    __shared__ int32_t lrp[C::RMAX + 1];
    __shared__ double red[NT / kWave];
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b_lo = g * per, b_hi = min(nblk, b_lo + per);
    double dpart = 0.0;
    for (int64_t b = b_lo; b < b_hi; ++b) {
        const int32_t r0 = blk_row[b], r1 = blk_row[b + 1];
        const int32_t nr = r1 - r0;
        const int32_t k0 = irp[r0], k1 = irp[r1];
        const int32_t nk = k1 - k0;
        if (nk > C::TMAX) {
            // One long row: the whole workgroup strides over it.
            T s = T(0);
            for (int32_t k = k0 + tid; k < k1; k += NT) s += av[k] * x[aj[k]];
            const double tot = block_sum<NT>((double)s, red);
            if (tid == 0) {
                const T v = (T)tot;
                y[r0] = v;
                if (DOT) dpart += (double)v * (double)x[r0];
            }
            __syncthreads();
            continue;
        }
        for (int i = tid; i <= nr; i += NT) lrp[i] = irp[r0 + i] - k0;
        {
            int32_t col[U];
            T val[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = u * NT + tid;
                col[u] = k < nk ? aj[k0 + k] : 0;
                val[u] = k < nk ? av[k0 + k] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = u * NT + tid;
                if (k < nk) prod[k] = val[u] * x[col[u]];
            }
        }
        __syncthreads();
        // Lane-group size: the largest power of two G <= 64 with G*nr <= NT.
        int G = 64;
        while (G > 1 && G * nr > NT) G >>= 1;
        const int lane = tid & (G - 1);
        const int ngrp = NT / G;
        for (int r = tid / G; r < nr; r += ngrp) {
            T s = T(0);
            const int e = lrp[r + 1];
            for (int k = lrp[r] + lane; k < e; k += G) s += prod[k];
            for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
            if (lane == 0) {
                y[r0 + r] = s;
                if (DOT) dpart += (double)s * (double)x[r0 + r];
            }
        }
        __syncthreads();
    }
    if (DOT) {
        const double bs = block_sum<NT>(dpart, red);
        double tot;
        if (last_block_total<NT>(bs, blockIdx.x, gridDim.x, dot.partials, &dot.st->ticket, red,
                                 &tot) &&
            tid == 0)
            cg_finish_sigma(dot.st, tot);
    }
}

// ===========================================================================
// DIA (Algorithm 3): one thread per row, RPT rows per thread strided by the
// workgroup size, diagonal-major values so each diagonal is a coalesced
// stream; x[i+off] is a shifted coalesced load that mostly hits in L2.
// ===========================================================================
constexpr int kDiaNT = 256;
template <typename T>
struct DiaCfg;
template <>
struct DiaCfg<double> {
    static constexpr int RPT = 4;
};
template <>
struct DiaCfg<float> {
    static constexpr int RPT = 8;
};

template <typename T, bool DOT>
__global__ __launch_bounds__(256) void dia_spmv_kernel(
    int32_t nrows, int32_t ncols, int32_t ndiag, const int32_t *__restrict__ doff,
    const T *__restrict__ av, const T *__restrict__ x, T *__restrict__ y, int64_t nblk,
    int64_t per, const int *__restrict__ done, DotSink dot)
{
    constexpr int NT = kDiaNT;
    constexpr int RPT = DiaCfg<T>::RPT;
    constexpr int ROWS = NT * RPT;
    __shared__ double red[NT / kWave];
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b_lo = g * per, b_hi = min(nblk, b_lo + per);
    double dpart = 0.0;
    for (int64_t b = b_lo; b < b_hi; ++b) {
        const int64_t row0 = b * ROWS;
        const bool rows_full = row0 + ROWS <= nrows;
        T sum[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) sum[r] = T(0);
        for (int d = 0; d < ndiag; ++d) {
            const int64_t off = doff[d];
            const T *__restrict__ a = av + (int64_t)d * nrows;
            if (rows_full && row0 + off >= 0 && row0 + ROWS - 1 + off < ncols) {
                T va[RPT], vx[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int64_t i = row0 + r * NT + tid;
                    va[r] = a[i];
                    vx[r] = x[i + off];
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) sum[r] += va[r] * vx[r];
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int64_t i = row0 + r * NT + tid;
                    const int64_t k = i + off;
                    if (i < nrows && k >= 0 && k < ncols) sum[r] += a[i] * x[k];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int64_t i = row0 + r * NT + tid;
            if (i < nrows) {
                y[i] = sum[r];
                if (DOT) dpart += (double)sum[r] * (double)x[i];
            }
        }
    }
    if (DOT) {
        const double bs = block_sum<NT>(dpart, red);
        double tot;
        if (last_block_total<NT>(bs, blockIdx.x, gridDim.x, dot.partials, &dot.st->ticket, red,
                                 &tot) &&
            tid == 0)
            cg_finish_sigma(dot.st, tot);
    }
}

// ===========================================================================
// COO (Algorithm 1) on the canonical sorted order: tiles of TILE entries;
// each workgroup stages row ids and products in LDS, every thread reduces a
// run of IPT consecutive entries, and a workgroup-wide segmented scan
// carries partial sums across threads.  Rows spanning tiles leave their
// pieces in a carry array that a fix-up kernel adds in tile order, so the
// result is deterministic without atomics.  Rows with no entry are written
// as 0 by the tile that sees the gap, so y needs no separate clearing.
// ===========================================================================
constexpr int kCooNT = 256;
constexpr int kCooIPT = 8;
constexpr int kCooTile = kCooNT * kCooIPT;

__device__ __forceinline__ int coo_pad(int j) { return j + (j >> 3); }

template <typename T>
struct SegPair {
    int h; // a segment head lies in the run
    T v;   // sum since the last head (or since the start of the run)
};

template <typename T>
__device__ __forceinline__ SegPair<T> seg_combine(SegPair<T> a, SegPair<T> b)
{
    return {a.h | b.h, b.h ? b.v : a.v + b.v};
}

// Exclusive segmented scan over the workgroup in thread order.
template <typename T, int NT>
__device__ SegPair<T> block_seg_excl_scan(SegPair<T> x, int *sh, T *sv)
{
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    SegPair<T> inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int h = __shfl_up(inc.h, off, kWave);
        const T v = __shfl_up(inc.v, off, kWave);
        if (lane >= off) inc = seg_combine<T>({h, v}, inc);
    }
    if (lane == kWave - 1) {
        sh[w] = inc.h;
        sv[w] = inc.v;
    }
    __syncthreads();
    SegPair<T> pre = {0, T(0)};
    for (int i = 0; i < w; ++i) pre = seg_combine<T>(pre, {sh[i], sv[i]});
    int eh = __shfl_up(inc.h, 1, kWave);
    T ev = __shfl_up(inc.v, 1, kWave);
    if (lane == 0) {
        eh = 0;
        ev = T(0);
    }
    return seg_combine<T>(pre, {eh, ev});
}

template <typename T>
__global__ __launch_bounds__(256) void coo_spmv_kernel(
    int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai, const int32_t *__restrict__ aj,
    const T *__restrict__ av, const T *__restrict__ x, T *__restrict__ y, T *__restrict__ carry,
    int64_t ntiles, const int *__restrict__ done)
{
    constexpr int NT = kCooNT, IPT = kCooIPT, TILE = kCooTile;
    constexpr int PADDED = TILE + TILE / IPT;
    __shared__ int32_t srow[PADDED];
    __shared__ T sval[PADDED];
    __shared__ int sh[NT / kWave];
    __shared__ T sv[NT / kWave];
    if (done && *done) return;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int tid = threadIdx.x;
    const int64_t k0 = tile * TILE;
    const int n = (int)min((int64_t)TILE, nnz - k0);
    {
        int32_t row[IPT], col[IPT];
        T val[IPT];
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const int j = e * NT + tid;
            row[e] = j < n ? ai[k0 + j] : 0;
            col[e] = j < n ? aj[k0 + j] : 0;
            val[e] = j < n ? av[k0 + j] : T(0);
        }
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const int j = e * NT + tid;
            if (j < n) {
                srow[coo_pad(j)] = row[e];
                sval[coo_pad(j)] = val[e] * x[col[e]];
            }
        }
    }
    const int32_t prev_row = k0 > 0 ? ai[k0 - 1] : -1;
    const int32_t next_row = k0 + n < nnz ? ai[k0 + n] : -1;
    __syncthreads();
    const int32_t first_row = srow[0];
    const bool tile_cont = prev_row == first_row; // first segment began in an earlier tile
    const int b0 = tid * IPT, b1 = min(b0 + IPT, n);
    // pass 1: this thread's run as a (head seen, tail sum) pair
    SegPair<T> mine = {0, T(0)};
    for (int j = b0; j < b1; ++j) {
        const int32_t pr = j == 0 ? prev_row : srow[coo_pad(j - 1)];
        if (srow[coo_pad(j)] != pr) {
            mine.h = 1;
            mine.v = T(0);
        }
        mine.v += sval[coo_pad(j)];
    }
    const SegPair<T> cin = block_seg_excl_scan<T, NT>(mine, sh, sv);
    // pass 2: emit every segment that closes inside this run
    T s = cin.v;
    for (int j = b0; j < b1; ++j) {
        const int32_t row = srow[coo_pad(j)];
        const int32_t pr = j == 0 ? prev_row : srow[coo_pad(j - 1)];
        if (row != pr) {
            if (j > 0) {
                if (tile_cont && pr == first_row) carry[2 * tile] = s;
                else y[pr] = s;
            }
            for (int32_t z = pr + 1; z < row; ++z) y[z] = T(0); // rows without entries
            s = T(0);
        }
        s += sval[coo_pad(j)];
    }
    if (b0 < n && b1 == n) {
        // the thread holding the tile's last entry closes or hands over its segment
        const int32_t last = srow[coo_pad(n - 1)];
        const bool is_cont = tile_cont && last == first_row;
        if (next_row == last) {
            carry[2 * tile + (is_cont ? 0 : 1)] = s;
        } else {
            if (is_cont) carry[2 * tile] = s;
            else y[last] = s;
            if (k0 + n == nnz)
                for (int32_t z = last + 1; z < nrows; ++z) y[z] = T(0);
        }
    }
}

// Adds the pieces of rows that span tiles, in tile order.  The owner of such
// a row is the tile holding its first entry.
template <typename T>
__global__ void coo_fixup_kernel(int64_t nnz, const int32_t *__restrict__ ai,
                                 const T *__restrict__ carry, T *__restrict__ y, int64_t ntiles,
                                 const int *__restrict__ done)
{
    constexpr int TILE = kCooTile;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    if (done && *done) return;
    const int64_t k0 = t * TILE;
    const int64_t ke = min(nnz, k0 + TILE);
    const int32_t last = ai[ke - 1];
    if (ke >= nnz || ai[ke] != last) return; // last row closes in this tile
    const int32_t first = ai[k0];
    if (k0 > 0 && ai[k0 - 1] == first && first == last) return; // a middle piece
    T v = carry[2 * t + 1];
    for (int64_t u = t + 1; u < ntiles; ++u) {
        v += carry[2 * u];
        const int64_t ue = min(nnz, (u + 1) * TILE);
        if (ai[ue - 1] != last || ue >= nnz || ai[ue] != last) break;
    }
    y[last] = v;
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ p, T v, int64_t n, const int *__restrict__ done)
{
    if (done && *done) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Fused p.Ap for COO (the COO kernel has no per-row epilogue of its own).
template <typename T>
__global__ __launch_bounds__(256) void dot_sigma_kernel(int64_t n, const T *__restrict__ a,
                                                        const T *__restrict__ b,
                                                        const int *__restrict__ done, DotSink dot)
{
    constexpr int NT = 256;
    __shared__ double red[NT / kWave];
    if (done && *done) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        s += (double)a[i] * (double)b[i];
    const double bs = block_sum<NT>(s, red);
    double tot;
    if (last_block_total<NT>(bs, blockIdx.x, gridDim.x, dot.partials, &dot.st->ticket, red,
                             &tot) &&
        threadIdx.x == 0)
        cg_finish_sigma(dot.st, tot);
}

// ===========================================================================
// Launch configuration
// ===========================================================================
constexpr int64_t kDotGrid = 2048; // workgroups (= partials) of a fused dot

static int64_t dia_blocks(const mxs_mat_s *A)
{
    const int64_t rows = (int64_t)kDiaNT * (A->dtype == MXS_F64 ? DiaCfg<double>::RPT
                                                                 : DiaCfg<float>::RPT);
    return (A->nrows + rows - 1) / rows;
}

// Workgroup count and row blocks per workgroup for CSR/DIA.  Without a fused
// dot every row block gets its own workgroup; with one the grid is capped so
// the final reduction reads at most kDotGrid partials.
static void grid_for(int64_t nblk, bool dot, uint32_t *grid, int64_t *per)
{
    int64_t g = nblk;
    if (dot) g = std::min<int64_t>(nblk, kDotGrid);
    g = std::max<int64_t>(g, 1);
    *per = (nblk + g - 1) / g;
    g = (nblk + *per - 1) / *per;
    *grid = pad_grid(std::max<int64_t>(g, 1));
}

int64_t spmv_dot_parts(const mxs_mat_s *A)
{
    if (A->fmt == MXS_COO) return kDotGrid;
    const int64_t nblk = A->fmt == MXS_CSR ? A->csr.nblk : dia_blocks(A);
    uint32_t grid;
    int64_t per;
    grid_for(nblk, true, &grid, &per);
    return grid;
}

mxs_status build_plan(mxs_mat_s *A, hipStream_t s)
{
    if (A->optimized) return MXS_OK;
    if (A->fmt == MXS_CSR) {
        const int32_t n = A->nrows;
        const bool f64 = A->dtype == MXS_F64;
        int32_t *flag = nullptr, *pos = nullptr;
        MXS_HIP(hipMallocAsync((void **)&flag, sizeof(int32_t) * (size_t)std::max(n, 1), s));
        MXS_HIP(hipMallocAsync((void **)&pos, sizeof(int32_t) * ((size_t)n + 1), s));
        const int nb = (int)((n + 255) / 256);
        if (n > 0) {
            if (f64)
                csr_block_flags<CsrCfg<double>::BUCKET, CsrCfg<double>::RMAX>
                    <<<nb, 256, 0, s>>>(A->idx0, n, flag);
            else
                csr_block_flags<CsrCfg<float>::BUCKET, CsrCfg<float>::RMAX>
                    <<<nb, 256, 0, s>>>(A->idx0, n, flag);
            MXS_HIP(hipGetLastError());
        }
        mxs_status st = scan_i32(flag, pos, n, s);
        if (st != MXS_OK) return st;
        int32_t nblk = 0;
        MXS_HIP(hipMemcpyAsync(&nblk, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        int32_t *blk = nullptr;
        MXS_HIP(hipMalloc((void **)&blk, sizeof(int32_t) * ((size_t)nblk + 1)));
        csr_block_scatter<<<std::max(nb, 1), 256, 0, s>>>(flag, pos, n, blk);
        MXS_HIP(hipGetLastError());
        MXS_HIP(hipFreeAsync(flag, s));
        MXS_HIP(hipFreeAsync(pos, s));
        MXS_HIP(hipStreamSynchronize(s));
        A->csr.blk_row = blk;
        A->csr.nblk = nblk;
        A->owned.push_back(blk);
    } else if (A->fmt == MXS_COO) {
        const int64_t nt = (A->nnz + kCooTile - 1) / kCooTile;
        void *carry = nullptr;
        if (nt > 0) {
            MXS_HIP(hipMalloc(&carry, 2 * (size_t)nt * dsize(A->dtype)));
            A->owned.push_back(carry);
        }
        A->coo.carry = carry;
        A->coo.ntiles = nt;
    }
    A->optimized = true;
    return MXS_OK;
}

mxs_status dot_sigma_launch(int64_t n, mxs_dtype t, const void *a, const void *b, const int *done,
                            const DotSink *dot, hipStream_t s);

template <typename T>
static mxs_status spmv_typed(const mxs_mat_s *A, const T *x, T *y, const int *done,
                             const DotSink *dot, hipStream_t s)
{
    const DotSink ds = dot ? *dot : DotSink{nullptr, nullptr};
    if (A->nrows == 0) return MXS_OK;
    switch (A->fmt) {
    case MXS_CSR: {
        const int64_t nblk = A->csr.nblk;
        uint32_t grid;
        int64_t per;
        grid_for(nblk, dot != nullptr, &grid, &per);
        if (dot)
            csr_spmv_kernel<T, true><<<grid, 256, 0, s>>>(
                A->idx0, A->idx1, (const T *)A->vals, x, y, A->csr.blk_row, nblk, per, done, ds);
        else
            csr_spmv_kernel<T, false><<<grid, 256, 0, s>>>(
                A->idx0, A->idx1, (const T *)A->vals, x, y, A->csr.blk_row, nblk, per, done, ds);
        return launch_status();
    }
    case MXS_DIA: {
        const int64_t nblk = dia_blocks(A);
        uint32_t grid;
        int64_t per;
        grid_for(nblk, dot != nullptr, &grid, &per);
        if (dot)
            dia_spmv_kernel<T, true><<<grid, kDiaNT, 0, s>>>(A->nrows, A->ncols, A->ndiag, A->idx0,
                                                             (const T *)A->vals, x, y, nblk, per,
                                                             done, ds);
        else
            dia_spmv_kernel<T, false><<<grid, kDiaNT, 0, s>>>(A->nrows, A->ncols, A->ndiag,
                                                              A->idx0, (const T *)A->vals, x, y,
                                                              nblk, per, done, ds);
        return launch_status();
    }
    case MXS_COO: {
        const int64_t nt = A->coo.ntiles;
        if (nt == 0) {
            fill_kernel<T><<<(uint32_t)std::min<int64_t>((A->nrows + 255) / 256, 4096), 256, 0, s>>>(
                y, T(0), A->nrows, done);
        } else {
            coo_spmv_kernel<T><<<pad_grid(nt), kCooNT, 0, s>>>(
                A->nnz, A->nrows, A->idx0, A->idx1, (const T *)A->vals, x, y, (T *)A->coo.carry,
                nt, done);
            MXS_HIP(hipGetLastError());
            coo_fixup_kernel<T><<<(uint32_t)((nt + 255) / 256), 256, 0, s>>>(
                A->nnz, A->idx0, (const T *)A->coo.carry, y, nt, done);
        }
        MXS_HIP(hipGetLastError());
        if (dot) return dot_sigma_launch(A->nrows, A->dtype, x, y, done, dot, s);
        return MXS_OK;
    }
    }
    return MXS_ERR_UNSUPPORTED;
}

mxs_status dot_sigma_launch(int64_t n, mxs_dtype t, const void *a, const void *b, const int *done,
                            const DotSink *dot, hipStream_t s)
{
    if (t == MXS_F64)
        dot_sigma_kernel<double><<<(uint32_t)kDotGrid, 256, 0, s>>>(n, (const double *)a,
                                                                    (const double *)b, done, *dot);
    else
        dot_sigma_kernel<float><<<(uint32_t)kDotGrid, 256, 0, s>>>(n, (const float *)a,
                                                                  (const float *)b, done, *dot);
    return launch_status();
}

mxs_status spmv_launch(const mxs_mat_s *A, const void *x, void *y, const int *done,
                       const DotSink *dot, hipStream_t s)
{
    if (A->dtype == MXS_F64)
        return spmv_typed<double>(A, (const double *)x, (double *)y, done, dot, s);
    return spmv_typed<float>(A, (const float *)x, (float *)y, done, dot, s);
}

}  // namespace mxs
