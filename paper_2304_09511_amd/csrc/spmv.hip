// SpMV kernels for gfx950: y = A*x in CSR, DIA and COO (Algorithms 2, 3, 1
// of Section III-B), plus the analysis that builds each format's plan.
//
// All three are HBM-bound streams (0.12-0.23 flop/byte in FP64), so the
// design goals are wide coalesced loads of the matrix arrays, x gathers that
// hit in L2, deterministic reductions without floating-point atomics, and
// enough bytes in flight per CU.  No MFMA: SpMV is not a dense contraction.
//
// Each workgroup issues all of its block's matrix loads back to back
// (branch-free: lanes past a block's end re-read its last entry and are
// masked), then the dependent x gathers, so every wave keeps many loads in
// flight; concurrency across workgroups hides the LDS phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

// Tunables (compile-time).
#ifndef MXS_CSR_IPT64
#define MXS_CSR_IPT64 10
#endif
#ifndef MXS_CSR_IPT32
#define MXS_CSR_IPT32 10
#endif
#ifndef MXS_CSR_IPT_MANY
#define MXS_CSR_IPT_MANY 8 // CSR tiles owning more rows than the LDS-staged path takes
#endif
#ifndef MXS_CSR_IPT_SPARSE
#define MXS_CSR_IPT_SPARSE 4 // CSR tiles of rows shorter than five entries on average
#endif
#ifndef MXS_COO_IPT64
#define MXS_COO_IPT64 8
#endif
#ifndef MXS_COO_IPT32
#define MXS_COO_IPT32 12
#endif
#ifndef MXS_DIA_WIN
#define MXS_DIA_WIN 0 // 1: stage the x windows of interior DIA blocks in LDS
#endif
#ifndef MXS_DIA_RPT64
#define MXS_DIA_RPT64 1
#endif
#ifndef MXS_DIA_RPT32
#define MXS_DIA_RPT32 2
#endif
#ifndef MXS_DIA_DU
#define MXS_DIA_DU 4
#endif
#ifndef MXS_DIA_SHARE
#define MXS_DIA_SHARE 1 // 1: one x load per run of three consecutive offsets, neighbours by lane shifts
#endif

#ifndef MXS_DIA_TU
#define MXS_DIA_TU 1 // runs of three offsets whose loads are issued together (1 measured 1-3% faster than 2 or 3)
#endif

#ifndef MXS_STREAM_NT
#define MXS_STREAM_NT 1 // non-temporal loads for matrix values read once per SpMV
#endif
#ifndef MXS_COO_IPT
#define MXS_COO_IPT 4
#endif
#ifndef MXS_COO_IPT_SCATTER
#define MXS_COO_IPT_SCATTER 1 // segmented-scan tiles of a column block (see coo_plan)
#endif
#ifndef MXS_PERSIST
#define MXS_PERSIST 0 // 1: at most one resident wave of workgroups, each over a run of blocks
#endif

namespace mxs {

// Matrix values and indices are read once per SpMV; loading them with the
// non-temporal hint keeps x (reused across rows) resident in L2.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
#if MXS_STREAM_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Persistent grid: at most as many workgroups as are resident at once.
template <typename K>
static int64_t resident_workgroups(K kernel, int nt)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int64_t> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair((const void *)kernel, dev);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess)
        per_cu = 4;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int64_t r = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * cus);
    cache[key] = r;
    return r;
}

// Workgroup count and blocks per workgroup for a persistent launch over
// `nblk` blocks: the grid is a multiple of 8 (for the XCD remap) and at most
// the resident capacity; workgroup g takes blocks [g*per, (g+1)*per).
static void persistent_grid(int64_t nblk, int64_t resident, uint32_t *grid, int64_t *per)
{
    const int64_t cap = std::max<int64_t>(kNumXcd, resident / kNumXcd * kNumXcd);
    int64_t g = std::min<int64_t>(pad_grid(std::max<int64_t>(nblk, 1)), cap);
    *per = (std::max<int64_t>(nblk, 1) + g - 1) / g;
    g = (std::max<int64_t>(nblk, 1) + *per - 1) / *per;
    *grid = pad_grid(g);
}

// ===========================================================================
// CSR (Algorithm 2), split by non-zeros: tile t covers entries
// [t*TILE, (t+1)*TILE) and owns the rows that start in it.  A workgroup
// loads its tile's columns and values at once (no dependent descriptor
// load in front of them), gathers x, stages the products in LDS and reduces
// each owned row with a lane group sized to the tile's row count.  The last
// owned row usually ends a few entries past the tile: the owner reads up to
// EXT more entries and finishes it.  Rows reaching further (long rows) leave
// a head / tail piece in a carry array that an ordered fix-up kernel adds.
// ===========================================================================
template <typename T>
struct CsrCfg;
template <>
struct CsrCfg<double> {
    static constexpr int NT = 256;
    static constexpr int IPT = MXS_CSR_IPT64;
    static constexpr int TILE = NT * IPT;
    static constexpr int EXT = NT;  // entries past the tile an owner may read
    static constexpr int RMAX = 256; // owned rows whose pointers are staged in LDS
};
template <>
struct CsrCfg<float> {
    static constexpr int NT = 256;
    static constexpr int IPT = MXS_CSR_IPT32;
    static constexpr int TILE = NT * IPT;
    static constexpr int EXT = NT;
    static constexpr int RMAX = 256;
};
// COO's row tiles use the same plan with their own tile sizes (measured
// best at 128^3: 8 entries per thread in FP64, 12 in FP32; CSR's entry
// tiles 10 in both).
template <typename T>
struct CooCfg;
template <>
struct CooCfg<double> {
    static constexpr int NT = 256;
    static constexpr int IPT = MXS_COO_IPT64;
    static constexpr int TILE = NT * IPT;
    static constexpr int EXT = NT;
};
template <>
struct CooCfg<float> {
    static constexpr int NT = 256;
    static constexpr int IPT = MXS_COO_IPT32;
    static constexpr int TILE = NT * IPT;
    static constexpr int EXT = NT;
};

// Per-tile flags of the plan.
constexpr int kCsrHeadCarry = 1 << 16; // head piece goes to the carry array
constexpr int kCsrLastCarry = 1 << 17; // last owned row reaches past EXT: tail piece carried
constexpr int kCsrLongRows = 1 << 18;  // an owned row has more than kLongRow entries
constexpr int kLongRow = 64;           // longer rows are reduced by a whole wave

// tile_row[t] = first row whose first entry is at position >= t*TILE
// (lower bound over irp); tile_row[ntiles] = nrows.
__global__ void csr_tile_rows_kernel(const int32_t *__restrict__ irp, int32_t nrows, int64_t ntiles,
                                     int tile, int32_t *__restrict__ tile_row)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        tile_row[t] = nrows;
        return;
    }
    const int64_t key = t * (int64_t)tile;
    int64_t lo = 0, hi = (int64_t)nrows + 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (irp[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    tile_row[t] = (int32_t)min(lo, (int64_t)nrows);
}

// tile_info[t]: entries the owner reads past its tile (low 16 bits) and the
// two carry flags; *any_carry is set when a fix-up pass is needed.  The
// long-row flag is added by csr_long_rows_kernel.
__global__ void csr_tile_info_kernel(const int32_t *__restrict__ irp, const int32_t *__restrict__ tile_row,
                                     int64_t nnz, int64_t ntiles, int tile, int ext,
                                     int32_t *__restrict__ info, int *__restrict__ any_carry)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int32_t r_lo = tile_row[t], r_hi = tile_row[t + 1];
    const int64_t k0 = t * (int64_t)tile;
    const int64_t tile_end = min(nnz, k0 + tile);
    int32_t v = 0;
    if (r_hi > r_lo) {
        const int64_t over = (int64_t)irp[r_hi] - tile_end;
        if (over > ext) v |= kCsrLastCarry;
        else if (over > 0) v |= (int32_t)over;
    }
    if (r_lo > 0 && irp[r_lo] > k0) {
        // head piece: the row that started before k0; its owner finished it
        // unless it reaches more than ext entries past the owner's tile
        const int64_t h_start = irp[r_lo - 1];
        const int64_t owner_end = (h_start / tile + 1) * (int64_t)tile;
        if ((int64_t)irp[r_lo] - owner_end > ext) v |= kCsrHeadCarry;
    }
    info[t] = v;
    if (v & kCsrLastCarry) atomicOr(any_carry, 1);
}

// Flags the tiles that own a row longer than kLongRow (a thread per row).
__global__ void csr_long_rows_kernel(const int32_t *__restrict__ irp, int32_t nrows, int tile,
                                     int32_t *__restrict__ info)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int32_t b = irp[r];
    if (irp[r + 1] - b > kLongRow) atomicOr(&info[b / tile], kCsrLongRows);
}

// Reduces a tile's owned rows [0, nr), whose products (or staged values) sit
// in LDS: lane groups of G lanes, the largest power of two with G*nr <= NT,
// take a row each.  With `queue` set, rows of more than kLongRow entries are
// put on an LDS list instead and then reduced by whole waves, so that one
// long row does not hold the workgroup for len/G steps while the other lanes
// wait.  lo(r) / hi(r) give a row's local entry range, part(b, e, lane, g)
// a lane's partial sum over [b, e) with stride g, put(r, sum) stores the row.
// A row's summation order depends only on its length and position.
template <typename T, int NT, int CAP, typename Lo, typename Hi, typename Part, typename Put>
__device__ __forceinline__ void reduce_tile_rows(int nr, bool queue, int32_t *longq, int *nlong,
                                                 Lo lo, Hi hi, Part part, Put put)
{
    const int tid = threadIdx.x;
    int G = 64;
    while (G > 1 && G * nr > NT) G >>= 1;
    queue = queue && G < kWave;
    const int lane = tid & (G - 1);
    for (int r = tid / G; r < nr; r += NT / G) {
        const int b = lo(r), e = hi(r);
        if (queue && e - b > kLongRow) {
            if (lane == 0) longq[min(atomicAdd(nlong, 1), CAP - 1)] = r;
            continue;
        }
        T sum = part(b, e, lane, G);
        for (int off = G >> 1; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
        if (lane == 0) put(r, sum);
    }
    if (queue) {
        __syncthreads();
        const int nl = min(*nlong, CAP);
        const int wl = tid & (kWave - 1);
        for (int q = tid / kWave; q < nl; q += NT / kWave) {
            const int r = longq[q];
            T sum = part(lo(r), hi(r), wl, kWave);
            for (int off = kWave >> 1; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
            if (wl == 0) put(r, sum);
        }
    }
}

#ifndef MXS_CSR_TRIM
#define MXS_CSR_TRIM 1 // 1: waves skip the second row-pointer load and extension loads they do not need
#endif

#ifndef MXS_DIA_YNT
#define MXS_DIA_YNT 1 // 1: DIA writes y with non-temporal stores
#endif

#ifndef MXS_CSR_GX_DEFAULT
#define MXS_CSR_GX_DEFAULT 0 // 1: the staged-gather implementation is CSR's default
#endif

#ifndef MXS_CSR_GXU
#define MXS_CSR_GXU 8 // staged-gather CSR: entries a lane gathers per step
#endif

#ifndef MXS_CSR_WPE
#define MXS_CSR_WPE 0 // >0: ask the compiler for this many waves per SIMD
#endif
#if MXS_CSR_WPE > 0
#define MXS_CSR_ATTR __attribute__((amdgpu_waves_per_eu(MXS_CSR_WPE)))
#else
#define MXS_CSR_ATTR
#endif

// GX (the staged-gather implementation): the tile's columns and values are
// staged in LDS and x is gathered in the reduction, by the lane group of each
// row.  Lanes then gather x for neighbouring rows at the same position in
// their rows, which for banded matrices are neighbouring addresses: fewer
// cache lines per gather instruction than gathering in entry order.
// IPTT: entries per thread of the plan's tiles (csr_plan_ipt).
template <typename T, bool DOT, bool GX, int IPTT>
__global__ __launch_bounds__(256) MXS_CSR_ATTR void csr_spmv_kernel(
    const int32_t *__restrict__ irp, const int32_t *__restrict__ aj, const T *__restrict__ av,
    const T *__restrict__ x, T *__restrict__ y, const int32_t *__restrict__ tile_row,
    const int32_t *__restrict__ tile_info, int64_t nnz, int64_t ntiles, int64_t per,
    T *__restrict__ carry, const int *__restrict__ done, double *__restrict__ partials, int acc)
{
    using C = CsrCfg<T>;
    constexpr int NT = C::NT, IPT = IPTT, TILE = NT * IPTT, EXT = C::EXT, RMAX = C::RMAX;
    static_assert(EXT == NT, "one overflow entry per thread");
    __shared__ T prod[TILE + EXT]; // products, or the values when GX
    __shared__ int32_t scol[GX ? TILE + EXT : 1];
    __shared__ int32_t lrp[RMAX + 1];
    __shared__ double red[NT / kWave];
    constexpr int LCAP = (TILE + EXT) / kLongRow;
    __shared__ int32_t longq[LCAP];
    __shared__ int nlong;
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t_lo = g * per, t_hi = min(ntiles, t_lo + per);
    double dpart = 0.0;
    for (int64_t tile = t_lo; tile < t_hi; ++tile) {
        const int64_t k0 = tile * TILE;
        const int32_t n = (int32_t)min((int64_t)TILE, nnz - k0);
        const int32_t r_lo = tile_row[tile], r_hi = tile_row[tile + 1];
        const int32_t info = tile_info[tile];
        const int32_t nr = r_hi - r_lo;
        const int32_t n_ext = info & 0xffff;
        const bool head_carry = info & kCsrHeadCarry;
        const bool last_carry = info & kCsrLastCarry;
        // row pointers of the owned rows (clamped indices, always in range)
        const int32_t lr = irp[r_lo + min(tid, nr)];
#if MXS_CSR_TRIM
        // the extension entries are read by the waves whose lanes reach them
        const bool ext_wave = (tid & ~(kWave - 1)) < n_ext; // uniform per wave
#else
        const bool ext_wave = n_ext > 0;
#endif
#if MXS_CSR_TRIM
        const int32_t lr_hi = nr >= NT ? irp[r_lo + min(tid + NT, nr)] : 0; // uniform test
#else
        const int32_t lr_hi = irp[r_lo + min(tid + NT, nr)];
#endif
        {
            // all matrix loads unconditional (lanes past the end re-read the
            // last entry, masked later) so they issue back to back
            const int32_t *__restrict__ ajb = aj + k0;
            const T *__restrict__ avb = av + k0;
            int32_t col[IPT + 1];
            T val[IPT + 1], xv[IPT + 1];
#pragma unroll
            for (int e = 0; e < IPT; ++e) col[e] = ld_stream(&ajb[(uint32_t)min(e * NT + tid, n - 1)]);
#pragma unroll
            for (int e = 0; e < IPT; ++e) val[e] = ld_stream(&avb[(uint32_t)min(e * NT + tid, n - 1)]);
            const uint32_t ke = (uint32_t)(n + min(tid, max(n_ext - 1, 0)));
            col[IPT] = ext_wave ? ld_stream(&ajb[ke]) : 0;
            val[IPT] = ext_wave ? ld_stream(&avb[ke]) : T(0);
            if constexpr (GX) {
#pragma unroll
                for (int e = 0; e < IPT; ++e) {
                    const int j = e * NT + tid;
                    if (j < n) {
                        prod[j] = val[e];
                        scol[j] = col[e];
                    }
                }
                if (tid < n_ext) {
                    prod[n + tid] = val[IPT];
                    scol[n + tid] = col[IPT];
                }
            } else {
#pragma unroll
                for (int e = 0; e < IPT; ++e) xv[e] = x[(uint32_t)col[e]];
                xv[IPT] = ext_wave ? x[(uint32_t)col[IPT]] : T(0);
#pragma unroll
                for (int e = 0; e < IPT; ++e) {
                    const int j = e * NT + tid;
                    if (j < n) prod[j] = val[e] * xv[e];
                }
                if (tid < n_ext) prod[n + tid] = val[IPT] * xv[IPT];
            }
        }
        const bool staged = nr <= RMAX;
        if (staged) {
            if (tid <= nr) lrp[tid] = lr - (int32_t)k0;
            if (tid + NT <= nr) lrp[tid + NT] = lr_hi - (int32_t)k0;
        }
        if (tid == 0) nlong = 0;
        __syncthreads();
        auto rp = [&](int r) -> int32_t { return staged ? lrp[r] : irp[r_lo + r] - (int32_t)k0; };
        if (head_carry) {
            // piece of a long row that began in an earlier tile
            const int32_t hl = min(rp(0), n);
            T hs = T(0);
            for (int j = tid; j < hl; j += NT) hs += GX ? prod[j] * x[(uint32_t)scol[j]] : prod[j];
            const double tot = block_sum<NT>((double)hs, red);
            if (tid == 0) carry[2 * tile] = (T)tot;
        }
        const int32_t lim = n + n_ext; // local end of the entries loaded
        reduce_tile_rows<T, NT, LCAP>(
            nr, (info & kCsrLongRows) != 0, longq, &nlong, [&](int r) { return rp(r); },
            [&](int r) { return min(rp(r + 1), lim); },
            [&](int b, int e, int lane, int G) {
                T sum = T(0);
                if constexpr (GX) {
                    // U entries per lane per step; lanes past the row's end
                    // re-read its last entry with a zero value
                    constexpr int U = MXS_CSR_GXU;
                    for (int k0l = b + lane; k0l < e; k0l += U * G) {
                        int32_t c[U];
                        T v[U], xg[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int k = k0l + u * G;
                            const int kk = min(k, e - 1);
                            c[u] = scol[kk];
                            v[u] = k < e ? prod[kk] : T(0);
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) xg[u] = x[(uint32_t)c[u]];
#pragma unroll
                        for (int u = 0; u < U; ++u) sum += v[u] * xg[u];
                    }
                } else {
                    for (int k = b + lane; k < e; k += G) sum += prod[k];
                }
                return sum;
            },
            [&](int r, T sum) {
                if (last_carry && r == nr - 1) {
                    carry[2 * tile + 1] = sum;
                } else {
                    const T yv = acc ? y[r_lo + r] + sum : sum;
                    y[r_lo + r] = yv;
                    if (DOT) dpart += (double)yv * (double)x[r_lo + r];
                }
            });
        __syncthreads();
    }
    if (DOT) {
        const double bs = block_sum<NT>(dpart, red);
        if (tid == 0) partials[blockIdx.x] = bs;
    }
}

// Matrices with far more rows than entries (e.g. the remainder of a split):
// fixed-size entry tiles would each own very many rows, so a thread takes a
// row instead.  Rows are short here by construction (the average is below
// one half), so the sequential inner loop is short.
constexpr int64_t kRowwiseGridMax = 8192;

template <typename T, bool DOT>
__global__ __launch_bounds__(256) void csr_rowwise_kernel(
    const int32_t *__restrict__ irp, const int32_t *__restrict__ aj, const T *__restrict__ av,
    const T *__restrict__ x, T *__restrict__ y, int32_t nrows, const int *__restrict__ done,
    double *__restrict__ partials, int acc)
{
    __shared__ double red[256 / kWave];
    if (done && *done) return;
    double dpart = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k1 = irp[r + 1];
        T s = T(0);
        for (int32_t k = irp[r]; k < k1; ++k) s += av[k] * x[aj[k]];
        const T yv = acc ? y[r] + s : s;
        y[r] = yv;
        if (DOT) dpart += (double)yv * (double)x[r];
    }
    if (DOT) {
        const double bs = block_sum<256>(dpart, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    }
}

static uint32_t rowwise_grid(int32_t nrows)
{
    return (uint32_t)std::clamp<int64_t>(((int64_t)nrows + 255) / 256, 1, kRowwiseGridMax);
}

// A wavefront per row (the "vector" CSR kernel): the lanes stride over the
// row's entries and a wave reduction sums them, so a long row is spread
// over 64 lanes; short rows leave most lanes idle.
constexpr int64_t kVectorGridMax = 16384;

template <typename T>
__global__ __launch_bounds__(256) void csr_vector_kernel(
    const int32_t *__restrict__ irp, const int32_t *__restrict__ aj, const T *__restrict__ av,
    const T *__restrict__ x, T *__restrict__ y, int32_t nrows, const int *__restrict__ done, int acc)
{
    if (done && *done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; r < nrows;
         r += nw) {
        const int32_t b = irp[r], e = irp[r + 1];
        T s = T(0);
        for (int32_t k = b + lane; k < e; k += kWave) s += av[k] * x[aj[k]];
        for (int off = kWave >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (lane == 0) y[r] = acc ? y[r] + s : s;
    }
}

static uint32_t vector_grid(int32_t nrows)
{
    return (uint32_t)std::clamp<int64_t>(((int64_t)nrows + 3) / 4, 1, kVectorGridMax);
}

// Rows too long for their owner's overflow window: owner's tail piece plus
// the head pieces of the following tiles, in tile order.
template <typename T, bool DOT>
__global__ __launch_bounds__(256) void csr_fixup_kernel(
    const int32_t *__restrict__ irp, const int32_t *__restrict__ tile_row,
    const int32_t *__restrict__ tile_info, const T *__restrict__ carry, const T *__restrict__ x,
    T *__restrict__ y, int64_t nnz, int64_t ntiles, int tile, const int *__restrict__ done,
    double *__restrict__ partials, int acc)
{
    __shared__ double red[256 / kWave];
    if (done && *done) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0;
    if (t < ntiles && (tile_info[t] & kCsrLastCarry)) {
        const int32_t r = tile_row[t + 1] - 1;
        const int64_t end = irp[r + 1];
        T v = carry[2 * t + 1];
        for (int64_t u = t + 1; u < ntiles; ++u) {
            v += carry[2 * u];
            if (end <= min(nnz, (u + 1) * (int64_t)tile)) break;
        }
        if (acc) v += y[r];
        y[r] = v;
        if (DOT) d = (double)v * (double)x[r];
    }
    if (DOT) {
        const double bs = block_sum<256>(d, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
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
    static constexpr int RPT = MXS_DIA_RPT64;
};
template <>
struct DiaCfg<float> {
    static constexpr int RPT = MXS_DIA_RPT32;
};

constexpr int kDiaStage = 256;  // diagonals whose offsets / window positions fit in LDS
constexpr int kDiaMaxRuns = 64;  // x windows per block
constexpr int kDiaWinMax = 6144; // x-window elements per block (48 KiB in FP64)
constexpr int kDiaDU = MXS_DIA_DU; // diagonals whose loads are issued together

// Interior blocks (every diagonal inside [0, ncols) for all of the block's
// rows) stage x in LDS: sorted offsets that lie within a block height of
// each other form one run, and run j needs x[row0 + f_j, row0 + f_j + len_j)
// once per block, instead of one shifted load per diagonal.  Each diagonal
// then reads its x values from LDS at its run position.  Other blocks load
// x from global memory with per-row range checks.
// Offset of diagonal d for the boundary path (spos holds window positions
// when windows are on, offsets otherwise).
__device__ __forceinline__ int64_t spos_off(const int32_t *spos, const int32_t *, bool win,
                                            const int32_t *__restrict__ doff, int d)
{
    return win ? (int64_t)doff[d] : (int64_t)spos[d];
}

// Lane shifts across the 64-lane wave (DPP wave_shr:1 / wave_shl:1): lane l
// receives lane l-1 (resp. l+1) of v; the lane without a source (0, resp.
// 63) receives `edge`.
__device__ __forceinline__ int dpp_shift(int edge, int v, bool right)
{
    return right ? __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false)
                 : __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float lane_shift(float edge, float v, bool right)
{
    return __builtin_bit_cast(float, dpp_shift(__builtin_bit_cast(int, edge),
                                               __builtin_bit_cast(int, v), right));
}
__device__ __forceinline__ double lane_shift(double edge, double v, bool right)
{
    const int2 e = __builtin_bit_cast(int2, edge), w = __builtin_bit_cast(int2, v);
    int2 o;
    o.x = dpp_shift(e.x, w.x, right);
    o.y = dpp_shift(e.y, w.y, right);
    return __builtin_bit_cast(double, o);
}

// Values come either diagonal-major (av[d*nrows + i], the container's
// layout; `blocked` false) or row-blocked (av[(b*ndiag + d)*ROWS + i - row0],
// the plan's copy; `blocked` true), where each block's diagonals are one
// contiguous stream.
template <typename T, bool DOT>
__global__ __launch_bounds__(256) void dia_spmv_kernel(
    int32_t nrows, int32_t ncols, int32_t ndiag, const int32_t *__restrict__ doff,
    const T *__restrict__ av, int blocked, const T *__restrict__ x, T *__restrict__ y, int64_t nblk,
    int64_t per, const int *__restrict__ done, double *__restrict__ partials,
    const int32_t *__restrict__ wpos, const int32_t *__restrict__ wruns, int32_t nruns,
    int32_t wlen, int32_t first_off, int32_t last_off, int32_t triples)
{
    constexpr int NT = kDiaNT;
    constexpr int RPT = DiaCfg<T>::RPT;
    constexpr int ROWS = NT * RPT;
    constexpr int DU = kDiaDU;
    extern __shared__ __align__(16) unsigned char dia_dyn[];
    T *xw = reinterpret_cast<T *>(dia_dyn);
    __shared__ int32_t spos[kDiaStage]; // window position (or offset) of each diagonal
    __shared__ int32_t srun[3 * kDiaMaxRuns];
    __shared__ double red[NT / kWave];
    if (done && *done) return;
    const int tid = threadIdx.x;
    const bool win = wlen > 0; // implies ndiag <= kDiaStage and nruns <= kDiaMaxRuns
    const bool staged = ndiag <= kDiaStage;
    if (staged)
        for (int i = tid; i < ndiag; i += NT) spos[i] = win ? wpos[i] : doff[i];
    if (win)
        for (int i = tid; i < 3 * nruns; i += NT) srun[i] = wruns[i];
    __syncthreads();
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b_lo = g * per, b_hi = min(nblk, b_lo + per);
    double dpart = 0.0;
    for (int64_t b = b_lo; b < b_hi; ++b) {
        const int64_t row0 = b * ROWS;
        T sum[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) sum[r] = T(0);
        // Offsets ascend, so all diagonals stay in range for the block's rows
        // iff the first and the last one do.
        const bool interior = staged && ndiag > 0 && row0 + ROWS <= nrows &&
                              row0 + first_off >= 0 && row0 + ROWS - 1 + last_off < ncols;
        // x at the block's own rows for the fused dot, loaded now so that its
        // latency hides under the diagonals' loads (square A: row < ncols)
        T xself[RPT];
        if (DOT) {
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                xself[r] = x[min(row0 + r * NT + tid, (int64_t)min(nrows, ncols) - 1)];
        }
        // value of diagonal d for the block's local row li is a_blk[d*dstride + li]
        const T *__restrict__ a_blk = blocked ? av + b * (int64_t)ndiag * ROWS : av + row0;
        const int64_t dstride = blocked ? (int64_t)ROWS : (int64_t)nrows;
        if (interior) {
            if (win) {
                // stage the x windows (loads unconditional: indices clamped)
                for (int i0 = 0; i0 < wlen; i0 += 8 * NT) {
                    T wv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int e = min(i0 + q * NT + tid, wlen - 1);
                        int j = 0;
                        for (int k = 1; k < nruns; ++k) j = e >= srun[3 * k + 2] ? k : j;
                        wv[q] = x[row0 + srun[3 * j] + (e - srun[3 * j + 2])];
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int e = i0 + q * NT + tid;
                        if (e < wlen) xw[e] = wv[q];
                    }
                }
                __syncthreads();
            }
            const T *__restrict__ x_blk = x + row0;
            int d = 0;
#if MXS_DIA_SHARE
            if (triples && !win) {
                // offsets o, o+1, o+2: one x load at o+1 per row; its
                // neighbours come from the adjacent lanes, and the two values
                // past the wave's ends from wave-uniform loads
                const int wbase = __builtin_amdgcn_readfirstlane(tid & ~(kWave - 1));
                constexpr int TU = MXS_DIA_TU;
                for (; d + 3 * TU <= ndiag; d += 3 * TU) {
                    T va[TU][3][RPT], xc[TU][RPT], el[TU][RPT], er[TU][RPT];
#pragma unroll
                    for (int t = 0; t < TU; ++t) {
                        const int32_t o0 = __builtin_amdgcn_readfirstlane(spos[d + 3 * t]);
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            const T *__restrict__ a = a_blk + (int64_t)(d + 3 * t + k) * dstride;
#pragma unroll
                            for (int r = 0; r < RPT; ++r)
                                va[t][k][r] = ld_stream(&a[(uint32_t)(r * NT + tid)]);
                        }
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const int64_t w0 = (int64_t)r * NT + wbase + o0; // wave's first row + o0
                            xc[t][r] = x_blk[(int64_t)o0 + 1 + r * NT + tid];
                            el[t][r] = x_blk[w0];
                            er[t][r] = x_blk[w0 + kWave + 1];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < TU; ++t)
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const T xl = lane_shift(el[t][r], xc[t][r], true);
                            const T xr = lane_shift(er[t][r], xc[t][r], false);
                            sum[r] += va[t][0][r] * xl;
                            sum[r] += va[t][1][r] * xc[t][r];
                            sum[r] += va[t][2][r] * xr;
                        }
                }
                for (; d + 3 <= ndiag; d += 3) {
                    const int32_t o0 = __builtin_amdgcn_readfirstlane(spos[d]);
                    T va[3][RPT], xc[RPT], el[RPT], er[RPT];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const T *__restrict__ a = a_blk + (int64_t)(d + k) * dstride;
#pragma unroll
                        for (int r = 0; r < RPT; ++r) va[k][r] = ld_stream(&a[(uint32_t)(r * NT + tid)]);
                    }
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int64_t w0 = (int64_t)r * NT + wbase + o0;
                        xc[r] = x_blk[(int64_t)o0 + 1 + r * NT + tid];
                        el[r] = x_blk[w0];
                        er[r] = x_blk[w0 + kWave + 1];
                    }
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const T xl = lane_shift(el[r], xc[r], true);
                        const T xr = lane_shift(er[r], xc[r], false);
                        sum[r] += va[0][r] * xl;
                        sum[r] += va[1][r] * xc[r];
                        sum[r] += va[2][r] * xr;
                    }
                }
            }
#endif
            for (; d + DU <= ndiag; d += DU) {
                T va[DU][RPT], vx[DU][RPT];
#pragma unroll
                for (int q = 0; q < DU; ++q) {
                    const int32_t p = __builtin_amdgcn_readfirstlane(spos[d + q]);
                    const T *__restrict__ a = a_blk + (int64_t)(d + q) * dstride;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const uint32_t li = (uint32_t)(r * NT + tid);
                        va[q][r] = ld_stream(&a[li]);
                        vx[q][r] = win ? xw[p + li] : x_blk[(int64_t)p + li];
                    }
                }
#pragma unroll
                for (int q = 0; q < DU; ++q)
#pragma unroll
                    for (int r = 0; r < RPT; ++r) sum[r] += va[q][r] * vx[q][r];
            }
            for (; d < ndiag; ++d) {
                const int32_t p = __builtin_amdgcn_readfirstlane(spos[d]);
                const T *__restrict__ a = a_blk + (int64_t)d * dstride;
                T va[RPT], vx[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const uint32_t li = (uint32_t)(r * NT + tid);
                    va[r] = ld_stream(&a[li]);
                    vx[r] = win ? xw[p + li] : x_blk[(int64_t)p + li];
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) sum[r] += va[r] * vx[r];
            }
            if (win) __syncthreads(); // the next block overwrites the windows
        } else {
            // boundary blocks: same chunks, loads at clamped indices (always
            // in range) and products masked by the row's range test
            const int64_t lmax = min((int64_t)ROWS, (int64_t)nrows - row0) - 1;
            int d = 0;
            for (; d < ndiag; d += DU) {
                T va[DU][RPT], vx[DU][RPT];
                bool ok[DU][RPT];
#pragma unroll
                for (int q = 0; q < DU; ++q) {
                    const int dq = min(d + q, ndiag - 1);
                    const int64_t off = staged ? spos_off(spos, wpos, win, doff, dq) : doff[dq];
                    const T *__restrict__ a = a_blk + (int64_t)dq * dstride;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int64_t li = r * NT + tid;
                        const int64_t k = row0 + li + off;
                        ok[q][r] = d + q < ndiag && li <= lmax && k >= 0 && k < ncols;
                        va[q][r] = ld_stream(&a[min(li, lmax)]);
                        vx[q][r] = x[min(max(k, (int64_t)0), (int64_t)ncols - 1)];
                    }
                }
#pragma unroll
                for (int q = 0; q < DU; ++q)
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        if (ok[q][r]) sum[r] += va[q][r] * vx[q][r];
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int64_t i = row0 + r * NT + tid;
            if (i < nrows) {
#if MXS_DIA_YNT
                __builtin_nontemporal_store(sum[r], &y[i]);
#else
                y[i] = sum[r];
#endif
                if (DOT) dpart += (double)sum[r] * (double)xself[r];
            }
        }
    }
    if (DOT) {
        const double bs = block_sum<NT>(dpart, red);
        if (tid == 0) partials[blockIdx.x] = bs;
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
constexpr int kCooGapQ = 32;      // long runs of empty rows a tile queues for its workgroup
constexpr int kCooShortGap = 64;  // runs up to this long are zeroed by the thread that meets them
constexpr int kCooIPT = MXS_COO_IPT;

template <int IPT>
__device__ __forceinline__ int coo_pad(int j) { return j + j / IPT; }

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

// IPT: entries per thread of the plan's segmented tiles (coo_plan).
template <typename T, int IPT>
__global__ __launch_bounds__(256) void coo_spmv_kernel(
    int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai, const int32_t *__restrict__ aj,
    const T *__restrict__ av, const T *__restrict__ x, T *__restrict__ y, T *__restrict__ carry,
    int64_t ntiles, int64_t per, const int *__restrict__ done, int acc)
{
    constexpr int NT = kCooNT, TILE = NT * IPT;
    constexpr int PADDED = TILE + TILE / IPT;
    __shared__ int32_t srow[PADDED];
    __shared__ T sval[PADDED];
    __shared__ int sh[NT / kWave];
    __shared__ T sv[NT / kWave];
    // runs of empty rows longer than kCooShortGap, zeroed by the whole
    // workgroup after the tile (a thread zeroes shorter runs, and long ones
    // that find the queue full, itself)
    __shared__ int32_t gap_lo[kCooGapQ], gap_hi[kCooGapQ];
    __shared__ int gap_n;
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t_lo = g * per, t_hi = min(ntiles, t_lo + per);
    auto zero_rows = [&](int32_t lo, int32_t hi) {
        if (hi - lo > kCooShortGap) {
            const int q = atomicAdd(&gap_n, 1);
            if (q < kCooGapQ) {
                gap_lo[q] = lo;
                gap_hi[q] = hi;
                return;
            }
        }
        for (int32_t z = lo; z < hi; ++z) y[z] = T(0);
    };

    for (int64_t tile = t_lo; tile < t_hi; ++tile) {
        const int64_t k0 = tile * TILE;
        const int n = (int)min((int64_t)TILE, nnz - k0);
        if (tid == 0) gap_n = 0; // read after the barriers below
        {
            // Unconditional loads (the last tile clamps to its final entry) so
            // they issue back to back: rows, columns, values, then x gathers.
            const int32_t *__restrict__ aib = ai + k0;
            const int32_t *__restrict__ ajb = aj + k0;
            const T *__restrict__ avb = av + k0;
            int32_t row[IPT], col[IPT];
            T val[IPT], xv[IPT];
#pragma unroll
            for (int e = 0; e < IPT; ++e) col[e] = ld_stream(&ajb[(uint32_t)min(e * NT + tid, n - 1)]);
#pragma unroll
            for (int e = 0; e < IPT; ++e) val[e] = ld_stream(&avb[(uint32_t)min(e * NT + tid, n - 1)]);
#pragma unroll
            for (int e = 0; e < IPT; ++e) row[e] = ld_stream(&aib[(uint32_t)min(e * NT + tid, n - 1)]);
#pragma unroll
            for (int e = 0; e < IPT; ++e) xv[e] = x[(uint32_t)col[e]];
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                const int j = e * NT + tid;
                if (j < n) {
                    srow[coo_pad<IPT>(j)] = row[e];
                    sval[coo_pad<IPT>(j)] = val[e] * xv[e];
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
            const int32_t pr = j == 0 ? prev_row : srow[coo_pad<IPT>(j - 1)];
            if (srow[coo_pad<IPT>(j)] != pr) {
                mine.h = 1;
                mine.v = T(0);
            }
            mine.v += sval[coo_pad<IPT>(j)];
        }
        const SegPair<T> cin = block_seg_excl_scan<T, NT>(mine, sh, sv);
        // pass 2: emit every segment that closes inside this run
        T s = cin.v;
        for (int j = b0; j < b1; ++j) {
            const int32_t rw = srow[coo_pad<IPT>(j)];
            const int32_t pr = j == 0 ? prev_row : srow[coo_pad<IPT>(j - 1)];
            if (rw != pr) {
                if (j > 0) {
                    if (tile_cont && pr == first_row) carry[2 * tile] = s;
                    else y[pr] = acc ? y[pr] + s : s;
                }
                if (!acc && rw > pr + 1) zero_rows(pr + 1, rw); // rows without entries
                s = T(0);
            }
            s += sval[coo_pad<IPT>(j)];
        }
        if (b0 < n && b1 == n) {
            // the thread holding the tile's last entry closes or hands over its segment
            const int32_t last = srow[coo_pad<IPT>(n - 1)];
            const bool is_cont = tile_cont && last == first_row;
            if (next_row == last) {
                carry[2 * tile + (is_cont ? 0 : 1)] = s;
            } else {
                if (is_cont) carry[2 * tile] = s;
                else y[last] = acc ? y[last] + s : s;
                if (k0 + n == nnz && !acc && nrows > last + 1) zero_rows(last + 1, nrows);
            }
        }
        __syncthreads();
        const int ng = min(gap_n, kCooGapQ);
        for (int q = 0; q < ng; ++q)
            for (int32_t z = gap_lo[q] + tid; z < gap_hi[q]; z += NT) y[z] = T(0);
        __syncthreads();
    }
}

// COO on the CSR tiling.  The plan (computed once from the row ids) gives
// each tile of TILE entries its first owned row -- the rows whose first entry
// lies in the tile -- and how far its last row reaches past the tile.  The
// kernel loads row ids with the columns and values, stages products and row
// ids in LDS, and rebuilds the owned rows' local start positions: an entry
// whose row differs from the previous entry's opens that row, and the empty
// rows before it start at the same position.  Rows are then reduced by lane
// groups as in CSR; rows longer than the owner's window leave carries.
constexpr int kCooRowsMax = 512; // owned rows per tile whose starts fit in LDS

template <typename T>
__global__ __launch_bounds__(256) void coo_rows_kernel(
    const int32_t *__restrict__ ai, const int32_t *__restrict__ aj, const T *__restrict__ av,
    const T *__restrict__ x, T *__restrict__ y, const int32_t *__restrict__ tile_row,
    const int32_t *__restrict__ tile_info, int64_t nnz, int64_t ntiles, int64_t per,
    T *__restrict__ carry, const int *__restrict__ done, int acc)
{
    using C = CooCfg<T>;
    constexpr int NT = C::NT, IPT = C::IPT, TILE = C::TILE, EXT = C::EXT, RM = kCooRowsMax;
    static_assert(EXT == NT, "one overflow entry per thread");
    __shared__ T prod[TILE + EXT];
    __shared__ int32_t srow[TILE];
    __shared__ int32_t lrp[RM + 1];
    __shared__ double red[NT / kWave];
    constexpr int LCAP = (TILE + EXT) / kLongRow;
    __shared__ int32_t longq[LCAP];
    __shared__ int nlong;
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t_lo = g * per, t_hi = min(ntiles, t_lo + per);
    for (int64_t tile = t_lo; tile < t_hi; ++tile) {
        const int64_t k0 = tile * TILE;
        const int32_t n = (int32_t)min((int64_t)TILE, nnz - k0);
        const int32_t r_lo = tile_row[tile], r_hi = tile_row[tile + 1];
        const int32_t info = tile_info[tile];
        const int32_t nr = r_hi - r_lo; // at most RM (checked by the plan)
        const int32_t n_ext = info & 0xffff;
        const bool head_carry = info & kCsrHeadCarry;
        const bool last_carry = info & kCsrLastCarry;
        const int32_t lim = n + n_ext; // local end of the entries loaded
        const int32_t prev_row = k0 > 0 ? ai[k0 - 1] : -1;
        const bool ext_wave = (tid & ~(kWave - 1)) < n_ext; // uniform per wave
        {
            // matrix loads unconditional (clamped indices) so they issue back to back
            const int32_t *__restrict__ aib = ai + k0;
            const int32_t *__restrict__ ajb = aj + k0;
            const T *__restrict__ avb = av + k0;
            int32_t row[IPT], col[IPT + 1];
            T val[IPT + 1], xv[IPT + 1];
#pragma unroll
            for (int e = 0; e < IPT; ++e) col[e] = ld_stream(&ajb[(uint32_t)min(e * NT + tid, n - 1)]);
            const uint32_t ke = (uint32_t)(n + min(tid, max(n_ext - 1, 0)));
            col[IPT] = ext_wave ? ld_stream(&ajb[ke]) : 0;
#pragma unroll
            for (int e = 0; e < IPT; ++e) val[e] = ld_stream(&avb[(uint32_t)min(e * NT + tid, n - 1)]);
            val[IPT] = ext_wave ? ld_stream(&avb[ke]) : T(0);
#pragma unroll
            for (int e = 0; e < IPT; ++e) row[e] = ld_stream(&aib[(uint32_t)min(e * NT + tid, n - 1)]);
#pragma unroll
            for (int e = 0; e < IPT; ++e) xv[e] = x[(uint32_t)col[e]];
            xv[IPT] = ext_wave ? x[(uint32_t)col[IPT]] : T(0);
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                const int j = e * NT + tid;
                if (j < n) {
                    prod[j] = val[e] * xv[e];
                    srow[j] = row[e];
                }
            }
            if (tid < n_ext) prod[n + tid] = val[IPT] * xv[IPT];
        }
        // owned rows without a start in the tile are the empty rows at the end
        for (int q = tid; q <= nr; q += NT) lrp[q] = lim;
        if (tid == 0) nlong = 0;
        __syncthreads();
        for (int j = tid; j < n; j += NT) {
            const int32_t R = srow[j];
            const int32_t P = j == 0 ? prev_row : srow[j - 1];
            if (R != P) {
                const int32_t q_hi = min(R, r_hi - 1);
                for (int32_t q = max(P + 1, r_lo); q <= q_hi; ++q) lrp[q - r_lo] = j;
            }
        }
        __syncthreads();
        if (head_carry) {
            // piece of a long row that began in an earlier tile
            const int32_t hl = min(lrp[0], n);
            T hs = T(0);
            for (int j = tid; j < hl; j += NT) hs += prod[j];
            const double tot = block_sum<NT>((double)hs, red);
            if (tid == 0) carry[2 * tile] = (T)tot;
        }
        reduce_tile_rows<T, NT, LCAP>(
            nr, (info & kCsrLongRows) != 0, longq, &nlong, [&](int r) { return lrp[r]; },
            [&](int r) { return min(lrp[r + 1], lim); },
            [&](int b, int e, int lane, int G) {
                T sum = T(0);
                for (int k = b + lane; k < e; k += G) sum += prod[k];
                return sum;
            },
            [&](int r, T sum) {
                if (last_carry && r == nr - 1) carry[2 * tile + 1] = sum;
                else y[r_lo + r] = acc ? y[r_lo + r] + sum : sum;
            });
        __syncthreads();
    }
}

// Rows longer than their owner's window: the owner's tail piece plus the head
// pieces of the following tiles, in tile order, while the row continues.
template <typename T>
__global__ void coo_rows_fixup_kernel(const int32_t *__restrict__ ai,
                                      const int32_t *__restrict__ tile_row,
                                      const int32_t *__restrict__ tile_info,
                                      const T *__restrict__ carry, T *__restrict__ y, int64_t nnz,
                                      int64_t ntiles, int tile, const int *__restrict__ done, int acc)
{
    if (done && *done) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles || !(tile_info[t] & kCsrLastCarry)) return;
    const int32_t r = tile_row[t + 1] - 1;
    T v = carry[2 * t + 1];
    for (int64_t u = t + 1; u < ntiles; ++u) {
        v += carry[2 * u];
        const int64_t ue = (u + 1) * (int64_t)tile; // first entry after tile u
        if (ue >= nnz || ai[ue] != r) break;
    }
    y[r] = acc ? y[r] + v : v;
}

// Adds the pieces of rows that span tiles, in tile order.  The owner of such
// a row is the tile holding its first entry.
template <typename T>
__global__ void coo_fixup_kernel(int64_t nnz, const int32_t *__restrict__ ai,
                                 const T *__restrict__ carry, T *__restrict__ y, int64_t ntiles,
                                 int32_t TILE, const int *__restrict__ done, int acc)
{
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
    y[last] = acc ? y[last] + v : v;
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ p, T v, int64_t n, const int *__restrict__ done)
{
    if (done && *done) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// p.Ap for COO (whose kernel has no per-row epilogue) and for the timed CG.
template <typename T>
__global__ __launch_bounds__(256) void dot_partials_kernel(int64_t n, const T *__restrict__ a,
                                                           const T *__restrict__ b,
                                                           const int *__restrict__ done,
                                                           double *__restrict__ partials)
{
    constexpr int NT = 256;
    __shared__ double red[NT / kWave];
    if (done && *done) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        s += (double)a[i] * (double)b[i];
    const double bs = block_sum<NT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// alpha = rho / (p.Ap) from the partials of the kernel that ran before.
__global__ __launch_bounds__(kFinNT) void sigma_finish_kernel(const double *__restrict__ partials,
                                                              int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (st->done) return;
    const double tot = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) cg_finish_sigma(st, tot);
}

// ===========================================================================
// Launch configuration and plans
// ===========================================================================
constexpr int64_t kDotGridMax = 2048; // workgroups of the plain p.Ap kernel

static int64_t dia_blocks(const mxs_mat_s *A)
{
    const int64_t rows = (int64_t)kDiaNT * (A->dtype == MXS_F64 ? DiaCfg<double>::RPT
                                                                 : DiaCfg<float>::RPT);
    return (A->nrows + rows - 1) / rows;
}

// Entries per thread of a CSR matrix's tiles: CsrCfg's (10) while a tile
// would own at most RMAX rows on average (the LDS-staged path; 127.2 us
// against 129.4 us with 8 on the 128^3 stencil); MXS_CSR_IPT_SPARSE (4)
// past 2 RMAX rows, rows of fewer than five entries (the 4M-row Zipf
// matrix's 6 column blocks, 2.7 entries per row: 649 against 679 us with 8;
// 0.5 random entries per row on 800,000 rows 13.9 against 19.2 us; 3 per
// row near the diagonal 50.6 against 52.4 us); MXS_CSR_IPT_MANY (8) between
// (6 per row near the diagonal: 88.8 against 94.0 us with 4).
static int csr_plan_ipt(const mxs_mat_s *A)
{
    const int wide = A->dtype == MXS_F64 ? CsrCfg<double>::IPT : CsrCfg<float>::IPT;
    const double rows_per_tile = (double)A->nrows * (CsrCfg<double>::NT * wide) /
                                 (double)std::max<int64_t>(A->nnz, 1);
    if (rows_per_tile <= CsrCfg<double>::RMAX) return wide;
    return rows_per_tile <= 2 * CsrCfg<double>::RMAX ? MXS_CSR_IPT_MANY : MXS_CSR_IPT_SPARSE;
}
static int coo_tile(mxs_dtype t) { return t == MXS_F64 ? CooCfg<double>::TILE : CooCfg<float>::TILE; }

// One workgroup per block/tile.  A fused dot writes one partial per
// workgroup, so its grid is capped (each workgroup then takes a contiguous
// run of blocks) to leave room for the fix-up partials.
template <typename T>
static void spmv_grid(const mxs_mat_s *A, bool dot, uint32_t *grid, int64_t *per)
{
    const int64_t nblk = A->fmt == MXS_CSR ? A->csr.ntiles
                         : A->fmt == MXS_DIA ? dia_blocks(A) : A->coo.ntiles;
#if MXS_PERSIST
    int64_t cap = A->fmt == MXS_CSR ? resident_workgroups(csr_spmv_kernel<T, false, false, CsrCfg<T>::IPT>, 256)
                  : A->fmt == MXS_DIA ? resident_workgroups(dia_spmv_kernel<T, false>, kDiaNT)
                                      : resident_workgroups(coo_spmv_kernel<T, kCooIPT>, kCooNT);
#else
    int64_t cap = INT64_MAX / 2;
#endif
    if (dot) cap = std::min<int64_t>(cap, kMaxParts / 2);
    persistent_grid(nblk, cap, grid, per);
}

static uint32_t fixup_grid(int64_t ntiles) { return (uint32_t)std::max<int64_t>(1, (ntiles + 255) / 256); }

int64_t spmv_dot_parts(const mxs_mat_s *A)
{
    if (A->fmt == MXS_COO || is_split(A) || (A->fmt == MXS_CSR && (A->colblk || A->csr.vec)))
        return kDotGridMax;
    if (A->fmt == MXS_CSR && A->csr.ell) return ell_grid(A->nrows, true);
    if (A->fmt == MXS_CSR && A->csr.rowwise) return rowwise_grid(A->nrows);
    if (A->fmt == MXS_ELL || A->fmt == MXS_SELL) return padded_grid(A, true);
    uint32_t grid;
    int64_t per;
    if (A->dtype == MXS_F64) spmv_grid<double>(A, true, &grid, &per);
    else spmv_grid<float>(A, true, &grid, &per);
    int64_t n = grid;
    if (A->fmt == MXS_CSR && A->csr.fixup) n += fixup_grid(A->csr.ntiles);
    return n;
}

// CSR plan: the entry tiles (first owned row and flags per tile) and the
// carries mxs_spmv uses; the ELL copy when rows have near-equal lengths (at
// most 5% padding; not for parts, nor with MXS_PLAN_NO_ELL); the column
// blocks (colblk.hip).
static mxs_status csr_plan(mxs_mat_s *A, PlanCtx &c, hipStream_t s)
{
    const int tile = CsrCfg<double>::NT * csr_plan_ipt(A);
    const int64_t nt = (A->nnz + tile - 1) / tile;
    CsrPlan P{};
    P.ntiles = nt;
    P.tile = tile;
    if (nt == 0) {
        if (c.build) A->csr = P;
        return MXS_OK;
    }
    // default: a thread per row when rows outnumber entries two to one
    P.rowwise = (int64_t)A->nrows > 2 * A->nnz;
    // tile_row [nt+1], tile_info [nt]
    int32_t *buf = (int32_t *)c.keep(sizeof(int32_t) * (2 * (size_t)nt + 1));
    void *carry = c.keep(2 * (size_t)nt * dsize(A->dtype));
    int *flag = (int *)c.counters();
    if (!flag) return MXS_ERR_INVALID_ARG; // no room for the measurement
    if (c.build) {
        int32_t *tile_row = buf, *info = buf + nt + 1;
        mxs_status st = fill_i32(flag, 0, 1, s);
        if (st != MXS_OK) return st;
        const uint32_t g = (uint32_t)((nt + 1 + 255) / 256);
        const int ext = A->dtype == MXS_F64 ? CsrCfg<double>::EXT : CsrCfg<float>::EXT;
        csr_tile_rows_kernel<<<g, 256, 0, s>>>(A->idx0, A->nrows, nt, tile, tile_row);
        csr_tile_info_kernel<<<g, 256, 0, s>>>(A->idx0, tile_row, A->nnz, nt, tile, ext, info, flag);
        if (A->nrows > 0)
            csr_long_rows_kernel<<<(uint32_t)(((int64_t)A->nrows + 255) / 256), 256, 0, s>>>(
                A->idx0, A->nrows, tile, info);
        MXS_HIP(hipGetLastError());
        int any = 0;
        MXS_HIP(hipMemcpyAsync(&any, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        P.tile_row = tile_row;
        P.tile_info = info;
        P.fixup = any != 0;
        P.carry = carry;
    }
    // ELL copy for rows of near-equal length: lanes of a wave then hold
    // neighbouring rows, and their gathers of x neighbouring addresses
    if (!A->sub && !(c.opts & MXS_PLAN_NO_ELL)) {
        int32_t K = 0;
        mxs_status st = longest_row_with(A->nrows, A->idx0, flag, &K, s);
        if (st != MXS_OK) return st;
        if (K > 0 && (double)K * A->nrows <= 1.05 * (double)A->nnz) {
            const size_t slots = (size_t)K * A->nrows;
            int32_t *col = (int32_t *)c.keep(slots * sizeof(int32_t));
            void *val = c.keep(slots * dsize(A->dtype));
            if (c.build) {
                st = ell_build(A, K, col, val, s);
                if (st != MXS_OK) return st;
                P.ell_k = K;
                P.ell_col = col;
                P.ell_val = val;
            }
        }
    }
    if (c.build) A->csr = P;
    // column blocks for scattered columns over a large x
    return colblk_plan(A, A->idx0, c, s);
}

// Row-blocked copy: out[(b*nd + d)*R + r] = av[d*nrows + b*R + r] (0 past the last row).
template <typename T>
__global__ void dia_block_copy_kernel(const T *__restrict__ av, int32_t nrows, int32_t nd, int R,
                                      int64_t elems, T *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / ((int64_t)nd * R);
        const int64_t rem = e - b * (int64_t)nd * R;
        const int64_t d = rem / R, r = rem - d * R;
        const int64_t row = b * R + r;
        out[e] = row < nrows ? av[d * nrows + row] : T(0);
    }
}

// DIA plan: the x windows of interior blocks (see dia_spmv_kernel) and,
// with MXS_PLAN_DIA_BLOCKED, a row-blocked copy of the values.
static mxs_status dia_plan(mxs_mat_s *A, PlanCtx &c, hipStream_t s)
{
    DiaPlan P{};
    const int nd = A->ndiag;
    if (nd == 0 || A->nrows == 0) {
        if (c.build) A->dia = P;
        return MXS_OK;
    }
    std::vector<int32_t> off(nd);
    MXS_HIP(hipMemcpyAsync(off.data(), A->idx0, sizeof(int32_t) * nd, hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    P.first_off = off[0];
    P.last_off = off[nd - 1];
    bool tri = nd % 3 == 0;
    for (int t = 0; tri && t < nd / 3; ++t)
        tri = off[3 * t + 1] == off[3 * t] + 1 && off[3 * t + 2] == off[3 * t] + 2;
    P.triples = tri ? 1 : 0;
    const int R = kDiaNT * (A->dtype == MXS_F64 ? DiaCfg<double>::RPT : DiaCfg<float>::RPT);
    std::vector<int32_t> runs, pos(nd);
    int64_t total = 0;
    int d0 = 0;
    for (int d = 1; d <= nd; ++d) {
        if (d == nd || (int64_t)off[d] - off[d - 1] > R) {
            const int64_t len = (int64_t)off[d - 1] - off[d0] + R;
            for (int q = d0; q < d; ++q) pos[q] = (int32_t)(total + off[q] - off[d0]);
            runs.push_back(off[d0]);
            runs.push_back((int32_t)len);
            runs.push_back((int32_t)total);
            total += len;
            d0 = d;
        }
    }
    // the row-blocked copy, on request, when its padding stays small
    if ((c.opts & MXS_PLAN_DIA_BLOCKED) && dia_blocks(A) * R <= (int64_t)A->nrows + A->nrows / 8) {
        const int64_t nb = dia_blocks(A);
        const size_t elems = (size_t)nb * nd * R;
        void *blk = c.keep(elems * dsize(A->dtype));
        if (c.build) {
            const uint32_t g = (uint32_t)std::min<int64_t>(((int64_t)elems + 255) / 256, 65536);
            if (A->dtype == MXS_F64)
                dia_block_copy_kernel<double><<<g, 256, 0, s>>>((const double *)A->vals, A->nrows, nd, R,
                                                                (int64_t)elems, (double *)blk);
            else
                dia_block_copy_kernel<float><<<g, 256, 0, s>>>((const float *)A->vals, A->nrows, nd, R,
                                                               (int64_t)elems, (float *)blk);
            MXS_HIP(hipGetLastError());
            P.blk = blk;
        }
    }
    const int64_t nruns = (int64_t)runs.size() / 3;
    // windows only when they fit and save at least a quarter of the x loads
    const bool use = MXS_DIA_WIN && nd <= kDiaStage && nruns <= kDiaMaxRuns &&
                     total <= kDiaWinMax && 4 * total <= 3 * (int64_t)nd * R;
    if (use) {
        int32_t *dev = (int32_t *)c.keep(sizeof(int32_t) * ((size_t)nd + runs.size()));
        if (c.build) {
            MXS_HIP(hipMemcpyAsync(dev, pos.data(), sizeof(int32_t) * nd, hipMemcpyHostToDevice, s));
            MXS_HIP(hipMemcpyAsync(dev + nd, runs.data(), sizeof(int32_t) * runs.size(),
                                   hipMemcpyHostToDevice, s));
            MXS_HIP(hipStreamSynchronize(s));
            P.pos = dev;
            P.runs = dev + nd;
            P.nruns = (int32_t)nruns;
            P.lds_elems = (int32_t)total;
        }
    }
    if (c.build) A->dia = P;
    return MXS_OK;
}

// Largest number of rows any tile owns.
__global__ void tile_rows_max_kernel(const int32_t *__restrict__ tile_row, int64_t ntiles,
                                     int *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) atomicMax(out, tile_row[t + 1] - tile_row[t]);
}


// COO plan: the CSR tiling derived from the row ids through a temporary row
// pointer array, usable when every tile owns at most kCooRowsMax rows;
// otherwise the segmented-scan tiles.  One carry array serves either.
static mxs_status coo_plan(mxs_mat_s *A, PlanCtx &c, hipStream_t s)
{
    CooPlan P{};
    if (A->nnz == 0) {
        if (c.build) A->coo = P;
        return MXS_OK;
    }
    const int tile = coo_tile(A->dtype);
    const int64_t nt = (A->nnz + tile - 1) / tile;
    // segmented tiles: 4 entries per thread, 1 for a column block, whose
    // gathers of x are scattered by construction (the 4M-row Zipf matrix's
    // 6 COO blocks: 677 against 737 us; 3 entries per row near the diagonal,
    // a matrix for the segmented kernel without blocks, lose with 1: 90.3
    // against 77.1 us)
    const int32_t seg_tile = kCooNT * (A->cblk_part ? MXS_COO_IPT_SCATTER : kCooIPT);
    const int64_t nt_seg = (A->nnz + seg_tile - 1) / seg_tile;
    int32_t *buf = (int32_t *)c.keep(sizeof(int32_t) * (2 * (size_t)nt + 1));
    // carries of either implementation (two values per tile)
    void *carry = c.keep(2 * (size_t)std::max(nt, nt_seg) * dsize(A->dtype));
    int *flags = (int *)c.counters(); // [0] any carry, [1] most rows in a tile
    if (!flags) return MXS_ERR_INVALID_ARG;
    // row pointers of the sorted row ids, for the build only
    const size_t mark = c.mark();
    int32_t *irp = (int32_t *)c.tmp(sizeof(int32_t) * ((size_t)A->nrows + 1));
    if (c.build) {
        int32_t *tile_row = buf, *info = buf + nt + 1;
        mxs_status st = coo_irp_launch(A->nnz, A->nrows, A->idx0, irp, s);
        if (st == MXS_OK) st = fill_i32(flags, 0, 2, s);
        if (st != MXS_OK) return st;
        const uint32_t g = (uint32_t)((nt + 1 + 255) / 256);
        const int ext = A->dtype == MXS_F64 ? CooCfg<double>::EXT : CooCfg<float>::EXT;
        csr_tile_rows_kernel<<<g, 256, 0, s>>>(irp, A->nrows, nt, tile, tile_row);
        csr_tile_info_kernel<<<g, 256, 0, s>>>(irp, tile_row, A->nnz, nt, tile, ext, info, flags);
        if (A->nrows > 0)
            csr_long_rows_kernel<<<(uint32_t)(((int64_t)A->nrows + 255) / 256), 256, 0, s>>>(
                irp, A->nrows, tile, info);
        tile_rows_max_kernel<<<g, 256, 0, s>>>(tile_row, nt, flags + 1);
        MXS_HIP(hipGetLastError());
        int h[2] = {0, 0};
        MXS_HIP(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        P.rows_ok = h[1] <= kCooRowsMax;
        P.tile_row = tile_row;
        P.tile_info = info;
        P.fixup = h[0] != 0;
        P.nt_rows = nt;
        P.nt_seg = nt_seg;
        P.seg_tile = seg_tile;
        P.carry_rows = P.carry_seg = carry;
        A->coo = P;
    }
    // column blocks for scattered columns over a large x (cut with irp)
    const mxs_status st = colblk_plan(A, irp, c, s);
    c.release(mark);
    return st;
}

// ---------------------------------------------------------------------------
// Implementations of each format's SpMV (no single one wins on every matrix):
//   COO 0: row tiles (the CSR tiling rebuilt from the row ids)
//       1: segmented-scan tiles  2: column blocks (colblk.hip)
//   CSR 0: entry tiles           1: a thread per row
//       2: entry tiles, x gathered per row from LDS-staged columns
//       3: a lane per row over an ELL copy made by the plan (rows of
//          near-equal length: at most 5% padding)
//       4: column blocks (colblk.hip)   5: a wavefront per row
//   DIA 0: row-blocked values, x shared over runs of three offsets
//       1: row-blocked values    2: diagonal-major values (no copy), x shared
// ---------------------------------------------------------------------------
int32_t impl_count(const mxs_mat_s *A)
{
    if (A->fmt == MXS_ELL || A->fmt == MXS_SELL) return 1;
    return A->fmt == MXS_CSR ? 6 : A->fmt == MXS_DIA ? 3 : A->fmt == MXS_COO ? 3 : 0;
}

bool impl_ok(const mxs_mat_s *A, int32_t impl)
{
    if (impl < 0 || impl >= impl_count(A)) return false;
    if (A->nnz == 0) return true;
    switch (A->fmt) {
    case MXS_COO: return impl == 2 ? !A->cblk.empty() : impl == 1 || A->coo.rows_ok;
    case MXS_CSR: return impl == 3 ? A->csr.ell_col != nullptr : impl == 4 ? !A->cblk.empty() : true;
    case MXS_DIA:
        if (impl == 0) return A->dia.blk != nullptr && A->dia.triples;
        if (impl == 1) return A->dia.blk != nullptr;
        return true;
    case MXS_ELL:
    case MXS_SELL: return true;
    default: return false;
    }
}

static int32_t default_impl(const mxs_mat_s *A)
{
    switch (A->fmt) {
    case MXS_COO: return !A->cblk.empty() ? 2 : impl_ok(A, 0) ? 0 : 1;
    case MXS_CSR:
        return !A->cblk.empty() ? 4 : A->csr.ell_col ? 3 : A->csr.rowwise ? 1 : MXS_CSR_GX_DEFAULT ? 2 : 0;
    case MXS_DIA: return impl_ok(A, 0) ? 0 : impl_ok(A, 1) ? 1 : 2;
    case MXS_ELL:
    case MXS_SELL: return 0;
    default: return -1;
    }
}

void set_impl(mxs_mat_s *A, int32_t impl)
{
    A->impl = impl;
    switch (A->fmt) {
    case MXS_COO:
        A->coo.rows = impl == 0 && A->coo.rows_ok;
        A->coo.ntiles = A->coo.rows ? A->coo.nt_rows : A->coo.nt_seg;
        A->coo.carry = A->coo.rows ? A->coo.carry_rows : A->coo.carry_seg;
        A->colblk = impl == 2 && !A->cblk.empty();
        break;
    case MXS_CSR:
        A->csr.rowwise = impl == 1;
        A->csr.gx = impl == 2;
        A->csr.ell = impl == 3;
        A->colblk = impl == 4 && !A->cblk.empty();
        A->csr.vec = impl == 5;
        break;
    case MXS_DIA:
        A->dia.use_blk = impl != 2 && A->dia.blk != nullptr;
        A->dia.use_share = impl != 1 && A->dia.triples;
        break;
    default: break;
    }
}

mxs_status tune(mxs_mat_s *A, const void *x, void *y, int32_t reps, int32_t *impl_out,
                double *ms, hipStream_t s)
{
    const int32_t n = impl_count(A);
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto &e : ev) MXS_HIP(hipEventCreate(&e));
    auto destroy = [&] {
        for (auto e : ev) (void)hipEventDestroy(e);
    };
    int32_t best = -1;
    double best_ms = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (ms) ms[i] = -1.0;
        if (!impl_ok(A, i)) continue;
        set_impl(A, i);
        mxs_status st = MXS_OK;
        for (int w = 0; w < 3 && st == MXS_OK; ++w) st = spmv_launch(A, x, y, nullptr, nullptr, s);
        for (int r = 0; r < reps && st == MXS_OK; ++r) {
            if (hipEventRecord(ev[2 * r], s) != hipSuccess) st = MXS_ERR_HIP;
            if (st == MXS_OK) st = spmv_launch(A, x, y, nullptr, nullptr, s);
            if (st == MXS_OK && hipEventRecord(ev[2 * r + 1], s) != hipSuccess) st = MXS_ERR_HIP;
        }
        if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
        std::vector<float> t((size_t)reps);
        for (int r = 0; r < reps && st == MXS_OK; ++r)
            if (hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]) != hipSuccess) st = MXS_ERR_HIP;
        if (st != MXS_OK) {
            destroy();
            return st;
        }
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        const double med = t[reps / 2];
        if (ms) ms[i] = med;
        if (best < 0 || med < best_ms) {
            best = i;
            best_ms = med;
        }
    }
    destroy();
    set_impl(A, best);
    if (impl_out) *impl_out = best;
    return MXS_OK;
}

mxs_status plan_walk(mxs_mat_s *A, PlanCtx &c, hipStream_t s)
{
    mxs_status st = MXS_OK;
    if (is_split(A)) {
        st = plan_walk(A->band, c, s);
        if (st == MXS_OK) st = plan_walk(A->rest, c, s);
    } else if (A->fmt == MXS_CSR) {
        st = csr_plan(A, c, s);
    } else if (A->fmt == MXS_DIA) {
        st = dia_plan(A, c, s);
    } else if (A->fmt == MXS_COO) {
        st = coo_plan(A, c, s);
    }
    if (st == MXS_OK && c.build) {
        if (!is_split(A)) set_impl(A, default_impl(A));
        A->plan_opts = c.opts;
        A->optimized = true;
    }
    return st;
}

void plan_reset(mxs_mat_s *A)
{
    if (!A) return;
    plan_reset(A->band);
    plan_reset(A->rest);
    for (mxs_mat_s *B : A->cblk) release(B);
    A->cblk.clear();
    A->colblk = false;
    A->csr = CsrPlan{};
    A->coo = CooPlan{};
    A->dia = DiaPlan{};
    A->optimized = false;
    A->impl = -1;
    A->plan_opts = 0;
}

size_t spmv_scratch_bytes(const mxs_mat_s *A)
{
    if (is_split(A)) return spmv_scratch_bytes(A->rest); // the band (DIA, ELL) has no carries
    size_t b = 0;
    if (A->fmt == MXS_CSR) b = 2 * (size_t)A->csr.ntiles * dsize(A->dtype);
    if (A->fmt == MXS_COO) b = 2 * (size_t)std::max(A->coo.nt_rows, A->coo.nt_seg) * dsize(A->dtype);
    // column blocks run one after the other on one stream: one region serves all
    for (const mxs_mat_s *B : A->cblk) b = std::max(b, spmv_scratch_bytes(B));
    return b;
}

template <typename T>
static mxs_status dot_sigma_typed(int64_t n, const T *a, const T *b, const int *done,
                                  const DotSink *dot, hipStream_t s)
{
    const uint32_t g = (uint32_t)std::clamp<int64_t>((n + 1023) / 1024, 1, kDotGridMax);
    dot_partials_kernel<T><<<g, 256, 0, s>>>(n, a, b, done, dot->partials);
    MXS_HIP(hipGetLastError());
    sigma_finish_kernel<<<1, kFinNT, 0, s>>>(dot->partials, g, dot->st);
    return launch_status();
}

mxs_status dot_sigma_launch(int64_t n, mxs_dtype t, const void *a, const void *b, const int *done,
                            const DotSink *dot, hipStream_t s)
{
    if (t == MXS_F64)
        return dot_sigma_typed<double>(n, (const double *)a, (const double *)b, done, dot, s);
    return dot_sigma_typed<float>(n, (const float *)a, (const float *)b, done, dot, s);
}

template <typename T>
static mxs_status spmv_typed(const mxs_mat_s *A, const T *x, T *y, const int *done,
                             const DotSink *dot, hipStream_t s, int acc, void *carry)
{
    if (A->nrows == 0) return MXS_OK;
    uint32_t grid = 0;
    int64_t per = 1;
    double *parts = dot ? dot->partials : nullptr;
    int64_t nparts = 0;
    const uint32_t fill_g = (uint32_t)std::min<int64_t>((A->nrows + 255) / 256, 4096);
    if (A->colblk) {
        // column blocks: the first writes y (unless accumulating), the rest add to it
        for (size_t b = 0; b < A->cblk.size(); ++b) {
            const mxs_status st =
                spmv_typed<T>(A->cblk[b], x, y, done, nullptr, s, acc || b > 0 ? 1 : 0, carry);
            if (st != MXS_OK) return st;
        }
        if (dot) return dot_sigma_typed<T>(A->nrows, x, y, done, dot, s);
        return MXS_OK;
    }
    switch (A->fmt) {
    case MXS_CSR: {
        const int64_t nt = A->csr.ntiles;
        if (nt == 0) {
            if (!acc) fill_kernel<T><<<fill_g, 256, 0, s>>>(y, T(0), A->nrows, done);
            MXS_HIP(hipGetLastError());
            if (dot) return dot_sigma_typed<T>(A->nrows, x, y, done, dot, s);
            return MXS_OK;
        }
        if (A->csr.ell && !acc) {
            mxs_status st = ell_launch(A->nrows, A->csr.ell_k, A->csr.ell_col, A->csr.ell_val, A->dtype,
                                       x, y, done, parts, s);
            if (st != MXS_OK) return st;
            nparts = ell_grid(A->nrows, dot != nullptr);
            break;
        }
        if (A->csr.vec) {
            csr_vector_kernel<T><<<vector_grid(A->nrows), 256, 0, s>>>(
                A->idx0, A->idx1, (const T *)A->vals, x, y, A->nrows, done, acc);
            MXS_HIP(hipGetLastError());
            if (dot) return dot_sigma_typed<T>(A->nrows, x, y, done, dot, s);
            return MXS_OK;
        }
        if (A->csr.rowwise) {
            grid = rowwise_grid(A->nrows);
            if (dot)
                csr_rowwise_kernel<T, true><<<grid, 256, 0, s>>>(A->idx0, A->idx1, (const T *)A->vals,
                                                                 x, y, A->nrows, done, parts, acc);
            else
                csr_rowwise_kernel<T, false><<<grid, 256, 0, s>>>(A->idx0, A->idx1,
                                                                  (const T *)A->vals, x, y, A->nrows,
                                                                  done, nullptr, acc);
            MXS_HIP(hipGetLastError());
            nparts = grid;
            break;
        }
        spmv_grid<T>(A, dot != nullptr, &grid, &per);
        const int32_t *tr = A->csr.tile_row, *ti = A->csr.tile_info;
        T *cr = (T *)(carry ? carry : A->csr.carry);
        constexpr int W = CsrCfg<T>::IPT, M = MXS_CSR_IPT_MANY, P = MXS_CSR_IPT_SPARSE;
        const int ipt = A->csr.tile / CsrCfg<T>::NT;
        auto kern = ipt == W ? (dot ? (A->csr.gx ? csr_spmv_kernel<T, true, true, W> : csr_spmv_kernel<T, true, false, W>)
                                    : (A->csr.gx ? csr_spmv_kernel<T, false, true, W> : csr_spmv_kernel<T, false, false, W>))
                  : ipt == M ? (dot ? (A->csr.gx ? csr_spmv_kernel<T, true, true, M> : csr_spmv_kernel<T, true, false, M>)
                                    : (A->csr.gx ? csr_spmv_kernel<T, false, true, M> : csr_spmv_kernel<T, false, false, M>))
                             : (dot ? (A->csr.gx ? csr_spmv_kernel<T, true, true, P> : csr_spmv_kernel<T, true, false, P>)
                                    : (A->csr.gx ? csr_spmv_kernel<T, false, true, P> : csr_spmv_kernel<T, false, false, P>));
        kern<<<grid, 256, 0, s>>>(A->idx0, A->idx1, (const T *)A->vals, x, y, tr, ti, A->nnz, nt, per,
                                  cr, done, dot ? parts : nullptr, acc);
        MXS_HIP(hipGetLastError());
        nparts = grid;
        if (A->csr.fixup) {
            const uint32_t fg = fixup_grid(nt);
            if (dot)
                csr_fixup_kernel<T, true><<<fg, 256, 0, s>>>(A->idx0, tr, ti, cr,
                                                             x, y, A->nnz, nt, A->csr.tile,
                                                             done, parts + grid, acc);
            else
                csr_fixup_kernel<T, false><<<fg, 256, 0, s>>>(A->idx0, tr, ti, cr,
                                                              x, y, A->nnz, nt, A->csr.tile,
                                                              done, nullptr, acc);
            MXS_HIP(hipGetLastError());
            nparts += fg;
        }
        break;
    }
    case MXS_DIA: {
        spmv_grid<T>(A, dot != nullptr, &grid, &per);
        const DiaPlan &P = A->dia;
        const size_t lds = sizeof(T) * (size_t)P.lds_elems;
        const T *vals = P.use_blk ? (const T *)P.blk : (const T *)A->vals;
        const int blocked = P.use_blk ? 1 : 0;
        const int32_t share = P.use_share ? 1 : 0;
        if (dot)
            dia_spmv_kernel<T, true><<<grid, kDiaNT, lds, s>>>(
                A->nrows, A->ncols, A->ndiag, A->idx0, vals, blocked, x, y, dia_blocks(A), per,
                done, parts, P.pos, P.runs, P.nruns, P.lds_elems, P.first_off, P.last_off, share);
        else
            dia_spmv_kernel<T, false><<<grid, kDiaNT, lds, s>>>(
                A->nrows, A->ncols, A->ndiag, A->idx0, vals, blocked, x, y, dia_blocks(A), per,
                done, parts, P.pos, P.runs, P.nruns, P.lds_elems, P.first_off, P.last_off, share);
        MXS_HIP(hipGetLastError());
        nparts = grid;
        break;
    }
    case MXS_COO: {
        const int64_t nt = A->coo.ntiles;
        if (nt == 0) {
            if (!acc) fill_kernel<T><<<fill_g, 256, 0, s>>>(y, T(0), A->nrows, done);
        } else {
            spmv_grid<T>(A, false, &grid, &per);
            T *cr = (T *)(carry ? carry : A->coo.carry);
            if (A->coo.rows) {
                coo_rows_kernel<T><<<grid, 256, 0, s>>>(A->idx0, A->idx1, (const T *)A->vals, x, y,
                                                        A->coo.tile_row, A->coo.tile_info, A->nnz,
                                                        nt, per, cr, done, acc);
                MXS_HIP(hipGetLastError());
                if (A->coo.fixup)
                    coo_rows_fixup_kernel<T><<<(uint32_t)((nt + 255) / 256), 256, 0, s>>>(
                        A->idx0, A->coo.tile_row, A->coo.tile_info, cr, y,
                        A->nnz, nt, coo_tile(A->dtype), done, acc);
            } else {
                auto kern = A->coo.seg_tile == kCooNT * kCooIPT ? coo_spmv_kernel<T, kCooIPT>
                                                                : coo_spmv_kernel<T, MXS_COO_IPT_SCATTER>;
                kern<<<grid, kCooNT, 0, s>>>(A->nnz, A->nrows, A->idx0, A->idx1, (const T *)A->vals,
                                             x, y, cr, nt, per, done, acc);
                MXS_HIP(hipGetLastError());
                coo_fixup_kernel<T><<<(uint32_t)((nt + 255) / 256), 256, 0, s>>>(
                    A->nnz, A->idx0, cr, y, nt, A->coo.seg_tile, done, acc);
            }
        }
        MXS_HIP(hipGetLastError());
        if (dot) return dot_sigma_typed<T>(A->nrows, x, y, done, dot, s);
        return MXS_OK;
    }
    case MXS_ELL:
    case MXS_SELL: {
        if (acc) return MXS_ERR_UNSUPPORTED;
        mxs_status st = padded_spmv(A, x, y, done, parts, s);
        if (st != MXS_OK) return st;
        nparts = padded_grid(A, dot != nullptr);
        break;
    }
    default:
        return MXS_ERR_UNSUPPORTED;
    }
    if (dot) {
        sigma_finish_kernel<<<1, kFinNT, 0, s>>>(dot->partials, nparts, dot->st);
        return launch_status();
    }
    return MXS_OK;
}

mxs_status spmv_acc_launch(const mxs_mat_s *A, const void *x, void *y, const int *done,
                           hipStream_t s, void *carry)
{
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    if (A->dtype == MXS_F64)
        return spmv_typed<double>(A, (const double *)x, (double *)y, done, nullptr, s, 1, carry);
    return spmv_typed<float>(A, (const float *)x, (float *)y, done, nullptr, s, 1, carry);
}

mxs_status spmv_launch(const mxs_mat_s *A, const void *x, void *y, const int *done,
                       const DotSink *dot, hipStream_t s, void *carry)
{
    if (is_split(A)) {
        // the band (DIA) or ELL part writes every row; the remainder adds onto it
        mxs_status st = spmv_launch(A->band, x, y, done, nullptr, s, carry);
        if (st == MXS_OK && A->rest->nnz > 0) st = spmv_acc_launch(A->rest, x, y, done, s, carry);
        if (st == MXS_OK && dot) st = dot_sigma_launch(A->nrows, A->dtype, y, x, done, dot, s);
        return st;
    }
    if (A->dtype == MXS_F64)
        return spmv_typed<double>(A, (const double *)x, (double *)y, done, dot, s, 0, carry);
    return spmv_typed<float>(A, (const float *)x, (float *)y, done, dot, s, 0, carry);
}

}  // namespace mxs
