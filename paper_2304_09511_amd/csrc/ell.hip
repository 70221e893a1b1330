// Padded formats named as further work in Section IX: ELL and SELL-C-sigma.
//
// ELL: every row gets K slots (K = the longest row), column-major, slot k of
// row i at k*nrows + i; slots past a row's length hold column -1 and +0.0.
// A thread owns a row: the k-th slots of 64 consecutive rows are one
// contiguous load per wavefront.
//
// SELL-C-sigma (Kreutzer et al., 2014) with C = 64, one wavefront per slice:
// rows sorted by descending length, stably, inside windows of sigma rows;
// slice s of 64 sorted positions is as wide as its longest row and starts
// at cs[s]; slot k of the position in lane l at cs[s] + 64 k + l.  A lane
// owns a position and writes y at the row perm[p].
//
// Conversions only move values (bit-exact), from and to COO/CSR; both
// formats are refused (MXS_ERR_DIA_TOO_SPARSE) when they would store more
// than 8 slots per entry.
#include "common.h"

#include <hipcub/device/device_radix_sort.hpp>

#include <algorithm>
#include <climits>
#include <vector>

namespace mxs {

constexpr int kSellC = 64; // slice height: one wavefront
// slots a lane loads at once in SpMV: 16 in FP64, 8 in FP32 (measured at
// 128^3: FP64 ELL 124.0 us against 125.0 with 8, FP32 76.7 us against 80.0
// with 16)
template <typename T>
constexpr int kPadU = sizeof(T) == 8 ? 16 : 8;

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p)
{
    return __builtin_nontemporal_load(p);
}

static uint32_t grid_of(int64_t n, int64_t cap = 1 << 30)
{
    return (uint32_t)std::clamp<int64_t>((n + 255) / 256, 1, cap);
}

// Row pointers of a COO/CSR source (borrowed for CSR, a temporary for COO).
static mxs_status source_irp(const mxs_mat_s *A, const int32_t **irp, int32_t **tmp, hipStream_t s)
{
    *tmp = nullptr;
    if (A->fmt == MXS_CSR) {
        *irp = A->idx0;
        return MXS_OK;
    }
    MXS_HIP(hipMallocAsync((void **)tmp, sizeof(int32_t) * ((size_t)A->nrows + 1), s));
    mxs_status st = coo_irp_launch(A->nnz, A->nrows, A->idx0, *tmp, s);
    *irp = *tmp;
    return st;
}

__global__ void row_len_max_kernel(int32_t nrows, const int32_t *__restrict__ irp, int *__restrict__ out)
{
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, irp[i + 1] - irp[i]);
    // wave maximum, then one atomic per wave
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

mxs_status longest_row_with(int32_t nrows, const int32_t *irp, int *d, int32_t *K, hipStream_t s)
{
    mxs_status st = fill_bytes0(d, sizeof(int), s);
    if (st == MXS_OK && nrows > 0) {
        row_len_max_kernel<<<grid_of(nrows, 4096), 256, 0, s>>>(nrows, irp, d);
        st = launch_status();
    }
    int h = 0;
    if (st == MXS_OK && hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = MXS_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    *K = h;
    return st;
}

static mxs_status longest_row(int32_t nrows, const int32_t *irp, int32_t *K, hipStream_t s)
{
    int *d = nullptr;
    MXS_HIP(hipMallocAsync((void **)&d, sizeof(int), s));
    const mxs_status st = longest_row_with(nrows, irp, d, K, s);
    (void)hipFreeAsync(d, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) return MXS_ERR_HIP;
    return st;
}

// ---------------------------------------------------------------------------
// ELL
// ---------------------------------------------------------------------------
template <typename T>
__global__ void ell_fill_kernel(int32_t nrows, int32_t K, const int32_t *__restrict__ irp,
                                const int32_t *__restrict__ aj, const T *__restrict__ av,
                                int32_t *__restrict__ col, T *__restrict__ val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = irp[i], len = irp[i + 1] - b;
        for (int32_t k = 0; k < K; ++k) {
            const int64_t q = (int64_t)k * nrows + i;
            col[q] = k < len ? aj[b + k] : -1;
            val[q] = k < len ? av[b + k] : T(0);
        }
    }
}

mxs_status ell_width(const mxs_mat_s *A, int32_t *K, hipStream_t s)
{
    const int32_t *irp;
    int32_t *tmp;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    if (st == MXS_OK) st = longest_row(A->nrows, irp, K, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    if (st == MXS_OK && (int64_t)*K * A->nrows > 8 * A->nnz) st = MXS_ERR_DIA_TOO_SPARSE;
    return st;
}

mxs_status ell_build(const mxs_mat_s *A, int32_t K, int32_t *col, void *vals, hipStream_t s)
{
    if (K == 0 || A->nrows == 0) return MXS_OK;
    const int32_t *irp;
    int32_t *tmp;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    if (st == MXS_OK) {
        if (A->dtype == MXS_F64)
            ell_fill_kernel<double><<<grid_of(A->nrows, 65536), 256, 0, s>>>(
                A->nrows, K, irp, A->idx1, (const double *)A->vals, col, (double *)vals);
        else
            ell_fill_kernel<float><<<grid_of(A->nrows, 65536), 256, 0, s>>>(
                A->nrows, K, irp, A->idx1, (const float *)A->vals, col, (float *)vals);
        st = launch_status();
    }
    if (tmp) (void)hipFreeAsync(tmp, s);
    return st;
}

// ---------------------------------------------------------------------------
// HYB: each row's first K entries in ELL, the rest in COO
// ---------------------------------------------------------------------------
__global__ void len_hist_kernel(int32_t nrows, const int32_t *__restrict__ irp, int *__restrict__ hist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&hist[irp[i + 1] - irp[i]], 1);
}

__global__ void hyb_rest_count_kernel(int32_t nrows, const int32_t *__restrict__ irp, int32_t K,
                                      int32_t *__restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        cnt[i] = max(irp[i + 1] - irp[i] - K, 0);
}

template <typename T>
__global__ void hyb_rest_fill_kernel(int32_t nrows, const int32_t *__restrict__ irp,
                                     const int32_t *__restrict__ aj, const T *__restrict__ av, int32_t K,
                                     const int32_t *__restrict__ off, int32_t *__restrict__ ri,
                                     int32_t *__restrict__ rj, T *__restrict__ rv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = irp[i], e = irp[i + 1];
        int32_t q = off[i];
        for (int32_t k = b + K; k < e; ++k, ++q) {
            ri[q] = (int32_t)i;
            rj[q] = aj[k];
            rv[q] = av[k];
        }
    }
}

mxs_status hyb_size(const mxs_mat_s *A, int32_t *K, int64_t *rest, hipStream_t s)
{
    const int32_t n = A->nrows;
    const int32_t *irp;
    int32_t *tmp;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    int32_t maxlen = 0;
    if (st == MXS_OK) st = longest_row(n, irp, &maxlen, s);
    if (st == MXS_OK && *K < 0) {
        // width rule: the largest k with at least max(4096, n/3) rows (all
        // rows when fewer) holding k or more entries
        int *hist = nullptr;
        std::vector<int> h((size_t)maxlen + 1, 0);
        if (hipMallocAsync((void **)&hist, sizeof(int) * ((size_t)maxlen + 1), s) != hipSuccess)
            st = MXS_ERR_OUT_OF_MEMORY;
        if (st == MXS_OK) st = fill_bytes0(hist, sizeof(int) * ((size_t)maxlen + 1), s);
        if (st == MXS_OK && n > 0) {
            len_hist_kernel<<<grid_of(n, 4096), 256, 0, s>>>(n, irp, hist);
            st = launch_status();
        }
        if (st == MXS_OK &&
            hipMemcpyAsync(h.data(), hist, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
            st = MXS_ERR_HIP;
        if (hist) (void)hipFreeAsync(hist, s);
        if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
        const int64_t need = std::min<int64_t>(n, std::max<int64_t>(4096, n / 3));
        int64_t ge = 0;
        int32_t k = 0;
        for (int32_t l = maxlen; l >= 1 && st == MXS_OK; --l) {
            ge += h[l];
            if (ge >= need && ge > 0) {
                k = l;
                break;
            }
        }
        *K = k;
    }
    int64_t r = 0;
    if (st == MXS_OK && n > 0) {
        // entries past the K-th of their row: sum of max(len - K, 0)
        int32_t *cnt = nullptr, *off = nullptr;
        if (hipMallocAsync((void **)&cnt, sizeof(int32_t) * ((size_t)n + 1) * 2, s) != hipSuccess)
            st = MXS_ERR_OUT_OF_MEMORY;
        off = cnt ? cnt + n + 1 : nullptr;
        if (st == MXS_OK) {
            hyb_rest_count_kernel<<<grid_of(n, 65536), 256, 0, s>>>(n, irp, *K, cnt);
            st = launch_status();
        }
        if (st == MXS_OK) st = scan_i32(cnt, off, n, s);
        int32_t h = 0;
        if (st == MXS_OK && hipMemcpyAsync(&h, off + n, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
            st = MXS_ERR_HIP;
        if (cnt) (void)hipFreeAsync(cnt, s);
        if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
        r = h;
    }
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;
    if ((int64_t)*K * n > 8 * A->nnz) return MXS_ERR_DIA_TOO_SPARSE;
    *rest = r;
    return MXS_OK;
}

mxs_status hyb_build(const mxs_mat_s *A, int32_t K, int32_t *ell_col, void *ell_val, int32_t *ri,
                     int32_t *rj, void *rv, hipStream_t s)
{
    const int32_t n = A->nrows;
    if (n == 0) return MXS_OK;
    const int32_t *irp;
    int32_t *tmp;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    if (st == MXS_OK && K > 0) {
        // ell_fill keeps each row's first K entries
        if (A->dtype == MXS_F64)
            ell_fill_kernel<double><<<grid_of(n, 65536), 256, 0, s>>>(n, K, irp, A->idx1,
                                                                      (const double *)A->vals,
                                                                      ell_col, (double *)ell_val);
        else
            ell_fill_kernel<float><<<grid_of(n, 65536), 256, 0, s>>>(n, K, irp, A->idx1,
                                                                     (const float *)A->vals,
                                                                     ell_col, (float *)ell_val);
        st = launch_status();
    }
    int32_t *cnt = nullptr;
    if (st == MXS_OK && hipMallocAsync((void **)&cnt, sizeof(int32_t) * ((size_t)n + 1) * 2, s) != hipSuccess)
        st = MXS_ERR_OUT_OF_MEMORY;
    int32_t *off = cnt ? cnt + n + 1 : nullptr;
    if (st == MXS_OK) {
        hyb_rest_count_kernel<<<grid_of(n, 65536), 256, 0, s>>>(n, irp, K, cnt);
        st = launch_status();
    }
    if (st == MXS_OK) st = scan_i32(cnt, off, n, s);
    if (st == MXS_OK) {
        if (A->dtype == MXS_F64)
            hyb_rest_fill_kernel<double><<<grid_of(n, 65536), 256, 0, s>>>(
                n, irp, A->idx1, (const double *)A->vals, K, off, ri, rj, (double *)rv);
        else
            hyb_rest_fill_kernel<float><<<grid_of(n, 65536), 256, 0, s>>>(
                n, irp, A->idx1, (const float *)A->vals, K, off, ri, rj, (float *)rv);
        st = launch_status();
    }
    if (cnt) (void)hipFreeAsync(cnt, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    return st;
}

// ---------------------------------------------------------------------------
// SELL-C-sigma
// ---------------------------------------------------------------------------
// key of row i: window in the high 32 bits, INT32_MAX - length in the low
// ones, so an ascending stable sort puts windows in order and longer rows
// first, equal lengths in row order.
__global__ void sell_keys_kernel(int32_t nrows, int32_t sigma, const int32_t *__restrict__ irp,
                                 uint64_t *__restrict__ key, int32_t *__restrict__ row)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t w = (uint64_t)(i / sigma);
        key[i] = (w << 32) | (uint64_t)(uint32_t)(INT32_MAX - (irp[i + 1] - irp[i]));
        row[i] = (int32_t)i;
    }
}

__global__ void sell_width_kernel(int32_t nrows, int64_t nslices, const int32_t *__restrict__ irp,
                                  const int32_t *__restrict__ perm, int32_t *__restrict__ width)
{
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslices) return;
    int32_t w = 0;
    const int64_t p1 = min((int64_t)nrows, (sl + 1) * kSellC);
    for (int64_t p = sl * kSellC; p < p1; ++p) w = max(w, irp[perm[p] + 1] - irp[perm[p]]);
    width[sl] = w;
}

__global__ void sell_offsets_kernel(const int32_t *__restrict__ wscan, int64_t nslices,
                                    int64_t *__restrict__ cs)
{
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl <= nslices) cs[sl] = (int64_t)kSellC * wscan[sl];
}

template <typename T>
__global__ void sell_fill_kernel(int32_t nrows, int64_t npos, const int32_t *__restrict__ irp,
                                 const int32_t *__restrict__ aj, const T *__restrict__ av,
                                 const int32_t *__restrict__ perm, const int64_t *__restrict__ cs,
                                 int32_t *__restrict__ col, T *__restrict__ val)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npos;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = p / kSellC, lane = p % kSellC;
        const int64_t base = cs[sl];
        const int32_t w = (int32_t)((cs[sl + 1] - base) / kSellC);
        int32_t b = 0, len = 0;
        if (p < nrows) {
            b = irp[perm[p]];
            len = irp[perm[p] + 1] - b;
        }
        for (int32_t k = 0; k < w; ++k) {
            const int64_t q = base + (int64_t)k * kSellC + lane;
            col[q] = k < len ? aj[b + k] : -1;
            val[q] = k < len ? av[b + k] : T(0);
        }
    }
}

// perm, and the slice widths' prefix sum scaled into cs (both caller
// arrays; cs has nslices + 1 entries).
static mxs_status sell_layout(const mxs_mat_s *A, const int32_t *irp, int32_t sigma, int32_t *perm,
                              int64_t *cs, hipStream_t s)
{
    const int32_t n = A->nrows;
    const int64_t ns = ((int64_t)n + kSellC - 1) / kSellC;
    mxs_status st = MXS_OK;
    if (n > 0) {
        uint64_t *key = nullptr, *key2 = nullptr;
        int32_t *row = nullptr;
        void *tmp = nullptr;
        size_t tb = 0;
        MXS_HIP(hipMallocAsync((void **)&key, sizeof(uint64_t) * (size_t)n * 2, s));
        MXS_HIP(hipMallocAsync((void **)&row, sizeof(int32_t) * (size_t)n, s));
        key2 = key + n;
        sell_keys_kernel<<<grid_of(n, 65536), 256, 0, s>>>(n, sigma, irp, key, row);
        st = launch_status();
        int wbits = 0;
        while (wbits < 31 && (((int64_t)n - 1) / sigma) >> wbits) ++wbits;
        const int end_bit = 32 + wbits;
        if (st == MXS_OK &&
            hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key2, row, perm, n, 0, end_bit, s) != hipSuccess)
            st = MXS_ERR_HIP;
        if (st == MXS_OK && hipMallocAsync(&tmp, std::max<size_t>(tb, 1), s) != hipSuccess) st = MXS_ERR_OUT_OF_MEMORY;
        if (st == MXS_OK &&
            hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key2, row, perm, n, 0, end_bit, s) != hipSuccess)
            st = MXS_ERR_HIP;
        if (tmp) (void)hipFreeAsync(tmp, s);
        (void)hipFreeAsync(key, s);
        (void)hipFreeAsync(row, s);
        if (st != MXS_OK) return st;
    }
    int32_t *width = nullptr, *wscan = nullptr;
    MXS_HIP(hipMallocAsync((void **)&width, sizeof(int32_t) * ((size_t)ns + 1) * 2, s));
    wscan = width + ns + 1;
    if (ns > 0) {
        sell_width_kernel<<<grid_of(ns), 256, 0, s>>>(n, ns, irp, perm, width);
        st = launch_status();
    }
    if (st == MXS_OK) st = scan_i32(width, wscan, ns, s);
    if (st == MXS_OK) {
        sell_offsets_kernel<<<grid_of(ns + 1), 256, 0, s>>>(wscan, ns, cs);
        st = launch_status();
    }
    (void)hipFreeAsync(width, s);
    return st;
}

mxs_status sell_size(const mxs_mat_s *A, int32_t sigma, int64_t *slots, hipStream_t s)
{
    const int32_t *irp;
    int32_t *tmp;
    const int64_t ns = ((int64_t)A->nrows + kSellC - 1) / kSellC;
    int32_t *perm = nullptr;
    int64_t *cs = nullptr;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    if (st == MXS_OK && hipMallocAsync((void **)&perm, sizeof(int32_t) * std::max<size_t>(A->nrows, 1), s) != hipSuccess)
        st = MXS_ERR_OUT_OF_MEMORY;
    if (st == MXS_OK && hipMallocAsync((void **)&cs, sizeof(int64_t) * ((size_t)ns + 1), s) != hipSuccess)
        st = MXS_ERR_OUT_OF_MEMORY;
    if (st == MXS_OK) st = sell_layout(A, irp, sigma, perm, cs, s);
    int64_t h = 0;
    if (st == MXS_OK && hipMemcpyAsync(&h, cs + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = MXS_ERR_HIP;
    if (perm) (void)hipFreeAsync(perm, s);
    if (cs) (void)hipFreeAsync(cs, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;
    if (h > 8 * A->nnz) return MXS_ERR_DIA_TOO_SPARSE;
    *slots = h;
    return MXS_OK;
}

mxs_status sell_build(const mxs_mat_s *A, int32_t sigma, int32_t *perm, int64_t *cs, int32_t *col,
                      void *vals, hipStream_t s)
{
    const int32_t *irp;
    int32_t *tmp;
    const int64_t ns = ((int64_t)A->nrows + kSellC - 1) / kSellC;
    mxs_status st = source_irp(A, &irp, &tmp, s);
    if (st == MXS_OK) st = sell_layout(A, irp, sigma, perm, cs, s);
    const int64_t npos = ns * kSellC;
    if (st == MXS_OK && npos > 0) {
        if (A->dtype == MXS_F64)
            sell_fill_kernel<double><<<grid_of(npos, 65536), 256, 0, s>>>(
                A->nrows, npos, irp, A->idx1, (const double *)A->vals, perm, cs, col, (double *)vals);
        else
            sell_fill_kernel<float><<<grid_of(npos, 65536), 256, 0, s>>>(
                A->nrows, npos, irp, A->idx1, (const float *)A->vals, perm, cs, col, (float *)vals);
        st = launch_status();
    }
    if (tmp) (void)hipFreeAsync(tmp, s);
    return st;
}

// ---------------------------------------------------------------------------
// ELL / SELL -> COO / CSR
// ---------------------------------------------------------------------------
// Row r's entries: its slots before the first padding slot.  `pos` is the
// slot-array index of slot 0 and `stride` the distance between slots.
struct PadRow {
    int64_t pos, stride;
    int32_t width, row;
};

// kernel view of an ELL or SELL handle
struct PadView {
    int32_t ell, nrows, width; // width: ELL slots per row
    const int32_t *col, *perm;
    const void *vals;
};

__device__ __forceinline__ PadRow pad_row(const PadView &A, const int64_t *cs, int64_t p)
{
    PadRow r;
    if (A.ell) {
        r = {p, (int64_t)A.nrows, A.width, (int32_t)p};
    } else {
        const int64_t sl = p / kSellC;
        r = {cs[sl] + p % kSellC, kSellC, (int32_t)((cs[sl + 1] - cs[sl]) / kSellC), A.perm[p]};
    }
    return r;
}

__global__ void pad_count_kernel(PadView A, const int64_t *__restrict__ cs, int32_t *__restrict__ len)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.nrows;
         p += (int64_t)gridDim.x * blockDim.x) {
        const PadRow r = pad_row(A, cs, p);
        int32_t k = 0;
        while (k < r.width && A.col[r.pos + k * r.stride] >= 0) ++k;
        len[r.row] = k;
    }
}

template <typename T>
__global__ void pad_emit_kernel(PadView A, const int64_t *__restrict__ cs, const int32_t *__restrict__ irp,
                                int32_t *__restrict__ ai, int32_t *__restrict__ aj, T *__restrict__ av)
{
    const T *__restrict__ v = (const T *)A.vals;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.nrows;
         p += (int64_t)gridDim.x * blockDim.x) {
        const PadRow r = pad_row(A, cs, p);
        const int32_t b = irp[r.row], len = irp[r.row + 1] - b;
        for (int32_t k = 0; k < len; ++k) {
            if (ai) ai[b + k] = r.row;
            aj[b + k] = A.col[r.pos + k * r.stride];
            av[b + k] = v[r.pos + k * r.stride];
        }
    }
}

mxs_status padded_to_rows(const mxs_mat_s *A, mxs_format dst, int32_t *idx0, int32_t *idx1,
                          void *vals, hipStream_t s)
{
    const int32_t n = A->nrows;
    int32_t *irp = dst == MXS_CSR ? idx0 : nullptr;
    int32_t *len = nullptr;
    if (!irp) MXS_HIP(hipMallocAsync((void **)&irp, sizeof(int32_t) * ((size_t)n + 1), s));
    MXS_HIP(hipMallocAsync((void **)&len, sizeof(int32_t) * ((size_t)n + 1), s));
    const PadView view{A->fmt == MXS_ELL ? 1 : 0, A->nrows, A->ndiag, A->idx0, A->idx1, A->vals};
    mxs_status st = MXS_OK;
    if (n > 0) {
        pad_count_kernel<<<grid_of(n, 65536), 256, 0, s>>>(view, A->sell_cs, len);
        st = launch_status();
    }
    if (st == MXS_OK) st = scan_i32(len, irp, n, s);
    if (st == MXS_OK && n > 0 && A->nnz > 0) {
        int32_t *ai = dst == MXS_COO ? idx0 : nullptr;
        if (A->dtype == MXS_F64)
            pad_emit_kernel<double><<<grid_of(n, 65536), 256, 0, s>>>(view, A->sell_cs, irp, ai, idx1,
                                                                      (double *)vals);
        else
            pad_emit_kernel<float><<<grid_of(n, 65536), 256, 0, s>>>(view, A->sell_cs, irp, ai, idx1,
                                                                     (float *)vals);
        st = launch_status();
    }
    (void)hipFreeAsync(len, s);
    if (dst != MXS_CSR) (void)hipFreeAsync(irp, s);
    return st;
}

// ---------------------------------------------------------------------------
// SpMV
// ---------------------------------------------------------------------------
// kPadU<T> slots per step, loads of a step issued together; slots past the
// width read nothing, padding slots (column -1) gather nothing.
template <typename T>
__device__ __forceinline__ T padded_row_sum(const int32_t *__restrict__ col, const T *__restrict__ val,
                                            int64_t pos, int64_t stride, int32_t w,
                                            const T *__restrict__ x)
{
    T sum = T(0);
    for (int32_t k = 0; k < w; k += kPadU<T>) {
        int32_t c[kPadU<T>];
        T v[kPadU<T>], xv[kPadU<T>];
#pragma unroll
        for (int u = 0; u < kPadU<T>; ++u) {
            const bool in = k + u < w;
            c[u] = in ? ld_nt(&col[pos + (int64_t)(k + u) * stride]) : -1;
            v[u] = in ? ld_nt(&val[pos + (int64_t)(k + u) * stride]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kPadU<T>; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < kPadU<T>; ++u)
            if (c[u] >= 0) sum += v[u] * xv[u];
    }
    return sum;
}

template <typename T, bool DOT>
__global__ __launch_bounds__(256) void ell_spmv_kernel(int32_t nrows, int32_t K,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val,
                                                       const T *__restrict__ x, T *__restrict__ y,
                                                       const int *__restrict__ done,
                                                       double *__restrict__ partials)
{
    __shared__ double red[256 / kWave];
    if (done && *done) return;
    double dpart = 0.0;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    for (int64_t i = b * 256 + threadIdx.x; i < nrows; i += (int64_t)gridDim.x * 256) {
        // the fused dot's x value first: its load overlaps the row's
        const T xi = DOT ? x[i] : T(0);
        const T yi = padded_row_sum(col, val, i, nrows, K, x);
        // y is read next by another kernel after a full vector pass: store it
        // past the caches
        __builtin_nontemporal_store(yi, &y[i]);
        if (DOT) dpart += (double)yi * (double)xi;
    }
    if (DOT) {
        const double bs = block_sum<256>(dpart, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    }
}

template <typename T, bool DOT>
__global__ __launch_bounds__(256) void sell_spmv_kernel(int32_t nrows, int64_t npos,
                                                        const int32_t *__restrict__ perm,
                                                        const int64_t *__restrict__ cs,
                                                        const int32_t *__restrict__ col,
                                                        const T *__restrict__ val,
                                                        const T *__restrict__ x, T *__restrict__ y,
                                                        const int *__restrict__ done,
                                                        double *__restrict__ partials)
{
    __shared__ double red[256 / kWave];
    if (done && *done) return;
    double dpart = 0.0;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    for (int64_t p = b * 256 + threadIdx.x; p < npos; p += (int64_t)gridDim.x * 256) {
        const int64_t sl = p / kSellC;
        const int64_t base = cs[sl];
        const int32_t w = (int32_t)((cs[sl + 1] - base) / kSellC);
        // the row id (and the fused dot's x value) first: their loads overlap the row's
        const int32_t i = p < nrows ? perm[p] : 0;
        const T xi = DOT && p < nrows ? x[i] : T(0);
        const T yi = padded_row_sum(col, val, base + p % kSellC, (int64_t)kSellC, w, x);
        if (p < nrows) {
            y[i] = yi;
            if (DOT) dpart += (double)yi * (double)xi;
        }
    }
    if (DOT) {
        const double bs = block_sum<256>(dpart, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    }
}

int64_t ell_grid(int32_t nrows, bool dot)
{
    return (int64_t)pad_grid(grid_of(nrows, dot ? 65536 : (1 << 30)));
}

template <typename T>
static mxs_status ell_typed(int32_t nrows, int32_t K, const int32_t *col, const T *val, const T *x, T *y,
                            const int *done, double *parts, hipStream_t s)
{
    const uint32_t g = (uint32_t)ell_grid(nrows, parts != nullptr);
    if (parts)
        ell_spmv_kernel<T, true><<<g, 256, 0, s>>>(nrows, K, col, val, x, y, done, parts);
    else
        ell_spmv_kernel<T, false><<<g, 256, 0, s>>>(nrows, K, col, val, x, y, done, nullptr);
    return launch_status();
}

mxs_status ell_launch(int32_t nrows, int32_t K, const int32_t *col, const void *vals, mxs_dtype t,
                      const void *x, void *y, const int *done, double *parts, hipStream_t s)
{
    if (t == MXS_F64)
        return ell_typed<double>(nrows, K, col, (const double *)vals, (const double *)x, (double *)y,
                                 done, parts, s);
    return ell_typed<float>(nrows, K, col, (const float *)vals, (const float *)x, (float *)y, done,
                            parts, s);
}

static int64_t padded_units(const mxs_mat_s *A)
{
    return A->fmt == MXS_ELL ? A->nrows : ((int64_t)A->nrows + kSellC - 1) / kSellC * kSellC;
}

// A multiple of 8 workgroups (xcd_remap is a permutation of such grids).
int64_t padded_grid(const mxs_mat_s *A, bool dot)
{
    return (int64_t)pad_grid(grid_of(padded_units(A), dot ? 65536 : (1 << 30)));
}

template <typename T>
static mxs_status padded_typed(const mxs_mat_s *A, const T *x, T *y, const int *done, double *parts,
                               hipStream_t s)
{
    const uint32_t g = (uint32_t)padded_grid(A, parts != nullptr);
    const T *v = (const T *)A->vals;
    if (A->fmt == MXS_ELL) {
        if (parts)
            ell_spmv_kernel<T, true><<<g, 256, 0, s>>>(A->nrows, A->ndiag, A->idx0, v, x, y, done, parts);
        else
            ell_spmv_kernel<T, false><<<g, 256, 0, s>>>(A->nrows, A->ndiag, A->idx0, v, x, y, done, nullptr);
    } else {
        const int64_t npos = padded_units(A);
        if (parts)
            sell_spmv_kernel<T, true><<<g, 256, 0, s>>>(A->nrows, npos, A->idx1, A->sell_cs, A->idx0, v, x,
                                                        y, done, parts);
        else
            sell_spmv_kernel<T, false><<<g, 256, 0, s>>>(A->nrows, npos, A->idx1, A->sell_cs, A->idx0, v, x,
                                                         y, done, nullptr);
    }
    return launch_status();
}

mxs_status padded_spmv(const mxs_mat_s *A, const void *x, void *y, const int *done, double *parts,
                       hipStream_t s)
{
    if (A->dtype == MXS_F64)
        return padded_typed<double>(A, (const double *)x, (double *)y, done, parts, s);
    return padded_typed<float>(A, (const float *)x, (float *)y, done, parts, s);
}

}  // namespace mxs
