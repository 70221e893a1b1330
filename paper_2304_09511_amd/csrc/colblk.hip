// Column blocks of a COO or CSR matrix (COO implementation 2, CSR 4).
//
// Algorithms 1 and 2 gather x[aj[k]] for every entry.  When x is much larger
// than one XCD's 4 MiB L2 and most entries lie far from the diagonal
// (uniformly scattered columns, say), nearly every gather misses L2 and the
// SpMV is bound by gather transactions, not by the matrix stream.
// mxs_optimize then splits the entries by column range into K full-height
// matrices of the same format whose x ranges fit one L2 each: block b holds,
// row by row, the entries with columns in [b*cb, (b+1)*cb), in their
// original order.  The blocks run in turn with the format's tile kernels,
// the first writing y and the others adding to it, so all gathers of a pass
// fall in one L2-sized window of x.  The cost: a second copy of the entries
// (with row ids for COO, K row-pointer arrays for CSR) and K passes over y.
// Per row the sum is the row's block sums added in block order.
#include "common.h"

#include <algorithm>

namespace mxs {

constexpr int64_t kColBlkX = 4ll << 20;     // bytes of x per block (one XCD's L2)
constexpr int64_t kColBlkMinX = 8ll << 20;  // x smaller than this: no blocks
constexpr int kColBlkMax = 32;

// Scattered entries, summed into *far: |j - i| >= half (half a block's
// width) and x[j] in another 128-byte line than the row's previous entry's
// x (lpl columns per line).  Entries that share lines (dense sub-blocks,
// say) gather cheaply however far they lie, and blocks would only add
// passes over y.
__global__ void colblk_far_kernel(const int32_t *__restrict__ irp, const int32_t *__restrict__ aj,
                                  int32_t nrows, int64_t half, int32_t lpl,
                                  unsigned long long *__restrict__ far)
{
    __shared__ unsigned long long red[256 / kWave];
    unsigned long long c = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t prev_line = -1;
        for (int32_t k = irp[r]; k < irp[r + 1]; ++k) {
            const int32_t line = aj[k] / lpl;
            c += (uint64_t)((aj[k] - r >= half || r - aj[k] >= half) && line != prev_line);
            prev_line = line;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / kWave; ++w) t += red[w];
        atomicAdd(far, t);
    }
}

// cnt[b*nrows + r] = entries of row r in column block b (cnt zeroed first).
// Columns ascend within a row, so a row's entries of one block are a run.
__global__ void colblk_count_kernel(const int32_t *__restrict__ irp, const int32_t *__restrict__ aj,
                                    int32_t nrows, int32_t cb, int32_t *__restrict__ cnt)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k0 = irp[r], k1 = irp[r + 1];
        int32_t k = k0;
        while (k < k1) {
            const int32_t b = aj[k] / cb;
            const int32_t start = k;
            while (k < k1 && aj[k] / cb == b) ++k;
            cnt[(int64_t)b * nrows + r] = k - start;
        }
    }
}

// Block b's entries of row r go to boff[b] + bip[b*(nrows+1) + r] onward,
// in their original order (with their row id in oi when oi is given).
template <typename T>
__global__ void colblk_fill_kernel(const int32_t *__restrict__ irp, const int32_t *__restrict__ aj,
                                   const T *__restrict__ av, int32_t nrows, int32_t cb,
                                   const int32_t *__restrict__ bip, const int64_t *__restrict__ boff,
                                   int32_t *__restrict__ oi, int32_t *__restrict__ oj,
                                   T *__restrict__ ov)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k1 = irp[r + 1];
        int32_t b = -1;
        int64_t dst = 0;
        for (int32_t k = irp[r]; k < k1; ++k) {
            const int32_t bk = aj[k] / cb;
            if (bk != b) {
                b = bk;
                dst = boff[b] + bip[(int64_t)b * ((int64_t)nrows + 1) + r];
            }
            if (oi) oi[dst] = (int32_t)r;
            oj[dst] = aj[k];
            ov[dst] = av[k];
            ++dst;
        }
    }
}

static uint32_t row_grid(int32_t nrows) { return (uint32_t)std::clamp<int64_t>(((int64_t)nrows + 255) / 256, 1, 16384); }

// Builds the blocks of COO or CSR matrix A when x exceeds kColBlkMinX bytes
// and at least half of the entries are scattered (colblk_far_kernel).  Optional: without memory for the copy the matrix keeps its
// other implementations.  The blocks are part handles owned by A.
static mxs_status colblk_make(mxs_mat_s *A, const int32_t *irp, hipStream_t s)
{
    const int64_t xb = (int64_t)A->ncols * (int64_t)dsize(A->dtype);
    const int K = (int)std::min<int64_t>((xb + kColBlkX - 1) / kColBlkX, kColBlkMax);
    const int32_t cb = (int32_t)(((int64_t)A->ncols + K - 1) / K);
    const int32_t n = A->nrows;
    const bool coo = A->fmt == MXS_COO;

    unsigned long long *far = nullptr;
    MXS_HIP(hipMallocAsync((void **)&far, sizeof(unsigned long long), s));
    mxs_status st = fill_bytes0(far, sizeof(unsigned long long), s);
    if (st == MXS_OK) {
        colblk_far_kernel<<<row_grid(n), 256, 0, s>>>(irp, A->idx1, n, cb / 2,
                                                      (int32_t)(128 / dsize(A->dtype)), far);
        st = launch_status();
    }
    unsigned long long h_far = 0;
    if (st == MXS_OK && hipMemcpyAsync(&h_far, far, sizeof h_far, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = MXS_ERR_HIP;
    (void)hipFreeAsync(far, s);
    MXS_HIP(hipStreamSynchronize(s));
    if (st != MXS_OK) return st;
    if (2 * (int64_t)h_far < A->nnz) return MXS_OK;

    // the copy: CSR keeps K row-pointer arrays, then the columns, then the
    // values; COO keeps the row ids, columns and values (its block row
    // pointers are only needed here)
    const size_t np = (size_t)K * ((size_t)n + 1);
    const size_t nidx = (coo ? 0 : np) + (size_t)A->nnz * (coo ? 2 : 1); // int32 words
    const size_t vbase = (nidx * sizeof(int32_t) + 255) / 256 * 256;      // values 256-byte aligned
    void *buf = nullptr;
    if (hipMalloc(&buf, vbase + (size_t)A->nnz * dsize(A->dtype)) != hipSuccess) {
        (void)hipGetLastError();
        return MXS_OK;
    }
    int32_t *cnt = nullptr, *tmp_bip = nullptr;
    if (hipMallocAsync((void **)&cnt, sizeof(int32_t) * (size_t)K * n, s) != hipSuccess ||
        (coo && hipMallocAsync((void **)&tmp_bip, sizeof(int32_t) * np, s) != hipSuccess)) {
        (void)hipGetLastError();
        if (cnt) (void)hipFreeAsync(cnt, s);
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        return MXS_OK;
    }
    A->owned.push_back(buf);
    int32_t *bip = coo ? tmp_bip : (int32_t *)buf;
    int32_t *oi = coo ? (int32_t *)buf : nullptr;
    int32_t *oj = coo ? oi + A->nnz : bip + np;
    void *ov = (char *)buf + vbase;
    auto free_tmp = [&] {
        if (tmp_bip) (void)hipFreeAsync(tmp_bip, s);
        tmp_bip = nullptr;
    };
    st = fill_bytes0(cnt, sizeof(int32_t) * (size_t)K * n, s);
    if (st == MXS_OK) {
        colblk_count_kernel<<<row_grid(n), 256, 0, s>>>(irp, A->idx1, n, cb, cnt);
        st = launch_status();
    }
    for (int b = 0; b < K && st == MXS_OK; ++b)
        st = scan_i32(cnt + (size_t)b * n, bip + (size_t)b * ((size_t)n + 1), n, s);
    (void)hipFreeAsync(cnt, s);
    std::vector<int32_t> tot((size_t)K, 0);
    for (int b = 0; b < K && st == MXS_OK; ++b)
        if (hipMemcpyAsync(&tot[(size_t)b], bip + (size_t)b * ((size_t)n + 1) + n, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            st = MXS_ERR_HIP;
    if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
    std::vector<int64_t> off((size_t)K + 1, 0);
    for (int b = 0; b < K; ++b) off[(size_t)b + 1] = off[(size_t)b] + tot[(size_t)b];
    if (st == MXS_OK && off[(size_t)K] != A->nnz) st = MXS_ERR_INVALID_ARG; // the counts cover every entry
    if (st != MXS_OK) {
        free_tmp();
        return st;
    }

    int64_t *boff = nullptr;
    if (hipMallocAsync((void **)&boff, sizeof(int64_t) * ((size_t)K + 1), s) != hipSuccess ||
        hipMemcpyAsync(boff, off.data(), sizeof(int64_t) * ((size_t)K + 1), hipMemcpyHostToDevice, s) !=
            hipSuccess)
        st = MXS_ERR_HIP;
    if (st == MXS_OK) {
        if (A->dtype == MXS_F64)
            colblk_fill_kernel<double><<<row_grid(n), 256, 0, s>>>(irp, A->idx1, (const double *)A->vals,
                                                                 n, cb, bip, boff, oi, oj, (double *)ov);
        else
            colblk_fill_kernel<float><<<row_grid(n), 256, 0, s>>>(irp, A->idx1, (const float *)A->vals,
                                                                n, cb, bip, boff, oi, oj, (float *)ov);
        st = launch_status();
    }
    if (boff) (void)hipFreeAsync(boff, s);
    free_tmp();
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;

    std::vector<mxs_mat_s *> blk;
    for (int b = 0; b < K && st == MXS_OK; ++b) {
        auto *B = new mxs_mat_s;
        B->fmt = A->fmt;
        B->dtype = A->dtype;
        B->nrows = A->nrows;
        B->ncols = A->ncols;
        B->nnz = tot[(size_t)b];
        B->idx0 = coo ? oi + off[(size_t)b] : bip + (size_t)b * ((size_t)n + 1);
        B->idx1 = oj + off[(size_t)b];
        B->vals = (const char *)ov + off[(size_t)b] * (int64_t)dsize(A->dtype);
        B->device = A->device;
        B->part = true;
        blk.push_back(B);
        st = build_plan(B, s);
    }
    if (st != MXS_OK) {
        for (auto *B : blk) release(B);
        return st;
    }
    A->cblk = std::move(blk);
    return MXS_OK;
}

mxs_status colblk_build(mxs_mat_s *A, hipStream_t s)
{
    const int64_t xb = (int64_t)A->ncols * (int64_t)dsize(A->dtype);
    if ((A->fmt != MXS_COO && A->fmt != MXS_CSR) || A->part || A->nnz == 0 || A->nrows == 0 ||
        xb < kColBlkMinX)
        return MXS_OK;
    if (A->fmt == MXS_CSR) return colblk_make(A, A->idx0, s);
    // COO: row pointers from the sorted row ids, for the build only
    int32_t *irp = nullptr;
    MXS_HIP(hipMallocAsync((void **)&irp, sizeof(int32_t) * ((size_t)A->nrows + 1), s));
    mxs_status st = coo_irp_launch(A->nnz, A->nrows, A->idx0, irp, s);
    if (st == MXS_OK) st = colblk_make(A, irp, s);
    (void)hipFreeAsync(irp, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
    return st;
}

}  // namespace mxs
