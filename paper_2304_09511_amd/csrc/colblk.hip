// Column blocks of a COO or CSR matrix (COO implementation 2, CSR 4).
//
// Algorithms 1 and 2 gather x[aj[k]] for every entry.  When x is much larger
// than one XCD's 4 MiB L2 and most entries lie far from the diagonal
// (uniformly scattered columns, say), nearly every gather misses L2 and the
// SpMV is bound by gather transactions, not by the matrix stream.
// mxs_optimize then splits the entries by column range into K full-height
// matrices of the same format whose x ranges about fit one L2 each: block b holds,
// row by row, the entries with columns in [b*cb, (b+1)*cb), in their
// original order.  The blocks run in turn with the format's tile kernels,
// the first writing y and the others adding to it, so all gathers of a pass
// fall in one window of x of about an L2's size.  The cost: a second copy of the entries
// (with row ids for COO, K row-pointer arrays for CSR) and K passes over y.
// Per row the sum is the row's block sums added in block order.
#include "common.h"

#include <algorithm>
#include <vector>

namespace mxs {

// Bytes of x per block: blocks of up to 6 MiB, a little more than one XCD's
// 4 MiB L2, measured best (4M-row Zipf matrix, CSR blocks of 2,048-entry
// tiles: 678 us with 6 blocks, 691 with 7, 716 with 8, 719 with 5; 8M rows:
// 1,645 against 1,880 us with 4 MiB blocks): a pass over y and the row
// pointers fewer outweighs the gathers that a window past the L2's size
// sends on to the MALL.
constexpr int64_t kColBlkX = 6ll << 20;
constexpr int64_t kColBlkMinX = 8ll << 20;  // x smaller than this: no blocks
constexpr int64_t kColBlkMinPerRow = 3;     // fewer entries per row on average: no blocks
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

// The same count from sorted COO arrays: entry k's predecessor in its row
// is entry k-1 when that holds the same row id.
__global__ void colblk_far_coo_kernel(const int32_t *__restrict__ ai, const int32_t *__restrict__ aj,
                                      int64_t nnz, int64_t half, int32_t lpl,
                                      unsigned long long *__restrict__ far)
{
    __shared__ unsigned long long red[256 / kWave];
    unsigned long long c = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = ai[k], j = aj[k];
        const int32_t prev_line = k > 0 && ai[k - 1] == ai[k] ? aj[k - 1] / lpl : -1;
        c += (uint64_t)((j - r >= half || r - j >= half) && aj[k] / lpl != prev_line);
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

// cnt[b] += entries with columns in block b (K <= kColBlkMax blocks of width cb).
__global__ void colblk_hist_kernel(const int32_t *__restrict__ aj, int64_t nnz, int32_t cb, int K,
                                   unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned int h[kColBlkMax];
    for (int b = threadIdx.x; b < K; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[aj[k] / cb], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < K; b += blockDim.x)
        if (h[b]) atomicAdd(&cnt[b], (unsigned long long)h[b]);
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
static uint32_t entry_grid(int64_t nnz) { return (uint32_t)std::clamp<int64_t>((nnz + 255) / 256, 1, 4096); }

// Column blocks of COO or CSR matrix A, laid out in the plan when x has at
// least kColBlkMinX bytes and at least half of the entries are scattered
// (not for parts, nor with MXS_PLAN_NO_COLBLK).  irp: A's row pointers in
// the build pass (CSR: its own; COO: a temporary of the plan).  The blocks
// are part handles owned by A, each with its own tiles and carries.
mxs_status colblk_plan(mxs_mat_s *A, const int32_t *irp, PlanCtx &c, hipStream_t s)
{
    const int64_t xb = (int64_t)A->ncols * (int64_t)dsize(A->dtype);
    if ((A->fmt != MXS_COO && A->fmt != MXS_CSR) || A->sub || A->part || A->nnz == 0 ||
        A->nrows == 0 || xb < kColBlkMinX || (c.opts & MXS_PLAN_NO_COLBLK))
        return MXS_OK;
    // every block passes over y and the row pointers: with fewer than three
    // entries per row on average that costs more than the gathers save
    // (random entries on 4M rows, CSR blocks against none: 118 against 48 us
    // at 0.5 per row, 178 against 146 at 2, 268 against 274 at 4)
    if (A->nnz < kColBlkMinPerRow * (int64_t)A->nrows) return MXS_OK;
    const int K = (int)std::min<int64_t>((xb + kColBlkX - 1) / kColBlkX, kColBlkMax);
    const int32_t cb = (int32_t)(((int64_t)A->ncols + K - 1) / K);
    const int32_t n = A->nrows;
    const bool coo = A->fmt == MXS_COO;

    // measured in both passes: scattered entries, entries per block
    auto *cnt = (unsigned long long *)c.counters(); // [0] scattered, [1 + b] block b
    if (!cnt) return MXS_ERR_INVALID_ARG;
    mxs_status st = fill_bytes0(cnt, sizeof(unsigned long long) * ((size_t)K + 1), s);
    if (st != MXS_OK) return st;
    const int32_t lpl = (int32_t)(128 / dsize(A->dtype));
    if (coo)
        colblk_far_coo_kernel<<<entry_grid(A->nnz), 256, 0, s>>>(A->idx0, A->idx1, A->nnz, cb / 2, lpl, cnt);
    else
        colblk_far_kernel<<<row_grid(n), 256, 0, s>>>(irp, A->idx1, n, cb / 2, lpl, cnt);
    colblk_hist_kernel<<<entry_grid(A->nnz), 256, 0, s>>>(A->idx1, A->nnz, cb, K, cnt + 1);
    MXS_HIP(hipGetLastError());
    std::vector<unsigned long long> h((size_t)K + 1);
    MXS_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    if (2 * (int64_t)h[0] < A->nnz) return MXS_OK;
    std::vector<int64_t> off((size_t)K + 1, 0);
    for (int b = 0; b < K; ++b) off[(size_t)b + 1] = off[(size_t)b] + (int64_t)h[(size_t)b + 1];
    if (off[(size_t)K] != A->nnz) return MXS_ERR_INVALID_ARG; // the counts cover every entry

    // kept: CSR has K row-pointer arrays, then the columns, then the values;
    // COO the row ids, columns and values (its block row pointers are only
    // needed while the copy is cut)
    const size_t np = (size_t)K * ((size_t)n + 1);
    int32_t *bip_keep = coo ? nullptr : (int32_t *)c.keep(sizeof(int32_t) * np);
    int32_t *oi = coo ? (int32_t *)c.keep(sizeof(int32_t) * (size_t)A->nnz) : nullptr;
    int32_t *oj = (int32_t *)c.keep(sizeof(int32_t) * (size_t)A->nnz);
    void *ov = c.keep((size_t)A->nnz * dsize(A->dtype));
    // temporaries: entries per (block, row), COO's block row pointers, block
    // offsets and the scan's partial sums
    const size_t mark = c.mark();
    int32_t *rc = (int32_t *)c.tmp(sizeof(int32_t) * (size_t)K * n);
    int32_t *bip = coo ? (int32_t *)c.tmp(sizeof(int32_t) * np) : bip_keep;
    auto *boff = (int64_t *)c.tmp(sizeof(int64_t) * ((size_t)K + 1));
    void *sws = c.tmp(scan_ws_bytes(n));
    if (c.build) {
        st = fill_bytes0(rc, sizeof(int32_t) * (size_t)K * n, s);
        if (st == MXS_OK) {
            colblk_count_kernel<<<row_grid(n), 256, 0, s>>>(irp, A->idx1, n, cb, rc);
            st = launch_status();
        }
        for (int b = 0; b < K && st == MXS_OK; ++b)
            st = scan_i32_ws(rc + (size_t)b * n, bip + (size_t)b * ((size_t)n + 1), n, sws, s);
        if (st == MXS_OK &&
            hipMemcpyAsync(boff, off.data(), sizeof(int64_t) * ((size_t)K + 1), hipMemcpyHostToDevice, s) !=
                hipSuccess)
            st = MXS_ERR_HIP;
        if (st == MXS_OK) {
            if (A->dtype == MXS_F64)
                colblk_fill_kernel<double><<<row_grid(n), 256, 0, s>>>(
                    irp, A->idx1, (const double *)A->vals, n, cb, bip, boff, oi, oj, (double *)ov);
            else
                colblk_fill_kernel<float><<<row_grid(n), 256, 0, s>>>(
                    irp, A->idx1, (const float *)A->vals, n, cb, bip, boff, oi, oj, (float *)ov);
            st = launch_status();
        }
        // off[] is a host array read by the copy above: wait for it
        if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
        if (st != MXS_OK) return st;
    }
    c.release(mark);

    // the blocks: handles of A's format over their parts of the copy
    std::vector<mxs_mat_s *> blk;
    for (int b = 0; b < K && st == MXS_OK; ++b) {
        auto *B = new mxs_mat_s;
        B->fmt = A->fmt;
        B->dtype = A->dtype;
        B->nrows = A->nrows;
        B->ncols = A->ncols;
        B->nnz = off[(size_t)b + 1] - off[(size_t)b];
        if (c.build) {
            B->idx0 = coo ? oi + off[(size_t)b] : bip + (size_t)b * ((size_t)n + 1);
            B->idx1 = oj + off[(size_t)b];
            B->vals = (const char *)ov + off[(size_t)b] * (int64_t)dsize(A->dtype);
        }
        B->device = A->device;
        B->part = true;
        B->sub = true;
        B->cblk_part = true;
        blk.push_back(B);
        st = plan_walk(B, c, s);
    }
    if (st != MXS_OK || !c.build) {
        for (auto *B : blk) release(B);
        return st;
    }
    A->cblk = std::move(blk);
    return MXS_OK;
}

}  // namespace mxs
