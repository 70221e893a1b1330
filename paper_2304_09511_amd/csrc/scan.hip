// Device prefix sums and fills used by the analysis and the conversions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "common.h"

namespace mxs {

constexpr int kScanNT = 256;
constexpr int kScanIPT = 16;
constexpr int kScanTile = kScanNT * kScanIPT;

__device__ __forceinline__ long long wave_incl_scan(long long v)
{
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const long long t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan over the workgroup in thread order; *total gets the sum.
__device__ long long block_excl_scan(long long v, long long *smem, long long *total)
{
    const long long inc = wave_incl_scan(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == kWave - 1) smem[w] = inc;
    __syncthreads();
    long long pre = 0, tot = 0;
    for (int i = 0; i < kScanNT / kWave; ++i) {
        if (i < w) pre += smem[i];
        tot += smem[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__global__ __launch_bounds__(kScanNT) void scan_tile_sums(const int32_t *__restrict__ in,
                                                          int64_t n, long long *__restrict__ sums)
{
    __shared__ long long smem[kScanNT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    long long s = 0;
    for (int e = 0; e < kScanIPT; ++e) {
        const int64_t i = base + e * kScanNT + threadIdx.x;
        if (i < n) s += in[i];
    }
    long long tot;
    block_excl_scan(s, smem, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place, carrying a running
// total across chunks; writes the grand total to out[n] (and flags overflow).
__global__ __launch_bounds__(kScanNT) void scan_tile_offsets(long long *__restrict__ sums,
                                                             int64_t ntiles,
                                                             int32_t *__restrict__ out, int64_t n,
                                                             int *__restrict__ overflow)
{
    __shared__ long long smem[kScanNT / kWave];
    long long carry = 0;
    for (int64_t c = 0; c < ntiles; c += kScanNT) {
        const int64_t i = c + threadIdx.x;
        const long long v = i < ntiles ? sums[i] : 0;
        long long tot;
        const long long ex = block_excl_scan(v, smem, &tot);
        if (i < ntiles) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        out[n] = (int32_t)std::min<long long>(carry, INT_MAX);
        *overflow = carry > INT_MAX;
    }
}

__global__ __launch_bounds__(kScanNT) void scan_tiles(const int32_t *__restrict__ in, int64_t n,
                                                      const long long *__restrict__ offs,
                                                      int32_t *__restrict__ out)
{
    __shared__ long long smem[kScanNT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    int32_t v[kScanIPT];
    long long s = 0;
#pragma unroll
    for (int e = 0; e < kScanIPT; ++e) {
        const int64_t i = base + e;
        v[e] = i < n ? in[i] : 0;
        s += v[e];
    }
    long long tot;
    long long run = offs[blockIdx.x] + block_excl_scan(s, smem, &tot);
#pragma unroll
    for (int e = 0; e < kScanIPT; ++e) {
        const int64_t i = base + e;
        if (i < n) out[i] = (int32_t)std::min<long long>(run, INT_MAX);
        run += v[e];
    }
}

size_t scan_ws_bytes(int64_t n)
{
    const int64_t ntiles = std::max<int64_t>((n + kScanTile - 1) / kScanTile, 1);
    return sizeof(long long) * (size_t)ntiles + 256;
}

// The scan with its temporaries (tile sums, overflow flag) in ws[scan_ws_bytes(n)].
mxs_status scan_i32_ws(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s)
{
    const int64_t ntiles = std::max<int64_t>((n + kScanTile - 1) / kScanTile, 1);
    long long *sums = (long long *)ws;
    int *ovf = (int *)((char *)ws + sizeof(long long) * (size_t)ntiles);
    scan_tile_sums<<<(uint32_t)ntiles, kScanNT, 0, s>>>(in, n, sums);
    MXS_HIP(hipGetLastError());
    scan_tile_offsets<<<1, kScanNT, 0, s>>>(sums, ntiles, out, n, ovf);
    MXS_HIP(hipGetLastError());
    if (n > 0) {
        scan_tiles<<<(uint32_t)ntiles, kScanNT, 0, s>>>(in, n, sums, out);
        MXS_HIP(hipGetLastError());
    }
    int h_ovf = 0;
    MXS_HIP(hipMemcpyAsync(&h_ovf, ovf, sizeof(int), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    return h_ovf ? MXS_ERR_INDEX_RANGE : MXS_OK;
}

mxs_status scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s)
{
    void *ws = nullptr;
    MXS_HIP(hipMallocAsync(&ws, scan_ws_bytes(n), s));
    const mxs_status st = scan_i32_ws(in, out, n, ws, s);
    (void)hipFreeAsync(ws, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) return MXS_ERR_HIP;
    return st;
}

__global__ void fill_i32_kernel(int32_t *__restrict__ p, int32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_zero_kernel(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

static uint32_t fill_grid(int64_t n)
{
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

mxs_status fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return MXS_OK;
    fill_i32_kernel<<<fill_grid(n), 256, 0, s>>>(p, v, n);
    return launch_status();
}

// Zero-fills `bytes` (a multiple of 4).
mxs_status fill_bytes0(void *p, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return MXS_OK;
    fill_u32_zero_kernel<<<fill_grid(n), 256, 0, s>>>((uint32_t *)p, n);
    return launch_status();
}

}  // namespace mxs
