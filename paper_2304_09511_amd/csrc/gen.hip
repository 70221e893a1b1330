// HPCG problem setup on the device (Section VII-D: Poisson on a regular 3-D
// grid with a 27-point stencil; the 7-point variant for the selector's data).
// Grid point (x, y, z) is row x + n*y + n*n*z; a row's entries are emitted in
// (dz, dy, dx) order, which is ascending column order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "common.h"

namespace mxs {

__device__ __forceinline__ int axis_span(int64_t g, int n, int d)
{
    // is neighbour g + d inside [0, n)?
    return (g + d >= 0) && (g + d < n);
}

__global__ void stencil_count_kernel(int32_t n, int32_t points, int32_t *__restrict__ cnt)
{
    const int64_t N = (int64_t)n * n * n;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gx = r % n, gy = (r / n) % n, gz = r / ((int64_t)n * n);
        int c;
        if (points == 27) {
            const int cx = 1 + axis_span(gx, n, -1) + axis_span(gx, n, 1);
            const int cy = 1 + axis_span(gy, n, -1) + axis_span(gy, n, 1);
            const int cz = 1 + axis_span(gz, n, -1) + axis_span(gz, n, 1);
            c = cx * cy * cz;
        } else {
            c = 1 + axis_span(gx, n, -1) + axis_span(gx, n, 1) + axis_span(gy, n, -1) +
                axis_span(gy, n, 1) + axis_span(gz, n, -1) + axis_span(gz, n, 1);
        }
        cnt[r] = c;
    }
}

template <typename T>
__global__ void stencil_write_kernel(int32_t n, int32_t points, T diag, T offdiag,
                                     const int32_t *__restrict__ pos, int32_t *__restrict__ ai,
                                     int32_t *__restrict__ aj, T *__restrict__ av)
{
    const int64_t N = (int64_t)n * n * n;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gx = r % n, gy = (r / n) % n, gz = r / ((int64_t)n * n);
        int32_t p = pos[r];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (points == 7 && abs(dx) + abs(dy) + abs(dz) > 1) continue;
                    if (!axis_span(gx, n, dx) || !axis_span(gy, n, dy) || !axis_span(gz, n, dz))
                        continue;
                    ai[p] = (int32_t)r;
                    aj[p] = (int32_t)(r + dx + (int64_t)n * dy + (int64_t)n * n * dz);
                    av[p] = (dx == 0 && dy == 0 && dz == 0) ? diag : offdiag;
                    ++p;
                }
    }
}

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t stencil_ws_bytes(int32_t n)
{
    const int64_t N = (int64_t)n * n * n;
    return up256(sizeof(int32_t) * (size_t)N) + up256(sizeof(int32_t) * ((size_t)N + 1)) +
           scan_ws_bytes(N);
}

// The generator with its temporaries (row lengths, their scan) in
// ws[stencil_ws_bytes(n)].
mxs_status stencil_coo_ws(int32_t n, int32_t points, double diag, double offdiag, int32_t *ai,
                          int32_t *aj, void *av, mxs_dtype t, void *ws, hipStream_t s)
{
    const int64_t N = (int64_t)n * n * n;
    if (N == 0) return MXS_OK;
    auto *cnt = (int32_t *)ws;
    auto *pos = (int32_t *)((char *)ws + up256(sizeof(int32_t) * (size_t)N));
    void *sws = (char *)pos + up256(sizeof(int32_t) * ((size_t)N + 1));
    const uint32_t g = (uint32_t)std::min<int64_t>((N + 255) / 256, 65536);
    stencil_count_kernel<<<g, 256, 0, s>>>(n, points, cnt);
    MXS_HIP(hipGetLastError());
    mxs_status st = scan_i32_ws(cnt, pos, N, sws, s);
    if (st == MXS_OK) {
        if (t == MXS_F64)
            stencil_write_kernel<double><<<g, 256, 0, s>>>(n, points, diag, offdiag, pos, ai, aj,
                                                           (double *)av);
        else
            stencil_write_kernel<float><<<g, 256, 0, s>>>(n, points, (float)diag, (float)offdiag,
                                                          pos, ai, aj, (float *)av);
        st = launch_status();
    }
    return st;
}

mxs_status stencil_coo(int32_t n, int32_t points, double diag, double offdiag, int32_t *ai,
                       int32_t *aj, void *av, mxs_dtype t, hipStream_t s)
{
    const int64_t N = (int64_t)n * n * n;
    if (N == 0) return MXS_OK;
    void *ws = nullptr;
    MXS_HIP(hipMallocAsync(&ws, stencil_ws_bytes(n), s));
    const mxs_status st = stencil_coo_ws(n, points, diag, offdiag, ai, aj, av, t, ws, s);
    MXS_HIP(hipFreeAsync(ws, s));
    return st;
}

}  // namespace mxs
