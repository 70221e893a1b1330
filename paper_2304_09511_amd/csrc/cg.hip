// BLAS-1 and the conjugate-gradient driver: HPCG's solver with the
// preconditioner disabled (Section VII-D), plus FP32-inner / FP64-outer
// iterative refinement built on the same kernels.
//
// Scalars live on the device (CgState).  One CG iteration is five launches:
//   1. q = A p with p.q partials fused into the SpMV epilogue (CSR, DIA;
//      COO adds one dot kernel)    2. alpha = rho / p.q (one workgroup)
//   3. x += alpha p, r -= alpha q with r.r partials fused
//   4. convergence test, beta (one workgroup)    5. p = r + beta p
// Every kernel returns at entry once the device flag `done` is set, so the
// host enqueues iterations in batches and reads the flag once per batch.
// Reductions are per-workgroup partials summed in index order by a
// single-workgroup kernel: deterministic, and no device-scope fences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

#include "common.h"

namespace mxs {

constexpr int kVNT = 256;
constexpr int kVU = 4;                // 16-byte vectors per array a thread loads in one step
constexpr int64_t kVecGridMax = 8192;

// Grid of the vector kernels over n values of es bytes: one step of kVU
// 16-byte vectors per thread (n*es/16/1024 workgroups), capped; larger
// vectors are covered by grid-stride steps.  Kernels and the finish kernels
// that sum their per-workgroup partials use the same grid.
static uint32_t vec_grid(int64_t n, size_t es = 8)
{
    const int64_t nv = (int64_t)((uint64_t)n * es / 16);
    return pad_grid(std::clamp<int64_t>((nv + kVNT * kVU - 1) / (kVNT * kVU), 1, kVecGridMax));
}

// The block of the vector kernels of the CG loop: with a grid of a multiple
// of 8 workgroups, XCD j (workgroups j, j + 8, ...) takes the j-th eighth
// of the vectors, the rows whose SpMV blocks the same XCD runs, so that a
// vector written by one kernel of the loop is read by the next through the
// same L2 (measured at 128^3: CG 24.5 -> 23.7 ms in DIA, 32.0 -> 31.0 ms in
// CSR).  Partials are stored at this block's index: index order is still
// vector order.  DESCEND: the XCD's blocks in descending order, so that a
// kernel following one that ran ascending (the SpMV, writing q) reads the
// most recently written lines first (a further 0.3-0.4 ms).
template <bool DESCEND = false>
__device__ __forceinline__ int64_t vec_block()
{
    if (gridDim.x % kNumXcd) return blockIdx.x;
    const uint32_t per = gridDim.x / kNumXcd, k = blockIdx.x / kNumXcd;
    return (int64_t)(blockIdx.x % kNumXcd) * per + (DESCEND ? per - 1 - k : k);
}

static bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// 16 bytes of T as one vector (two FP64 or four FP32 values): one 128-bit
// load or store per lane, a wave's access one contiguous KiB.
template <typename T>
using V16 = T __attribute__((ext_vector_type(16 / sizeof(T))));

#define VEC_LOOP(i, n)                                                         \
    for (int64_t i = (int64_t)blockIdx.x * kVNT + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * kVNT)

struct Aux {
    double norm2[2]; // results of norm kernels
    int nonfinite;
    int pad;
};

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// Per-workgroup partials of a.b.  VEC (both 16-byte aligned): each thread
// loads kVU 16-byte vectors of each array (non-temporal) before adding, then
// the scalar tail of n mod (16/sizeof(T)); a fixed order per thread.
template <typename T, bool VEC>
__global__ __launch_bounds__(kVNT) void dot_kernel(int64_t n, const T *__restrict__ a,
                                                   const T *__restrict__ b, double *partials)
{
    __shared__ double red[kVNT / kWave];
    double s = 0.0;
    int64_t tail = 0;
    if constexpr (VEC) {
        using V = V16<T>;
        constexpr int W = 16 / sizeof(T);
        const int64_t nv = n / W;
        const V *__restrict__ av = (const V *)a;
        const V *__restrict__ bv = (const V *)b;
        for (int64_t v0 = (int64_t)blockIdx.x * kVNT * kVU + threadIdx.x; v0 < nv;
             v0 += (int64_t)gridDim.x * kVNT * kVU) {
            V as[kVU], bs[kVU];
#pragma unroll
            for (int u = 0; u < kVU; ++u) {
                const int64_t v = min(v0 + (int64_t)u * kVNT, nv - 1); // in range; sums masked
                as[u] = __builtin_nontemporal_load(&av[v]);
                bs[u] = __builtin_nontemporal_load(&bv[v]);
            }
#pragma unroll
            for (int u = 0; u < kVU; ++u)
                if (v0 + (int64_t)u * kVNT < nv)
#pragma unroll
                    for (int w = 0; w < W; ++w) s += (double)as[u][w] * (double)bs[u][w];
        }
        tail = nv * W;
    }
    for (int64_t i = tail + (int64_t)blockIdx.x * kVNT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVNT)
        s += (double)a[i] * (double)b[i];
    const double bs = block_sum<kVNT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

template <typename T>
static void dot_partials(int64_t n, const T *a, const T *b, double *parts, uint32_t g, hipStream_t s)
{
    if (al16(a) && al16(b))
        dot_kernel<T, true><<<g, kVNT, 0, s>>>(n, a, b, parts);
    else
        dot_kernel<T, false><<<g, kVNT, 0, s>>>(n, a, b, parts);
}

// *out = sum of the partials (single workgroup)
__global__ __launch_bounds__(kFinNT) void total_kernel(const double *__restrict__ partials,
                                                     int64_t nparts, double *out)
{
    __shared__ double red[kFinNT / kWave];
    const double t = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) *out = t;
}

mxs_status dot_launch(int64_t n, mxs_dtype t, const void *a, const void *b, double *result,
                      hipStream_t s)
{
    const uint32_t g = vec_grid(n);
    double *parts = nullptr;
    MXS_HIP(hipMallocAsync((void **)&parts, sizeof(double) * g, s));
    if (t == MXS_F64)
        dot_partials<double>(n, (const double *)a, (const double *)b, parts, g, s);
    else
        dot_partials<float>(n, (const float *)a, (const float *)b, parts, g, s);
    MXS_HIP(hipGetLastError());
    total_kernel<<<1, kFinNT, 0, s>>>(parts, g, result);
    MXS_HIP(hipGetLastError());
    MXS_HIP(hipFreeAsync(parts, s));
    return MXS_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free dot product (mxs_dot_noalloc): the same two kernels, with
// the workgroup partials in a fixed device array instead of a buffer
// allocated per call.  Every GPU the library runs on holds its own copy of
// the array, at its own address, until the process ends.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device, fetched once per
// device and kept.  Calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr int kScratchParts = 8192; // 64 KiB of FP64 partials per device
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchParts];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kScratchDevices] = {};

static mxs_status scratch_address(double **out)
{
    int dev = 0;
    MXS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        snprintf(g_last_error, sizeof g_last_error,
                 "mxs_dot_noalloc: device %d is beyond the %d devices the scratch table covers", dev,
                 kScratchDevices);
        return MXS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        MXS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MXS_OK;
}

mxs_status dot_noalloc_launch(int64_t n, mxs_dtype t, const void *a, const void *b, double *result,
                              hipStream_t s)
{
    const uint32_t g = vec_grid(n);
    if ((int64_t)g > kScratchParts) {
        snprintf(g_last_error, sizeof g_last_error,
                 "mxs_dot_noalloc: %u workgroup partials exceed the scratch array's %d", g,
                 kScratchParts);
        return MXS_ERR_UNSUPPORTED;
    }
    double *parts = nullptr;
    const mxs_status st = scratch_address(&parts);
    if (st != MXS_OK) return st;
    // every workgroup writes its own partial and the total reads exactly g:
    // nothing in the array needs clearing between calls
    if (t == MXS_F64)
        dot_partials<double>(n, (const double *)a, (const double *)b, parts, g, s);
    else
        dot_partials<float>(n, (const float *)a, (const float *)b, parts, g, s);
    MXS_HIP(hipGetLastError());
    total_kernel<<<1, kFinNT, 0, s>>>(parts, g, result);
    MXS_HIP(hipGetLastError());
    return MXS_OK;
}

template <typename T>
__global__ __launch_bounds__(kVNT) void axpby_kernel(int64_t n, T alpha, const T *__restrict__ x,
                                                     T beta, T *__restrict__ y)
{
    if (beta == T(0)) {
        VEC_LOOP(i, n) y[i] = alpha * x[i];
    } else {
        VEC_LOOP(i, n) y[i] = alpha * x[i] + beta * y[i];
    }
}

mxs_status axpby_launch(int64_t n, mxs_dtype t, double alpha, const void *x, double beta, void *y,
                        hipStream_t s)
{
    if (n == 0) return MXS_OK;
    if (t == MXS_F64)
        axpby_kernel<double><<<vec_grid(n), kVNT, 0, s>>>(n, alpha, (const double *)x, beta,
                                                          (double *)y);
    else
        axpby_kernel<float><<<vec_grid(n), kVNT, 0, s>>>(n, (float)alpha, (const float *)x,
                                                         (float)beta, (float *)y);
    return launch_status();
}

// ---------------------------------------------------------------------------
// CG kernels
// ---------------------------------------------------------------------------
__global__ void cg_state_init(CgState *st, double rtol, long long maxit)
{
    st->rho0 = st->rho = st->sigma = st->alpha = st->beta = st->rr = 0.0;
    st->rtol = rtol;
    st->iters = 0;
    st->maxit = maxit;
    st->done = 0;
    st->status = (int)MXS_NOT_CONVERGED;
    st->nonfinite = 0;
    st->pad = 0;
    st->rmax = st->delta = st->thresh = st->rtrue2 = 0.0;
    st->nupd = 0;
    st->noupd = 1;
    st->last = 0;
    st->rho_next = 0.0;
    st->rho_pend = 0;
    st->rmax_pend = 0;
    st->rmax_next = 0.0;
}

// r = b - q (q = A x0), p = r, partials of r.r; flags NaN/Inf in b or x0.
__global__ __launch_bounds__(kVNT) void cg_start_kernel(int64_t n, const double *__restrict__ b,
                                                        const double *__restrict__ x,
                                                        const double *__restrict__ q,
                                                        double *__restrict__ r,
                                                        double *__restrict__ p, double *partials,
                                                        CgState *st)
{
    __shared__ double red[kVNT / kWave];
    double s = 0.0;
    int bad = 0;
    VEC_LOOP(i, n)
    {
        const double bi = b[i], xi = x[i];
        if (!__builtin_isfinite(bi) || !__builtin_isfinite(xi)) bad = 1;
        const double ri = bi - q[i];
        r[i] = ri;
        p[i] = ri;
        s += ri * ri;
    }
    if (bad) atomicOr(&st->nonfinite, 1);
    const double bs = block_sum<kVNT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// rho0 = r0.r0; stops at once for NaN/Inf input or a zero residual.
__global__ __launch_bounds__(kFinNT) void start_finish_kernel(const double *__restrict__ partials,
                                                            int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    const double tot = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) {
        if (st->nonfinite) {
            st->status = (int)MXS_ERR_NONFINITE;
            st->done = 1;
        } else {
            st->rho0 = st->rho = st->rr = tot;
            if (tot == 0.0) {
                st->status = (int)MXS_OK;
                st->done = 1;
            }
        }
    }
}

// x += alpha p; r -= alpha q; with FUSED, partials of r.r.  VEC (all four
// vectors 16-byte aligned): each thread loads kVU 16-byte vectors of every
// array before any arithmetic, then the scalar tail of n mod (16/sizeof(T)).
// x (touched by no other kernel of the loop) and q (dead after this) go
// through non-temporal loads and stores, leaving the caches to p, r and
// the matrix (CG at 128^3: 22.87 -> 22.54 ms DIA).
template <typename T, bool FUSED, bool VEC>
__global__ __launch_bounds__(kVNT) void cg_xr_kernel(int64_t n, T *__restrict__ x,
                                                     T *__restrict__ r, const T *__restrict__ p,
                                                     const T *__restrict__ q, double *partials,
                                                     const CgState *st)
{
    __shared__ double red[kVNT / kWave];
    if (st->done) return;
    const T a = (T)st->alpha;
    const int64_t vb = vec_block<true>();
    double s = 0.0;
    int64_t tail = 0;
    if constexpr (VEC) {
        using V = V16<T>;
        constexpr int W = 16 / sizeof(T);
        const int64_t nv = n / W;
        V *__restrict__ xv = (V *)x;
        V *__restrict__ rv = (V *)r;
        const V *__restrict__ pv = (const V *)p;
        const V *__restrict__ qv = (const V *)q;
        for (int64_t v0 = vb * kVNT * kVU + threadIdx.x; v0 < nv;
             v0 += (int64_t)gridDim.x * kVNT * kVU) {
            V xs[kVU], rs[kVU], ps[kVU], qs[kVU];
#pragma unroll
            for (int u = 0; u < kVU; ++u) {
                const int64_t v = min(v0 + (int64_t)u * kVNT, nv - 1); // in range; stores masked
                xs[u] = __builtin_nontemporal_load(&xv[v]);
                rs[u] = rv[v];
                ps[u] = pv[v];
                qs[u] = __builtin_nontemporal_load(&qv[v]);
            }
#pragma unroll
            for (int u = 0; u < kVU; ++u) {
                const int64_t v = v0 + (int64_t)u * kVNT;
                if (v < nv) {
                    const V xn = xs[u] + a * ps[u];
                    const V rn = rs[u] - a * qs[u];
                    __builtin_nontemporal_store(xn, &xv[v]);
                    rv[v] = rn;
                    if (FUSED)
#pragma unroll
                        for (int w = 0; w < W; ++w) s += (double)rn[w] * (double)rn[w];
                }
            }
        }
        tail = nv * W;
    }
    for (int64_t i = tail + vb * kVNT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVNT) {
        const T xi = x[i] + a * p[i];
        const T ri = r[i] - a * q[i];
        x[i] = xi;
        r[i] = ri;
        if (FUSED) s += (double)ri * (double)ri;
    }
    if (FUSED) {
        const double bs = block_sum<kVNT>(s, red);
        if (threadIdx.x == 0) partials[vb] = bs;
    }
}

// partials of r.r on their own (the timed, unfused iteration).
template <typename T>
__global__ __launch_bounds__(kVNT) void cg_rr_kernel(int64_t n, const T *__restrict__ r,
                                                     double *partials, const CgState *st)
{
    __shared__ double red[kVNT / kWave];
    if (st->done) return;
    double s = 0.0;
    VEC_LOOP(i, n) s += (double)r[i] * (double)r[i];
    const double bs = block_sum<kVNT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// After r.r of the new residual: converged, capped, or beta for the next p.
__global__ __launch_bounds__(kFinNT) void rho_finish_kernel(const double *__restrict__ partials,
                                                          int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (st->done) return;
    const double rr = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (sqrt(rr) <= st->rtol * sqrt(st->rho0)) {
            st->status = (int)MXS_OK;
            st->done = 1;
        } else if (st->iters >= st->maxit) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        } else {
            st->beta = rr / st->rho;
        }
        st->rho = rr;
    }
}

// The end of a plain CG iteration in one launch: every workgroup sums the
// r.r partials of cg_xr_kernel (in index order, so every workgroup gets the
// same value), takes the convergence test and beta = r.r / rho, and updates
// p = r + beta p (not when converged or capped).  Workgroup 0 records the
// scalars; the new rho goes to rho_next (see CgState), since the other
// workgroups read rho during this launch.  The first step's vector loads are
// issued before the reduction so that their latency overlaps it.
template <typename T>
__global__ __launch_bounds__(kVNT) void cg_rho_p_kernel(int64_t n, const T *__restrict__ r,
                                                        T *__restrict__ p,
                                                        const double *__restrict__ partials,
                                                        int64_t nparts, CgState *st)
{
    __shared__ double red[kVNT / kWave];
    __shared__ double bc;
    if (st->done) return;
    const int64_t vb = vec_block<>();
    using V = V16<T>;
    constexpr int W = 16 / sizeof(T);
    const int64_t nv = n / W;
    const V *__restrict__ rv = (const V *)r;
    V *__restrict__ pv = (V *)p;
    const int64_t v0 = vb * kVNT * kVU + threadIdx.x;
    V rs[kVU], ps[kVU];
    if (v0 < nv) {
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = min(v0 + (int64_t)u * kVNT, nv - 1);
            rs[u] = rv[v];
            ps[u] = pv[v];
        }
    }
    const double rr0 = reduce_partials<kVNT>(partials, nparts, red);
    if (threadIdx.x == 0) bc = rr0;
    __syncthreads();
    const double rr = bc;
    const bool conv = sqrt(rr) <= st->rtol * sqrt(st->rho0);
    const bool cap = st->iters >= st->maxit;
    const double beta = rr / st->rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr = rr;
        st->rho_next = rr;
        st->rho_pend = 1;
        if (conv) {
            st->status = (int)MXS_OK;
            st->done = 1;
        } else if (cap) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        } else {
            st->beta = beta;
        }
    }
    if (conv || cap) return;
    const T b = (T)beta;
    if (v0 < nv) {
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = v0 + (int64_t)u * kVNT;
            if (v < nv) pv[v] = rs[u] + b * ps[u];
        }
    }
    for (int64_t w0 = v0 + (int64_t)gridDim.x * kVNT * kVU; w0 < nv; w0 += (int64_t)gridDim.x * kVNT * kVU) {
        V rt[kVU], pt[kVU];
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = min(w0 + (int64_t)u * kVNT, nv - 1);
            rt[u] = rv[v];
            pt[u] = pv[v];
        }
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = w0 + (int64_t)u * kVNT;
            if (v < nv) pv[v] = rt[u] + b * pt[u];
        }
    }
    for (int64_t i = nv * W + vb * kVNT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVNT)
        p[i] = r[i] + b * p[i];
}

// Up to this many r.r partials every workgroup of cg_rho_p_kernel sums them
// itself (measured: 10.0 us against 4.6 + 7.6 us for a finish kernel and the
// update at 1,024 partials, 30.8 against 4.6 + 25.1 us at 3,456).
constexpr uint32_t kFoldParts = 2048;

// p = r + beta p (r and p are workspace vectors: 16-byte aligned).
template <typename T>
__global__ __launch_bounds__(kVNT) void cg_p_kernel(int64_t n, const T *__restrict__ r,
                                                    T *__restrict__ p, const CgState *st)
{
    if (st->done) return;
    const T b = (T)st->beta;
    const int64_t vb = vec_block<>();
    using V = V16<T>;
    constexpr int W = 16 / sizeof(T);
    const int64_t nv = n / W;
    const V *__restrict__ rv = (const V *)r;
    V *__restrict__ pv = (V *)p;
    for (int64_t v0 = vb * kVNT * kVU + threadIdx.x; v0 < nv;
         v0 += (int64_t)gridDim.x * kVNT * kVU) {
        V rs[kVU], ps[kVU];
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = min(v0 + (int64_t)u * kVNT, nv - 1);
            rs[u] = rv[v];
            ps[u] = pv[v];
        }
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = v0 + (int64_t)u * kVNT;
            if (v < nv) pv[v] = rs[u] + b * ps[u];
        }
    }
    for (int64_t i = nv * W + vb * kVNT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVNT)
        p[i] = r[i] + b * p[i];
}

// ---------------------------------------------------------------------------
// PCG kernels (HPCG's preconditioned CG)
// ---------------------------------------------------------------------------
// partials of r.z
__global__ __launch_bounds__(kVNT) void pcg_rz_kernel(int64_t n, const double *__restrict__ r,
                                                      const double *__restrict__ z,
                                                      double *partials, const CgState *st)
{
    __shared__ double red[kVNT / kWave];
    if (st->done) return;
    double s = 0.0;
    VEC_LOOP(i, n) s += r[i] * z[i];
    const double bs = block_sum<kVNT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// beta = r.z / (previous r.z) (0 on the first iteration); rho = r.z, the
// numerator of the next alpha.  r.z <= 0 means the preconditioner is not
// positive definite: breakdown.
__global__ __launch_bounds__(kFinNT) void pcg_rz_finish_kernel(const double *__restrict__ partials,
                                                             int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (st->done) return;
    const double rz = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) {
        if (!(rz > 0.0) || !__builtin_isfinite(rz)) {
            st->status = (int)MXS_ERR_BREAKDOWN;
            st->done = 1;
        } else {
            st->beta = st->iters > 0 ? rz / st->rho : 0.0;
            st->rho = rz;
        }
    }
}

// p = z + beta p
__global__ __launch_bounds__(kVNT) void pcg_p_kernel(int64_t n, const double *__restrict__ z,
                                                     double *__restrict__ p, const CgState *st)
{
    if (st->done) return;
    const double b = st->beta;
    VEC_LOOP(i, n) p[i] = z[i] + b * p[i];
}

// After r.r of the new residual: converged or capped.
__global__ __launch_bounds__(kFinNT) void pcg_rr_finish_kernel(const double *__restrict__ partials,
                                                             int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (st->done) return;
    const double rr = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (sqrt(rr) <= st->rtol * sqrt(st->rho0)) {
            st->status = (int)MXS_OK;
            st->done = 1;
        } else if (st->iters >= st->maxit) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        }
    }
}

// partials of sum (a - c)^2 (c may be null); with w non-null also w = a - c.
__global__ __launch_bounds__(kVNT) void diff_norm2_kernel(int64_t n, const double *__restrict__ a,
                                                          const double *__restrict__ c,
                                                          double *__restrict__ w, double *partials)
{
    __shared__ double red[kVNT / kWave];
    double s = 0.0;
    VEC_LOOP(i, n)
    {
        const double v = c ? a[i] - c[i] : a[i];
        if (w) w[i] = v;
        s += v * v;
    }
    const double bs = block_sum<kVNT>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

__global__ __launch_bounds__(kVNT) void nonfinite_kernel(int64_t n, const double *__restrict__ a,
                                                         const double *__restrict__ b, int *flag)
{
    int bad = 0;
    VEC_LOOP(i, n)
    {
        if (!__builtin_isfinite(a[i]) || !__builtin_isfinite(b[i])) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

// Inner solve start: r32 = fp32(r / s); d = 0; p32 = r32; partials of r32.r32.
__global__ __launch_bounds__(kVNT) void ir_inner_start_kernel(int64_t n, const double *__restrict__ r,
                                                              double s, float *__restrict__ r32,
                                                              float *__restrict__ d32,
                                                              float *__restrict__ p32,
                                                              double *partials)
{
    __shared__ double red[kVNT / kWave];
    double acc = 0.0;
    VEC_LOOP(i, n)
    {
        const float v = (float)(r[i] / s);
        r32[i] = v;
        p32[i] = v;
        d32[i] = 0.0f;
        acc += (double)v * (double)v;
    }
    const double bs = block_sum<kVNT>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// x += s * fp64(d)
__global__ __launch_bounds__(kVNT) void ir_correct_kernel(int64_t n, double *__restrict__ x,
                                                          const float *__restrict__ d32, double s)
{
    VEC_LOOP(i, n) x[i] += s * (double)d32[i];
}

// ---------------------------------------------------------------------------
// Mixed CG with reliable updates: FP32 recurrences (A32 SpMV, FP32 vectors,
// FP64-accumulated dots) and a correction d accumulated in FP32; when the
// recursive residual falls to delta * (largest since the last update) or to
// rtol * ||b||, x += d in FP64 and the residual is recomputed as b - A x in
// FP64 and replaces the FP32 one, keeping the search direction (residual
// replacement, van der Vorst and Ye; the mixed precision named in Section I).
// The update kernels run every iteration but return at entry unless the
// finish kernel of that iteration asked for an update (st->noupd == 0).
// ---------------------------------------------------------------------------

// r = b - q (FP64); r32 = fp32(r); partials of r.r in [0, grid) and of
// r32.r32 in [grid, 2 grid).  START also sets p32 = r32, d32 = 0 and flags
// NaN/Inf in b or x.
template <bool START>
__global__ __launch_bounds__(kVNT) void ru_resid_kernel(int64_t n, const double *__restrict__ b,
                                                        const double *__restrict__ x,
                                                        const double *__restrict__ q,
                                                        float *__restrict__ r32,
                                                        float *__restrict__ p32,
                                                        float *__restrict__ d32, double *partials,
                                                        CgState *st)
{
    __shared__ double red[kVNT / kWave];
    if (!START && st->noupd) return;
    double s1 = 0.0, s2 = 0.0;
    int bad = 0;
    VEC_LOOP(i, n)
    {
        const double bi = b[i];
        if (START && (!__builtin_isfinite(bi) || !__builtin_isfinite(x[i]))) bad = 1;
        const double ri = bi - q[i];
        const float v = (float)ri;
        r32[i] = v;
        if (START) {
            p32[i] = v;
            d32[i] = 0.0f;
        }
        s1 += ri * ri;
        s2 += (double)v * (double)v;
    }
    if (START && bad) atomicOr(&st->nonfinite, 1);
    const double b1 = block_sum<kVNT>(s1, red);
    const double b2 = block_sum<kVNT>(s2, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = b1;
        partials[gridDim.x + blockIdx.x] = b2;
    }
}

// After a residual replacement: converged, stopped at the cap, or the
// recurrence continues from the new FP32 residual (beta, rho, rmax).
template <bool START>
__global__ __launch_bounds__(kFinNT) void ru_resid_finish_kernel(const double *__restrict__ partials,
                                                               int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (!START && st->noupd) return;
    const double rt2 = reduce_partials<kFinNT>(partials, nparts, red);
    const double r32sq = reduce_partials<kFinNT>(partials + nparts, nparts, red);
    if (threadIdx.x == 0) {
        st->rtrue2 = rt2;
        st->noupd = 1;
        if (START && st->nonfinite) {
            st->status = (int)MXS_ERR_NONFINITE;
            st->done = 1;
        } else if (sqrt(rt2) <= st->thresh) {
            st->status = (int)MXS_OK;
            st->done = 1;
        } else if (st->last) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        } else {
            if (START) st->rho0 = r32sq;
            else st->beta = r32sq / st->rho;
            st->rho = r32sq;
            st->rmax = sqrt(r32sq);
            st->done = 0;
        }
    }
}

// After r32.r32 of the new FP32 residual: ask for an update, stop at the
// cap, or take beta for the next direction.
__global__ __launch_bounds__(kFinNT) void ru_rho_finish_kernel(const double *__restrict__ partials,
                                                             int64_t nparts, CgState *st)
{
    __shared__ double red[kFinNT / kWave];
    if (st->done) return;
    const double rr = reduce_partials<kFinNT>(partials, nparts, red);
    if (threadIdx.x == 0) {
        const double rn = sqrt(rr);
        st->rr = rr;
        const bool cap = st->iters >= st->maxit;
        if (rn <= st->delta * st->rmax || rn <= st->thresh) {
            // update pending: done = 2 parks the iteration kernels until
            // the residual replacement has run (it resets done)
            st->noupd = 0;
            st->done = 2;
            st->last = cap ? 1 : 0;
            st->nupd += 1;
        } else if (cap) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        } else {
            if (rn > st->rmax) st->rmax = rn;
            st->beta = rr / st->rho;
            st->rho = rr;
        }
    }
}

// The end of a reliable-update step in one launch (as cg_rho_p_kernel for
// plain CG): every workgroup sums the r.r partials of the x/r update in
// index order, takes the same decision as ru_rho_finish_kernel (an update
// pending, the cap, or beta = r.r / rho) and, when the step goes on,
// updates p = r + beta p.  Workgroup 0 records the scalars; the new rho and
// rmax go to rho_next / rmax_next, moved in by the next p.q finish, since
// the other workgroups read rho and rmax during this launch.
__global__ __launch_bounds__(kVNT) void ru_rho_p_kernel(int64_t n, const float *__restrict__ r,
                                                        float *__restrict__ p,
                                                        const double *__restrict__ partials,
                                                        int64_t nparts, CgState *st)
{
    __shared__ double red[kVNT / kWave];
    __shared__ double bc;
    if (st->done) return;
    const int64_t vb = vec_block<>();
    using V = V16<float>;
    constexpr int W = 4;
    const int64_t nv = n / W;
    const V *__restrict__ rv = (const V *)r;
    V *__restrict__ pv = (V *)p;
    const int64_t v0 = vb * kVNT * kVU + threadIdx.x;
    V rs[kVU], ps[kVU];
    if (v0 < nv) {
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = min(v0 + (int64_t)u * kVNT, nv - 1);
            rs[u] = rv[v];
            ps[u] = pv[v];
        }
    }
    const double rr0 = reduce_partials<kVNT>(partials, nparts, red);
    if (threadIdx.x == 0) bc = rr0;
    __syncthreads();
    const double rr = bc, rn = sqrt(rr), rmax = st->rmax, rho = st->rho;
    const bool cap = st->iters >= st->maxit;
    const bool upd = rn <= st->delta * rmax || rn <= st->thresh;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr = rr;
        if (upd) {
            st->noupd = 0;
            st->done = 2;
            st->last = cap ? 1 : 0;
            st->nupd += 1;
        } else if (cap) {
            st->status = (int)MXS_NOT_CONVERGED;
            st->done = 1;
        } else {
            st->rmax_next = rn > rmax ? rn : rmax;
            st->rmax_pend = 1;
            st->beta = rr / rho;
            st->rho_next = rr;
            st->rho_pend = 1;
        }
    }
    if (upd || cap) return;
    const float b = (float)(rr / rho);
    if (v0 < nv) {
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = v0 + (int64_t)u * kVNT;
            if (v < nv) pv[v] = rs[u] + b * ps[u];
        }
    }
    for (int64_t w0 = v0 + (int64_t)gridDim.x * kVNT * kVU; w0 < nv; w0 += (int64_t)gridDim.x * kVNT * kVU) {
        V rt[kVU], pt[kVU];
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = min(w0 + (int64_t)u * kVNT, nv - 1);
            rt[u] = rv[v];
            pt[u] = pv[v];
        }
#pragma unroll
        for (int u = 0; u < kVU; ++u) {
            const int64_t v = w0 + (int64_t)u * kVNT;
            if (v < nv) pv[v] = rt[u] + b * pt[u];
        }
    }
    for (int64_t i = nv * W + vb * kVNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVNT)
        p[i] = r[i] + b * p[i];
}

// x += fp64(d); d = 0 -- when an update is pending, or always with FORCE
// (the final fold after the loop).
template <bool FORCE>
__global__ __launch_bounds__(kVNT) void ru_apply_kernel(int64_t n, double *__restrict__ x,
                                                        float *__restrict__ d32, const CgState *st)
{
    if (!FORCE && st->noupd) return;
    VEC_LOOP(i, n)
    {
        x[i] += (double)d32[i];
        d32[i] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

struct Ws {
    CgState *st, *st32;
    Aux *aux;
    double *parts;
    double *r, *p, *q, *z;
    float *d32, *r32, *p32, *q32;
};

// mixed: 0, 1, 2 as in mxs_cg_opts; 3: PCG (one more vector, z)
static size_t layout(int64_t n, int32_t mixed, char *base, Ws *w)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + o : nullptr;
        o += up256(bytes);
        return p;
    };
    Ws t;
    t.st = (CgState *)take(sizeof(CgState));
    t.st32 = (CgState *)take(sizeof(CgState));
    t.aux = (Aux *)take(sizeof(Aux));
    t.parts = (double *)take(sizeof(double) * (size_t)kMaxParts);
    t.r = (double *)take(sizeof(double) * (size_t)n);
    t.p = (double *)take(sizeof(double) * (size_t)n);
    t.q = (double *)take(sizeof(double) * (size_t)n);
    t.z = mixed == 3 ? (double *)take(sizeof(double) * (size_t)n) : nullptr;
    t.d32 = t.r32 = t.p32 = t.q32 = nullptr;
    if (mixed == 1 || mixed == 2) {
        t.d32 = (float *)take(sizeof(float) * (size_t)n);
        t.r32 = (float *)take(sizeof(float) * (size_t)n);
        t.p32 = (float *)take(sizeof(float) * (size_t)n);
        t.q32 = (float *)take(sizeof(float) * (size_t)n);
    }
    if (w) *w = t;
    return o;
}

size_t cg_workspace_bytes(int64_t n, int32_t mixed, int64_t, int64_t)
{
    return layout(n, mixed, nullptr, nullptr);
}

size_t pcg_workspace_bytes(int64_t n) { return layout(n, 3, nullptr, nullptr); }

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
namespace {

// Pinned host copy of a CgState, one per host thread (kept for the process).
CgState *pinned_state()
{
    thread_local CgState *p = nullptr;
    if (!p) {
        if (hipHostMalloc((void **)&p, sizeof(CgState) * 2, hipHostMallocPortable) != hipSuccess)
            p = nullptr;
    }
    return p;
}

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> ev; // marks: cls.size() + 1 per iteration
    size_t used = 0;
    double ms[4] = {0, 0, 0, 0}; // spmv, dot, vector updates, preconditioner
    std::vector<int> cls = {0, 1, 2}; // class of each interval of an iteration
    hipStream_t s = nullptr;

    mxs_status mark()
    {
        if (!on) return MXS_OK;
        if (used == ev.size()) {
            hipEvent_t e;
            MXS_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        MXS_HIP(hipEventRecord(ev[used++], s));
        return MXS_OK;
    }
    // After a synchronisation: fold the recorded intervals into the totals.
    mxs_status collect()
    {
        if (!on) return MXS_OK;
        const size_t k = cls.size();
        for (size_t i = 0; i + k < used; i += k + 1) {
            for (size_t j = 0; j < k; ++j) {
                float t;
                MXS_HIP(hipEventElapsedTime(&t, ev[i + j], ev[i + j + 1]));
                ms[cls[j]] += t;
            }
        }
        used = 0;
        return MXS_OK;
    }
    ~Timer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

template <typename T>
mxs_status enqueue_iteration(const mxs_mat_s *A, int64_t n, T *x, T *r, T *p, T *q, double *parts,
                             CgState *st, Timer &tm, hipStream_t s)
{
    mxs_status e;
    const DotSink ds{parts, st};
    const mxs_dtype dt = sizeof(T) == 8 ? MXS_F64 : MXS_F32;
    const uint32_t g = vec_grid(n, sizeof(T));
    // x is the caller's; the other vectors are in the workspace (aligned)
    auto xr = al16(x) ? cg_xr_kernel<T, true, true> : cg_xr_kernel<T, true, false>;
    if (!tm.on) {
        if ((e = spmv_launch(A, p, q, &st->done, &ds, s)) != MXS_OK) return e;
        xr<<<g, kVNT, 0, s>>>(n, x, r, p, q, parts, st);
        if (g <= kFoldParts) {
            cg_rho_p_kernel<T><<<g, kVNT, 0, s>>>(n, r, p, parts, g, st);
        } else {
            rho_finish_kernel<<<1, kFinNT, 0, s>>>(parts, g, st);
            cg_p_kernel<T><<<g, kVNT, 0, s>>>(n, r, p, st);
        }
        return launch_status();
    }
    // Timed iteration: the same steps unfused, one kernel class at a time.
    if ((e = tm.mark()) != MXS_OK) return e;
    if ((e = spmv_launch(A, p, q, &st->done, nullptr, s)) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    if ((e = dot_sigma_launch(n, dt, p, q, &st->done, &ds, s)) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    (al16(x) ? cg_xr_kernel<T, false, true> : cg_xr_kernel<T, false, false>)<<<g, kVNT, 0, s>>>(
        n, x, r, p, q, parts, st);
    cg_rr_kernel<T><<<g, kVNT, 0, s>>>(n, r, parts, st);
    rho_finish_kernel<<<1, kFinNT, 0, s>>>(parts, g, st);
    cg_p_kernel<T><<<g, kVNT, 0, s>>>(n, r, p, st);
    if ((e = launch_status()) != MXS_OK) return e;
    return tm.mark();
}

// Runs iterations (each enqueued by `iter`) until the device flag is set,
// reading the flag every `every` iterations; returns with the final state in
// *host.
template <typename Iter>
mxs_status run_loop(const CgState *st, int64_t maxit, int32_t every, Timer &tm, CgState *host,
                    hipStream_t s, Iter &&iter)
{
    const int64_t C = std::max<int32_t>(every, 1);
    MXS_HIP(hipMemcpyAsync(host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    int64_t launched = 0;
    while (!host->done && launched < maxit + C) {
        for (int64_t c = 0; c < C; ++c) {
            mxs_status e = iter();
            if (e != MXS_OK) return e;
        }
        launched += C;
        MXS_HIP(hipMemcpyAsync(host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        mxs_status e = tm.collect();
        if (e != MXS_OK) return e;
    }
    return MXS_OK;
}

// One reliable-update iteration as the timed solve runs it: the FP32 CG
// step, then the update kernels (no-ops unless this step asked for an
// update), then the next direction; the untimed solve runs enqueue_ru_step
// and, only when asked, enqueue_ru_update (the same kernels in the same
// order on the device).
mxs_status enqueue_ru_iteration(const mxs_mat_s *A, const mxs_mat_s *A32, int64_t n,
                                const double *b, double *x, double *q64, float *d32, float *r32,
                                float *p32, float *q32, double *parts, CgState *st, Timer &tm,
                                hipStream_t s)
{
    mxs_status e;
    const DotSink ds{parts, st};
    const uint32_t g = vec_grid(n);       // FP64 and mixed kernels
    const uint32_t g32 = vec_grid(n, 4);  // FP32 vector kernels
    if (tm.on) {
        if ((e = tm.mark()) != MXS_OK) return e;
        if ((e = spmv_launch(A32, p32, q32, &st->done, nullptr, s)) != MXS_OK) return e;
        if ((e = tm.mark()) != MXS_OK) return e;
        if ((e = dot_sigma_launch(n, MXS_F32, p32, q32, &st->done, &ds, s)) != MXS_OK) return e;
        if ((e = tm.mark()) != MXS_OK) return e;
    } else {
        if ((e = spmv_launch(A32, p32, q32, &st->done, &ds, s)) != MXS_OK) return e;
    }
    cg_xr_kernel<float, true, true><<<g32, kVNT, 0, s>>>(n, d32, r32, p32, q32, parts, st);
    ru_rho_finish_kernel<<<1, kFinNT, 0, s>>>(parts, g32, st);
    ru_apply_kernel<false><<<g, kVNT, 0, s>>>(n, x, d32, st);
    if ((e = launch_status()) != MXS_OK) return e;
    if ((e = spmv_launch(A, x, q64, &st->noupd, nullptr, s)) != MXS_OK) return e;
    ru_resid_kernel<false><<<g, kVNT, 0, s>>>(n, b, x, q64, r32, nullptr, nullptr, parts, st);
    ru_resid_finish_kernel<false><<<1, kFinNT, 0, s>>>(parts, g, st);
    cg_p_kernel<float><<<g32, kVNT, 0, s>>>(n, r32, p32, st);
    if ((e = launch_status()) != MXS_OK) return e;
    return tm.mark();
}

// The reliable-update loop without the update kernels in every iteration:
// one FP32 CG step (SpMV with p.q, x/r update, r.r finish, direction) ...
mxs_status enqueue_ru_step(const mxs_mat_s *A32, int64_t n, float *d32, float *r32, float *p32,
                           float *q32, double *parts, CgState *st, hipStream_t s)
{
    mxs_status e;
    const DotSink ds{parts, st};
    const uint32_t g32 = vec_grid(n, 4);
    if ((e = spmv_launch(A32, p32, q32, &st->done, &ds, s)) != MXS_OK) return e;
    cg_xr_kernel<float, true, true><<<g32, kVNT, 0, s>>>(n, d32, r32, p32, q32, parts, st);
    if (g32 <= kFoldParts) {
        ru_rho_p_kernel<<<g32, kVNT, 0, s>>>(n, r32, p32, parts, g32, st);
    } else {
        ru_rho_finish_kernel<<<1, kFinNT, 0, s>>>(parts, g32, st);
        cg_p_kernel<float><<<g32, kVNT, 0, s>>>(n, r32, p32, st);
    }
    return launch_status();
}

// ... and, enqueued by the host when a step left an update pending (done =
// 2; the steps after it returned at entry), the residual replacement and
// the direction update of the step that asked for it.
mxs_status enqueue_ru_update(const mxs_mat_s *A, int64_t n, const double *b, double *x, double *q64,
                             float *d32, float *r32, float *p32, double *parts, CgState *st,
                             hipStream_t s)
{
    mxs_status e;
    const uint32_t g = vec_grid(n);
    const uint32_t g32 = vec_grid(n, 4);
    ru_apply_kernel<false><<<g, kVNT, 0, s>>>(n, x, d32, st);
    if ((e = launch_status()) != MXS_OK) return e;
    if ((e = spmv_launch(A, x, q64, &st->noupd, nullptr, s)) != MXS_OK) return e;
    ru_resid_kernel<false><<<g, kVNT, 0, s>>>(n, b, x, q64, r32, nullptr, nullptr, parts, st);
    ru_resid_finish_kernel<false><<<1, kFinNT, 0, s>>>(parts, g, st);
    cg_p_kernel<float><<<g32, kVNT, 0, s>>>(n, r32, p32, st);
    return launch_status();
}

// Runs reliable-update steps in chunks of `every`, reading the state after
// each chunk: done = 1 ends the loop, done = 2 (an update pending) has the
// update enqueued before the next chunk.  A chunk that meets an update
// wastes its remaining steps (each returns at entry), against four
// launches per step saved on the steps without one.
template <typename Step, typename Upd>
mxs_status run_ru_loop(const CgState *st, int64_t maxit, int32_t every, CgState *host, hipStream_t s,
                       Step &&step, Upd &&upd)
{
    const int64_t C = std::max<int32_t>(every, 1);
    MXS_HIP(hipMemcpyAsync(host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    int64_t launched = 0, updates = 0;
    while (host->done != 1 && launched < maxit + C * (updates + 2)) {
        if (host->done == 2) {
            mxs_status e = upd();
            if (e != MXS_OK) return e;
            ++updates;
        }
        for (int64_t c = 0; c < C; ++c) {
            mxs_status e = step();
            if (e != MXS_OK) return e;
        }
        launched += C;
        MXS_HIP(hipMemcpyAsync(host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
    }
    return MXS_OK;
}

// ||a - c||^2 (c may be null; w = a - c when non-null) into *out.
mxs_status norm2(int64_t n, const double *a, const double *c, double *w, double *parts,
                 double *out, hipStream_t s)
{
    const uint32_t g = vec_grid(n);
    diff_norm2_kernel<<<g, kVNT, 0, s>>>(n, a, c, w, parts);
    total_kernel<<<1, kFinNT, 0, s>>>(parts, g, out);
    return launch_status();
}

}  // namespace

mxs_status cg_solve(const mxs_mat_s *A, const mxs_mat_s *A32, const double *b, double *x,
                    const mxs_cg_opts *o, mxs_cg_result *res, void *wsp, size_t bytes,
                    hipStream_t s)
{
    const int64_t n = A->nrows;
    *res = mxs_cg_result{};
    if (spmv_dot_parts(A) > kMaxParts || (A32 && spmv_dot_parts(A32) > kMaxParts))
        return MXS_ERR_UNSUPPORTED;
    if (layout(n, o->mixed, nullptr, nullptr) > bytes) return MXS_ERR_INVALID_ARG;
    Ws w;
    layout(n, o->mixed, (char *)wsp, &w);
    CgState *host = pinned_state();
    if (!host) return MXS_ERR_OUT_OF_MEMORY;
    Timer tm;
    tm.on = o->timing != 0;
    tm.s = s;
    const uint32_t g = vec_grid(n);
    mxs_status e;

    if (!o->mixed) {
        cg_state_init<<<1, 1, 0, s>>>(w.st, o->rtol, (long long)o->maxit);
        if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
        cg_start_kernel<<<g, kVNT, 0, s>>>(n, b, x, w.q, w.r, w.p, w.parts, w.st);
        start_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st);
        MXS_HIP(hipGetLastError());
        if (o->maxit > 0) {
            if ((e = run_loop(w.st, o->maxit, o->check_every, tm, host, s, [&] {
                     return enqueue_iteration<double>(A, n, x, w.r, w.p, w.q, w.parts, w.st, tm, s);
                 })) != MXS_OK)
                return e;
        } else {
            MXS_HIP(hipMemcpyAsync(host, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            MXS_HIP(hipStreamSynchronize(s));
        }
        const CgState f = *host;
        if (f.status == (int)MXS_ERR_NONFINITE) return MXS_ERR_NONFINITE;
        res->iters = f.iters;
        res->rel_resid = f.rho0 > 0.0 ? std::sqrt(f.rr) / std::sqrt(f.rho0) : 0.0;
        res->t_spmv_ms = tm.ms[0];
        res->t_dot_ms = tm.ms[1];
        res->t_axpy_ms = tm.ms[2];
        // true residual ||b - A x|| / ||b||
        if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
        if ((e = norm2(n, b, w.q, nullptr, w.parts, &w.aux->norm2[0], s)) != MXS_OK) return e;
        if ((e = norm2(n, b, nullptr, nullptr, w.parts, &w.aux->norm2[1], s)) != MXS_OK) return e;
        double nn[2];
        MXS_HIP(hipMemcpyAsync(nn, w.aux->norm2, sizeof(nn), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        res->true_rel_resid = nn[1] > 0.0 ? std::sqrt(nn[0]) / std::sqrt(nn[1]) : std::sqrt(nn[0]);
        if (f.status == (int)MXS_ERR_BREAKDOWN) return MXS_ERR_BREAKDOWN;
        return f.status == (int)MXS_OK ? MXS_OK : MXS_NOT_CONVERGED;
    }

    if (o->mixed == 2) {
        // ---- mixed precision with reliable updates ----
        if ((e = fill_bytes0(w.aux, sizeof(Aux), s)) != MXS_OK) return e;
        if ((e = norm2(n, b, nullptr, nullptr, w.parts, &w.aux->norm2[1], s)) != MXS_OK) return e;
        double b2;
        MXS_HIP(hipMemcpyAsync(&b2, &w.aux->norm2[1], sizeof(double), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        const double bn = std::sqrt(b2);
        CgState init{};
        init.rtol = o->rtol;
        init.maxit = (long long)o->maxit;
        init.status = (int)MXS_NOT_CONVERGED;
        init.delta = o->ru_delta;
        init.thresh = o->rtol * bn;
        init.noupd = 1;
        *host = init;
        MXS_HIP(hipMemcpyAsync(w.st32, host, sizeof(CgState), hipMemcpyHostToDevice, s));
        if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
        ru_resid_kernel<true><<<g, kVNT, 0, s>>>(n, b, x, w.q, w.r32, w.p32, w.d32, w.parts, w.st32);
        ru_resid_finish_kernel<true><<<1, kFinNT, 0, s>>>(w.parts, g, w.st32);
        MXS_HIP(hipGetLastError());
        if (o->maxit > 0 && tm.on) {
            // timed: every iteration with its (mostly idle) update kernels
            if ((e = run_loop(w.st32, o->maxit, o->check_every, tm, host, s, [&] {
                     return enqueue_ru_iteration(A, A32, n, b, x, w.q, w.d32, w.r32, w.p32, w.q32,
                                                 w.parts, w.st32, tm, s);
                 })) != MXS_OK)
                return e;
        } else if (o->maxit > 0) {
            if ((e = run_ru_loop(
                     w.st32, o->maxit, o->check_every, host, s,
                     [&] { return enqueue_ru_step(A32, n, w.d32, w.r32, w.p32, w.q32, w.parts, w.st32, s); },
                     [&] {
                         return enqueue_ru_update(A, n, b, x, w.q, w.d32, w.r32, w.p32, w.parts, w.st32, s);
                     })) != MXS_OK)
                return e;
        } else {
            MXS_HIP(hipMemcpyAsync(host, w.st32, sizeof(CgState), hipMemcpyDeviceToHost, s));
            MXS_HIP(hipStreamSynchronize(s));
        }
        const CgState f = *host;
        if (f.status == (int)MXS_ERR_NONFINITE) return MXS_ERR_NONFINITE;
        // fold in a correction not yet applied (cap or breakdown; zero otherwise)
        ru_apply_kernel<true><<<g, kVNT, 0, s>>>(n, x, w.d32, w.st32);
        MXS_HIP(hipGetLastError());
        if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
        if ((e = norm2(n, b, w.q, nullptr, w.parts, &w.aux->norm2[0], s)) != MXS_OK) return e;
        double r2;
        MXS_HIP(hipMemcpyAsync(&r2, &w.aux->norm2[0], sizeof(double), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        res->iters = f.iters;
        res->outer_iters = f.nupd;
        res->rel_resid = res->true_rel_resid = bn > 0.0 ? std::sqrt(r2) / bn : std::sqrt(r2);
        res->t_spmv_ms = tm.ms[0];
        res->t_dot_ms = tm.ms[1];
        res->t_axpy_ms = tm.ms[2];
        if (f.status == (int)MXS_ERR_BREAKDOWN) return MXS_ERR_BREAKDOWN;
        return f.status == (int)MXS_OK ? MXS_OK : MXS_NOT_CONVERGED;
    }

    // ---- mixed precision: FP64 residual and update, FP32 inner CG ----
    if ((e = fill_bytes0(w.aux, sizeof(Aux), s)) != MXS_OK) return e;
    nonfinite_kernel<<<g, kVNT, 0, s>>>(n, b, x, &w.aux->nonfinite);
    MXS_HIP(hipGetLastError());
    if ((e = norm2(n, b, nullptr, nullptr, w.parts, &w.aux->norm2[1], s)) != MXS_OK) return e;
    Aux ha;
    MXS_HIP(hipMemcpyAsync(&ha, w.aux, sizeof(Aux), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    if (ha.nonfinite) return MXS_ERR_NONFINITE;
    const double bn = std::sqrt(ha.norm2[1]);
    mxs_status status = MXS_NOT_CONVERGED;
    for (int32_t outer = 0;; ++outer) {
        if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
        if ((e = norm2(n, b, w.q, w.r, w.parts, &w.aux->norm2[0], s)) != MXS_OK) return e;
        double r2;
        MXS_HIP(hipMemcpyAsync(&r2, &w.aux->norm2[0], sizeof(double), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
        const double rn = std::sqrt(r2);
        res->rel_resid = res->true_rel_resid = bn > 0.0 ? rn / bn : rn;
        if (rn <= o->rtol * bn) {
            status = MXS_OK;
            break;
        }
        if (outer >= o->max_outer) break;
        cg_state_init<<<1, 1, 0, s>>>(w.st32, o->inner_rtol, (long long)o->maxit);
        ir_inner_start_kernel<<<g, kVNT, 0, s>>>(n, w.r, rn, w.r32, w.d32, w.p32, w.parts);
        start_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st32);
        MXS_HIP(hipGetLastError());
        if (o->maxit > 0) {
            if ((e = run_loop(w.st32, o->maxit, o->check_every, tm, host, s, [&] {
                     return enqueue_iteration<float>(A32, n, w.d32, w.r32, w.p32, w.q32, w.parts,
                                                     w.st32, tm, s);
                 })) != MXS_OK)
                return e;
            res->iters += host->iters;
        }
        ir_correct_kernel<<<g, kVNT, 0, s>>>(n, x, w.d32, rn);
        MXS_HIP(hipGetLastError());
        res->outer_iters += 1;
    }
    res->t_spmv_ms = tm.ms[0];
    res->t_dot_ms = tm.ms[1];
    res->t_axpy_ms = tm.ms[2];
    return status;
}

// ---------------------------------------------------------------------------
// PCG with the multigrid preconditioner, HPCG's recurrences: z = M^{-1} r,
// beta = r.z / (previous r.z), p = z + beta p, alpha = r.z / p.Ap,
// x += alpha p, r -= alpha Ap; stop on ||r|| <= rtol ||r_0||.
// ---------------------------------------------------------------------------
namespace {
mxs_status enqueue_pcg_iteration(const mxs_mg_s *M, const mxs_mat_s *A, int64_t n, double *x,
                                 const Ws &w, Timer &tm, hipStream_t s)
{
    mxs_status e;
    const DotSink ds{w.parts, w.st};
    const uint32_t g = vec_grid(n);
    if ((e = tm.mark()) != MXS_OK) return e;
    if ((e = mg_apply(M, w.r, w.z, &w.st->done, s)) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    pcg_rz_kernel<<<g, kVNT, 0, s>>>(n, w.r, w.z, w.parts, w.st);
    pcg_rz_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st);
    if ((e = tm.mark()) != MXS_OK) return e;
    pcg_p_kernel<<<g, kVNT, 0, s>>>(n, w.z, w.p, w.st);
    if ((e = launch_status()) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    if (!tm.on) {
        if ((e = spmv_launch(A, w.p, w.q, &w.st->done, &ds, s)) != MXS_OK) return e;
        (al16(x) ? cg_xr_kernel<double, true, true> : cg_xr_kernel<double, true, false>)<<<g, kVNT, 0, s>>>(
            n, x, w.r, w.p, w.q, w.parts, w.st);
        pcg_rr_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st);
        return launch_status();
    }
    // timed: the same steps unfused, one kernel class at a time
    if ((e = spmv_launch(A, w.p, w.q, &w.st->done, nullptr, s)) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    if ((e = dot_sigma_launch(n, MXS_F64, w.p, w.q, &w.st->done, &ds, s)) != MXS_OK) return e;
    if ((e = tm.mark()) != MXS_OK) return e;
    (al16(x) ? cg_xr_kernel<double, false, true> : cg_xr_kernel<double, false, false>)<<<g, kVNT, 0, s>>>(
        n, x, w.r, w.p, w.q, w.parts, w.st);
    cg_rr_kernel<double><<<g, kVNT, 0, s>>>(n, w.r, w.parts, w.st);
    pcg_rr_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st);
    if ((e = launch_status()) != MXS_OK) return e;
    return tm.mark();
}
}  // namespace

mxs_status pcg_solve(const mxs_mg_s *M, const mxs_mat_s *A, const double *b, double *x,
                     const mxs_cg_opts *o, mxs_cg_result *res, void *wsp, size_t bytes,
                     hipStream_t s)
{
    const int64_t n = A->nrows;
    *res = mxs_cg_result{};
    if (spmv_dot_parts(A) > kMaxParts) return MXS_ERR_UNSUPPORTED;
    if (layout(n, 3, nullptr, nullptr) > bytes) return MXS_ERR_INVALID_ARG;
    Ws w;
    layout(n, 3, (char *)wsp, &w);
    CgState *host = pinned_state();
    if (!host) return MXS_ERR_OUT_OF_MEMORY;
    Timer tm;
    tm.on = o->timing != 0;
    tm.s = s;
    // intervals: preconditioner, r.z, p update, SpMV, p.Ap, x/r updates and r.r
    tm.cls = {3, 1, 2, 0, 1, 2};
    const uint32_t g = vec_grid(n);
    mxs_status e;
    cg_state_init<<<1, 1, 0, s>>>(w.st, o->rtol, (long long)o->maxit);
    if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
    cg_start_kernel<<<g, kVNT, 0, s>>>(n, b, x, w.q, w.r, w.p, w.parts, w.st);
    start_finish_kernel<<<1, kFinNT, 0, s>>>(w.parts, g, w.st);
    MXS_HIP(hipGetLastError());
    if (o->maxit > 0) {
        if ((e = run_loop(w.st, o->maxit, o->check_every, tm, host, s,
                          [&] { return enqueue_pcg_iteration(M, A, n, x, w, tm, s); })) != MXS_OK)
            return e;
    } else {
        MXS_HIP(hipMemcpyAsync(host, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        MXS_HIP(hipStreamSynchronize(s));
    }
    const CgState f = *host;
    if (f.status == (int)MXS_ERR_NONFINITE) return MXS_ERR_NONFINITE;
    res->iters = f.iters;
    res->rel_resid = f.rho0 > 0.0 ? std::sqrt(f.rr) / std::sqrt(f.rho0) : 0.0;
    res->t_spmv_ms = tm.ms[0];
    res->t_dot_ms = tm.ms[1];
    res->t_axpy_ms = tm.ms[2];
    res->t_precond_ms = tm.ms[3];
    if ((e = spmv_launch(A, x, w.q, nullptr, nullptr, s)) != MXS_OK) return e;
    if ((e = norm2(n, b, w.q, nullptr, w.parts, &w.aux->norm2[0], s)) != MXS_OK) return e;
    if ((e = norm2(n, b, nullptr, nullptr, w.parts, &w.aux->norm2[1], s)) != MXS_OK) return e;
    double nn[2];
    MXS_HIP(hipMemcpyAsync(nn, w.aux->norm2, sizeof(nn), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    res->true_rel_resid = nn[1] > 0.0 ? std::sqrt(nn[0]) / std::sqrt(nn[1]) : std::sqrt(nn[0]);
    if (f.status == (int)MXS_ERR_BREAKDOWN) return MXS_ERR_BREAKDOWN;
    return f.status == (int)MXS_OK ? MXS_OK : MXS_NOT_CONVERGED;
}

}  // namespace mxs
