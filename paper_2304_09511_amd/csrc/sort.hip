// Sorting owned COO input into canonical (row, column) order (the containers
// are kept sorted, as Morpheus does before SpMV; Sections III-B and VII-B).
// A device radix sort of the combined key row*ncols + col carries the entry
// permutation; rows and columns are decoded from the sorted keys and values
// are gathered through the permutation.  The caller has already checked that
// every index is in range, so keys fit in ceil(log2(nrows*ncols)) bits.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <vector>

#include "common.h"

namespace mxs {

namespace {

__global__ void sort_keys_kernel(int64_t nnz, int32_t ncols, const int32_t *__restrict__ ai,
                                 const int32_t *__restrict__ aj, uint64_t *__restrict__ key,
                                 int32_t *__restrict__ perm)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        key[k] = (uint64_t)ai[k] * (uint64_t)ncols + (uint64_t)aj[k];
        perm[k] = (int32_t)k;
    }
}

template <typename T>
__global__ void sort_emit_kernel(int64_t nnz, int32_t ncols, const uint64_t *__restrict__ key,
                                 const int32_t *__restrict__ perm, const T *__restrict__ av_in,
                                 int32_t *__restrict__ ai, int32_t *__restrict__ aj,
                                 T *__restrict__ av_out)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t q = key[k];
        ai[k] = (int32_t)(q / (uint64_t)ncols);
        aj[k] = (int32_t)(q % (uint64_t)ncols);
        av_out[k] = av_in[perm[k]];
    }
}

uint32_t grid_for(int64_t n) { return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

int key_bits(int32_t nrows, int32_t ncols)
{
    const uint64_t span = (uint64_t)nrows * (uint64_t)ncols;
    int b = 1;
    while (b < 64 && (span - 1) >> b) ++b;
    return b;
}

}  // namespace

mxs_status sort_coo(int32_t nrows, int32_t ncols, int64_t nnz, int32_t *ai, int32_t *aj, void *av,
                    mxs_dtype dtype, hipStream_t s)
{
    if (nnz <= 1) return MXS_OK;
    const size_t vs = dsize(dtype);
    std::vector<void *> tmp;
    auto release = [&]() {
        for (void *p : tmp) (void)hipFreeAsync(p, s);
        (void)hipStreamSynchronize(s);
    };
    auto talloc = [&](size_t bytes, void **p) -> mxs_status {
        *p = nullptr;
        const hipError_t e = hipMallocAsync(p, std::max<size_t>(bytes, 256), s);
        if (e != hipSuccess) return note_hip_error(e, "hipMallocAsync (sort_coo)");
        tmp.push_back(*p);
        return MXS_OK;
    };
    void *k0, *k1, *p0, *p1, *vcopy, *scratch = nullptr;
    mxs_status st;
    if ((st = talloc(8 * nnz, &k0)) != MXS_OK || (st = talloc(8 * nnz, &k1)) != MXS_OK ||
        (st = talloc(4 * nnz, &p0)) != MXS_OK || (st = talloc(4 * nnz, &p1)) != MXS_OK ||
        (st = talloc(vs * nnz, &vcopy)) != MXS_OK)
        return release(), st;
    const int bits = key_bits(nrows, ncols);
    hipcub::DoubleBuffer<uint64_t> keys((uint64_t *)k0, (uint64_t *)k1);
    hipcub::DoubleBuffer<int32_t> vals((int32_t *)p0, (int32_t *)p1);
    size_t scratch_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, scratch_bytes, keys, vals, (int)nnz, 0,
                                                      bits, s);
    if (e != hipSuccess) return release(), note_hip_error(e, "DeviceRadixSort size (sort_coo)");
    if ((st = talloc(scratch_bytes, &scratch)) != MXS_OK) return release(), st;
    sort_keys_kernel<<<grid_for(nnz), 256, 0, s>>>(nnz, ncols, ai, aj, keys.Current(), vals.Current());
    if ((st = launch_status()) != MXS_OK) return release(), st;
    e = hipcub::DeviceRadixSort::SortPairs(scratch, scratch_bytes, keys, vals, (int)nnz, 0, bits, s);
    if (e != hipSuccess) return release(), note_hip_error(e, "DeviceRadixSort (sort_coo)");
    e = hipMemcpyAsync(vcopy, av, vs * nnz, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return release(), note_hip_error(e, "hipMemcpyAsync (sort_coo)");
    if (dtype == MXS_F64)
        sort_emit_kernel<double><<<grid_for(nnz), 256, 0, s>>>(nnz, ncols, keys.Current(), vals.Current(),
                                                               (const double *)vcopy, ai, aj, (double *)av);
    else
        sort_emit_kernel<float><<<grid_for(nnz), 256, 0, s>>>(nnz, ncols, keys.Current(), vals.Current(),
                                                              (const float *)vcopy, ai, aj, (float *)av);
    st = launch_status();
    release();
    return st;
}

}  // namespace mxs
