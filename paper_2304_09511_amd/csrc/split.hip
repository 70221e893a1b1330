// Split matrices: a DIA band plus a remainder in COO or CSR (the hybrid
// DIA/CSR format among the further formats of Section IX; the distributed
// HPCG runs of Section VII-D split each process's matrix into a local part
// and a remote part with separate formats, Table III).
//
// The band is the diagonals that hold at least one entry and at least
// min_fill times as many entries as they have slots inside the matrix (the
// comparison in FP64).  Entries on those diagonals go to the band, in the
// diagonal-major DIA layout with +0.0 in empty slots; all others keep their
// canonical order in the remainder.  y = A x runs the band's DIA kernel
// (which writes every row) and then the remainder's kernel in accumulate mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace mxs {

namespace {

#define SPLIT_LOOP(i, n)                                                          \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

uint32_t grid_of(int64_t n)
{
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

// count[j - i + nrows - 1] = entries on each diagonal.  A banded matrix has
// few distinct diagonals, so each workgroup first counts its chunk of
// entries in an LDS hash table keyed by diagonal (open addressing, a few
// probes) and then adds one total per diagonal to the global counts; entries
// that find no free slot are counted in global memory directly.
constexpr int kHashSlots = 1024;
constexpr int kHashProbes = 8;
constexpr int64_t kCountChunk = 16384; // entries per workgroup
constexpr uint32_t kHashEmpty = 0xffffffffu; // diagonal indices are below 2^32 - 1

__global__ __launch_bounds__(256) void split_count_kernel(int64_t nnz, int32_t nrows,
                                                          const int32_t *__restrict__ ai,
                                                          const int32_t *__restrict__ aj,
                                                          int32_t *__restrict__ count)
{
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ int32_t hcnt[kHashSlots];
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
        hkey[i] = kHashEmpty;
        hcnt[i] = 0;
    }
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * kCountChunk;
    const int64_t k1 = min(nnz, k0 + kCountChunk);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const uint32_t key = (uint32_t)((int64_t)aj[k] - ai[k] + nrows - 1);
        uint32_t slot = (key * 2654435761u) >> 22; // Fibonacci hashing to 10 bits
        bool done = false;
        for (int p = 0; p < kHashProbes && !done; ++p) {
            const uint32_t old = atomicCAS(&hkey[slot], kHashEmpty, key);
            if (old == kHashEmpty || old == key) {
                atomicAdd(&hcnt[slot], 1);
                done = true;
            }
            slot = (slot + 1) & (kHashSlots - 1);
        }
        if (!done) atomicAdd(&count[key], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x)
        if (hkey[i] != kHashEmpty) atomicAdd(&count[hkey[i]], hcnt[i]);
}

// keep[s] = 1 for band diagonals; *rest_nnz gets the entries of the others
__global__ void split_select_kernel(int64_t span, int32_t nrows, int32_t ncols,
                                    const int32_t *__restrict__ count, double min_fill,
                                    int32_t *__restrict__ keep, unsigned long long *rest_nnz)
{
    unsigned long long rest = 0;
    SPLIT_LOOP(s, span)
    {
        const int64_t d = s - (nrows - 1);
        const int64_t lo = d < 0 ? -d : 0;
        const int64_t hi = min((int64_t)nrows, (int64_t)ncols - d);
        const int32_t c = count[s];
        const int band = c > 0 && (double)c >= min_fill * (double)(hi - lo);
        keep[s] = band;
        if (!band) rest += (unsigned long long)c;
    }
    if (rest) atomicAdd(rest_nnz, rest);
}

// band_doff[map[s]] = offset of diagonal s, for the band diagonals
__global__ void split_offsets_kernel(int64_t span, int32_t nrows, const int32_t *__restrict__ keep,
                                     const int32_t *__restrict__ map, int32_t *__restrict__ doff)
{
    SPLIT_LOOP(s, span)
    if (keep[s]) doff[map[s]] = (int32_t)(s - (nrows - 1));
}

// Band values into place; remainder flags (1 = entry stays in the remainder).
template <typename T>
__global__ void split_band_kernel(int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai,
                                  const int32_t *__restrict__ aj, const T *__restrict__ av,
                                  const int32_t *__restrict__ keep, const int32_t *__restrict__ map,
                                  T *__restrict__ band, int32_t *__restrict__ rflag)
{
    SPLIT_LOOP(k, nnz)
    {
        const int32_t i = ai[k];
        const int64_t s = (int64_t)aj[k] - i + nrows - 1;
        if (keep[s]) {
            band[(int64_t)map[s] * nrows + i] = av[k];
            rflag[k] = 0;
        } else {
            rflag[k] = 1;
        }
    }
}

// Remainder entries to their compacted positions (canonical order kept).
template <typename T>
__global__ void split_rest_kernel(int64_t nnz, const int32_t *__restrict__ ai,
                                  const int32_t *__restrict__ aj, const T *__restrict__ av,
                                  const int32_t *__restrict__ rflag, const int32_t *__restrict__ pos,
                                  int32_t *__restrict__ rai, int32_t *__restrict__ raj,
                                  T *__restrict__ rav)
{
    SPLIT_LOOP(k, nnz)
    {
        if (rflag[k]) {
            const int32_t p = pos[k];
            rai[p] = ai[k];
            raj[p] = aj[k];
            rav[p] = av[k];
        }
    }
}

template <typename T>
__global__ void split_zero_kernel(T *__restrict__ p, int64_t n)
{
    SPLIT_LOOP(i, n) p[i] = T(0);
}

// Scratch of a split: per-diagonal counts, band flags and band positions.
struct SplitMap {
    int64_t span = 0;
    int32_t *count = nullptr, *keep = nullptr, *map = nullptr;
    unsigned long long *rest = nullptr;
    int32_t ndiag = 0;
    int64_t rest_nnz = 0;
    hipStream_t s = nullptr;
    ~SplitMap()
    {
        for (void *p : {(void *)count, (void *)keep, (void *)map, (void *)rest})
            if (p) (void)hipFreeAsync(p, s);
        (void)hipStreamSynchronize(s);
    }
};

// The row ids of A's entries (CSR: expanded into *tmp, which the caller frees).
mxs_status row_ids(const mxs_mat_s *A, const int32_t **ai, int32_t **tmp, hipStream_t s)
{
    *tmp = nullptr;
    if (A->fmt == MXS_COO) {
        *ai = A->idx0;
        return MXS_OK;
    }
    MXS_HIP(hipMallocAsync((void **)tmp, sizeof(int32_t) * (size_t)std::max<int64_t>(A->nnz, 1), s));
    *ai = *tmp;
    return csr_row_index(A->idx0, A->nrows, A->nnz, *tmp, s);
}

mxs_status build_map(const mxs_mat_s *A, const int32_t *ai, double min_fill, SplitMap *m,
                     hipStream_t s)
{
    m->s = s;
    m->span = (int64_t)A->nrows + A->ncols - 1;
    if (m->span <= 0 || A->nnz == 0) return MXS_OK;
    MXS_HIP(hipMallocAsync((void **)&m->count, sizeof(int32_t) * (size_t)m->span, s));
    MXS_HIP(hipMallocAsync((void **)&m->keep, sizeof(int32_t) * (size_t)m->span, s));
    MXS_HIP(hipMallocAsync((void **)&m->map, sizeof(int32_t) * ((size_t)m->span + 1), s));
    MXS_HIP(hipMallocAsync((void **)&m->rest, sizeof(unsigned long long), s));
    mxs_status st = fill_i32(m->count, 0, m->span, s);
    if (st == MXS_OK) st = fill_bytes0(m->rest, sizeof(unsigned long long), s);
    if (st != MXS_OK) return st;
    split_count_kernel<<<(uint32_t)((A->nnz + kCountChunk - 1) / kCountChunk), 256, 0, s>>>(
        A->nnz, A->nrows, ai, A->idx1, m->count);
    split_select_kernel<<<grid_of(m->span), 256, 0, s>>>(m->span, A->nrows, A->ncols, m->count,
                                                         min_fill, m->keep, m->rest);
    if ((st = launch_status()) != MXS_OK) return st;
    if ((st = scan_i32(m->keep, m->map, m->span, s)) != MXS_OK) return st; // syncs
    unsigned long long rest = 0;
    MXS_HIP(hipMemcpyAsync(&m->ndiag, m->map + m->span, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipMemcpyAsync(&rest, m->rest, sizeof(rest), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    m->rest_nnz = (int64_t)rest;
    return MXS_OK;
}

template <typename T>
mxs_status split_fill(const mxs_mat_s *A, const int32_t *ai, const SplitMap &m, int32_t *doff,
                      T *band, int32_t *rai, int32_t *raj, T *rav, hipStream_t s)
{
    const int64_t n = A->nnz;
    if (m.ndiag > 0) {
        split_offsets_kernel<<<grid_of(m.span), 256, 0, s>>>(m.span, A->nrows, m.keep, m.map, doff);
        const int64_t slots = (int64_t)m.ndiag * A->nrows;
        split_zero_kernel<T><<<grid_of(slots), 256, 0, s>>>(band, slots);
        mxs_status st = launch_status();
        if (st != MXS_OK) return st;
    }
    if (n == 0) return MXS_OK;
    int32_t *rflag = nullptr, *pos = nullptr;
    MXS_HIP(hipMallocAsync((void **)&rflag, sizeof(int32_t) * (size_t)n, s));
    MXS_HIP(hipMallocAsync((void **)&pos, sizeof(int32_t) * ((size_t)n + 1), s));
    split_band_kernel<T><<<grid_of(n), 256, 0, s>>>(n, A->nrows, ai, A->idx1, (const T *)A->vals,
                                                    m.keep, m.map, band, rflag);
    mxs_status st = launch_status();
    if (st == MXS_OK) st = scan_i32(rflag, pos, n, s); // syncs
    if (st == MXS_OK && m.rest_nnz > 0) {
        split_rest_kernel<T><<<grid_of(n), 256, 0, s>>>(n, ai, A->idx1, (const T *)A->vals, rflag,
                                                        pos, rai, raj, rav);
        st = launch_status();
    }
    (void)hipFreeAsync(rflag, s);
    (void)hipFreeAsync(pos, s);
    MXS_HIP(hipStreamSynchronize(s));
    return st;
}

}  // namespace

mxs_status split_size(const mxs_mat_s *A, double min_fill, int32_t *band_ndiag, int64_t *rest_nnz,
                      hipStream_t s)
{
    const int32_t *ai = nullptr;
    int32_t *tmp = nullptr;
    mxs_status st = row_ids(A, &ai, &tmp, s);
    SplitMap m;
    if (st == MXS_OK) st = build_map(A, ai, min_fill, &m, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (st != MXS_OK) return st;
    *band_ndiag = m.ndiag;
    *rest_nnz = A->nnz == 0 ? 0 : m.rest_nnz;
    return MXS_OK;
}


mxs_status split(const mxs_mat_s *A, double min_fill, mxs_format rest_fmt, int32_t *band_doff,
                 void *band_vals, int32_t *rest_idx0, int32_t *rest_idx1, void *rest_vals,
                 mxs_mat_s **out, hipStream_t s)
{
    const int32_t *ai = nullptr;
    int32_t *tmp = nullptr, *rai_tmp = nullptr;
    mxs_status st = row_ids(A, &ai, &tmp, s);
    SplitMap m;
    if (st == MXS_OK) st = build_map(A, ai, min_fill, &m, s);
    const int64_t rest_nnz = A->nnz == 0 ? 0 : m.rest_nnz;
    // the remainder's row ids: the caller's array (COO) or scratch (CSR)
    int32_t *rai = rest_idx0;
    if (st == MXS_OK && rest_fmt == MXS_CSR && rest_nnz > 0) {
        if (hipMallocAsync((void **)&rai_tmp, sizeof(int32_t) * (size_t)rest_nnz, s) != hipSuccess)
            st = MXS_ERR_OUT_OF_MEMORY;
        rai = rai_tmp;
    }
    if (st == MXS_OK) {
        if (A->dtype == MXS_F64)
            st = split_fill<double>(A, ai, m, band_doff, (double *)band_vals, rai, rest_idx1,
                                    (double *)rest_vals, s);
        else
            st = split_fill<float>(A, ai, m, band_doff, (float *)band_vals, rai, rest_idx1,
                                   (float *)rest_vals, s);
    }
    if (st == MXS_OK && rest_fmt == MXS_CSR)
        st = coo_irp_launch(rest_nnz, A->nrows, rai, rest_idx0, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (rai_tmp) (void)hipFreeAsync(rai_tmp, s);
    if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
    if (st != MXS_OK) return st;

    auto *band = new mxs_mat_s;
    band->fmt = MXS_DIA;
    band->dtype = A->dtype;
    band->nrows = A->nrows;
    band->ncols = A->ncols;
    band->ndiag = m.ndiag;
    band->idx0 = band_doff;
    band->vals = band_vals;
    band->device = A->device;
    if ((st = dia_slot_count(band, &band->nnz, s)) != MXS_OK) {
        delete band;
        return st;
    }
    auto *rest = new mxs_mat_s;
    rest->fmt = rest_fmt;
    rest->dtype = A->dtype;
    rest->nrows = A->nrows;
    rest->ncols = A->ncols;
    rest->nnz = rest_nnz;
    rest->idx0 = rest_idx0;
    rest->idx1 = rest_idx1;
    rest->vals = rest_vals;
    rest->device = A->device;
    auto *h = new mxs_mat_s;
    h->fmt = MXS_HDC;
    h->dtype = A->dtype;
    h->nrows = A->nrows;
    h->ncols = A->ncols;
    h->nnz = band->nnz + rest_nnz;
    h->ndiag = m.ndiag;
    h->device = A->device;
    band->part = rest->part = true;
    band->sub = rest->sub = true;
    h->band = band;
    h->rest = rest;
    *out = h;
    return MXS_OK;
}

}  // namespace mxs
