// Validation of the three containers and conversions between them
// (Section III-B definitions; the runtime format switching of Sections I-II).
// Every conversion moves values without arithmetic, so its output is
// bit-exact; outputs are canonical (rows ascending, columns ascending within
// a row, DIA offsets ascending with +0.0 in empty slots).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace mxs {

static uint32_t grid1d(int64_t n, int nt = 256, int64_t cap = 65536)
{
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + nt - 1) / nt, cap));
}

#define GRID_STRIDE(i, n)                                                          \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

enum { F_RANGE = 1, F_UNSORTED = 2, F_DUP = 4 };

static mxs_status flags_status(int f)
{
    if (f & F_RANGE) return MXS_ERR_INDEX_RANGE;
    if (f & F_UNSORTED) return MXS_ERR_UNSORTED;
    if (f & F_DUP) return MXS_ERR_DUPLICATE;
    return MXS_OK;
}

// ---------------------------------------------------------------------------
// COO check: range, then (row, col) order, then duplicates
// ---------------------------------------------------------------------------
__global__ void coo_check_kernel(int64_t nnz, int32_t nrows, int32_t ncols,
                                 const int32_t *__restrict__ ai, const int32_t *__restrict__ aj,
                                 int *__restrict__ flags)
{
    int f = 0;
    GRID_STRIDE(k, nnz)
    {
        const int32_t r = ai[k], c = aj[k];
        if (r < 0 || r >= nrows || c < 0 || c >= ncols) f |= F_RANGE;
        if (k > 0) {
            const int32_t pr = ai[k - 1], pc = aj[k - 1];
            if (r < pr || (r == pr && c < pc)) f |= F_UNSORTED;
            else if (r == pr && c == pc) f |= F_DUP;
        }
    }
    if (f) atomicOr(flags, f);
}

static mxs_status read_flags(int *dflags, hipStream_t s, int *out)
{
    MXS_HIP(hipMemcpyAsync(out, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipFreeAsync(dflags, s));
    MXS_HIP(hipStreamSynchronize(s));
    return MXS_OK;
}

static mxs_status alloc_flags(int **d, hipStream_t s)
{
    MXS_HIP(hipMallocAsync((void **)d, sizeof(int), s));
    return fill_i32(*d, 0, 1, s);
}

mxs_status check_coo(const mxs_mat_s *A, hipStream_t s)
{
    if (A->nnz == 0) return MXS_OK;
    int *d = nullptr;
    mxs_status st = alloc_flags(&d, s);
    if (st != MXS_OK) return st;
    coo_check_kernel<<<grid1d(A->nnz), 256, 0, s>>>(A->nnz, A->nrows, A->ncols, A->idx0, A->idx1, d);
    MXS_HIP(hipGetLastError());
    int f = 0;
    st = read_flags(d, s, &f);
    return st != MXS_OK ? st : flags_status(f);
}

// ---------------------------------------------------------------------------
// CSR check: row pointers first (so that entry checks stay in bounds), then
// columns in range and strictly ascending within each row.
// ---------------------------------------------------------------------------
__global__ void csr_irp_check_kernel(int32_t nrows, int64_t nnz, const int32_t *__restrict__ irp,
                                     int *__restrict__ flags)
{
    int f = 0;
    GRID_STRIDE(r, (int64_t)nrows + 1)
    {
        const int32_t v = irp[r];
        if (r == 0 && v != 0) f |= F_RANGE;
        if (r == nrows && v != nnz) f |= F_RANGE;
        if (r > 0 && v < irp[r - 1]) f |= F_RANGE;
    }
    if (f) atomicOr(flags, f);
}

__global__ void mark_row_starts(int32_t nrows, const int32_t *__restrict__ irp,
                                uint8_t *__restrict__ start)
{
    GRID_STRIDE(r, nrows)
    {
        if (irp[r + 1] > irp[r]) start[irp[r]] = 1;
    }
}

__global__ void csr_entry_check_kernel(int64_t nnz, int32_t ncols, const int32_t *__restrict__ aj,
                                       const uint8_t *__restrict__ start, int *__restrict__ flags)
{
    int f = 0;
    GRID_STRIDE(k, nnz)
    {
        const int32_t c = aj[k];
        if (c < 0 || c >= ncols) f |= F_RANGE;
        if (k > 0 && !start[k]) {
            const int32_t pc = aj[k - 1];
            if (c < pc) f |= F_UNSORTED;
            else if (c == pc) f |= F_DUP;
        }
    }
    if (f) atomicOr(flags, f);
}

mxs_status check_csr(const mxs_mat_s *A, hipStream_t s)
{
    int *d = nullptr;
    mxs_status st = alloc_flags(&d, s);
    if (st != MXS_OK) return st;
    csr_irp_check_kernel<<<grid1d((int64_t)A->nrows + 1), 256, 0, s>>>(A->nrows, A->nnz, A->idx0, d);
    MXS_HIP(hipGetLastError());
    int f = 0;
    if ((st = read_flags(d, s, &f)) != MXS_OK) return st;
    if (f) return flags_status(f);
    if (A->nnz == 0) return MXS_OK;
    uint8_t *start = nullptr;
    MXS_HIP(hipMallocAsync((void **)&start, (size_t)((A->nnz + 3) / 4) * 4, s));
    if ((st = fill_bytes0(start, (size_t)((A->nnz + 3) / 4) * 4, s)) != MXS_OK) return st;
    mark_row_starts<<<grid1d(A->nrows), 256, 0, s>>>(A->nrows, A->idx0, start);
    MXS_HIP(hipGetLastError());
    if ((st = alloc_flags(&d, s)) != MXS_OK) return st;
    csr_entry_check_kernel<<<grid1d(A->nnz), 256, 0, s>>>(A->nnz, A->ncols, A->idx1, start, d);
    MXS_HIP(hipGetLastError());
    MXS_HIP(hipFreeAsync(start, s));
    if ((st = read_flags(d, s, &f)) != MXS_OK) return st;
    return flags_status(f);
}

// ---------------------------------------------------------------------------
// DIA: offsets are few, so they are checked on the host.
// ---------------------------------------------------------------------------
static int64_t offset_slots(int64_t nrows, int64_t ncols, int64_t off)
{
    // rows i in [0, nrows) with 0 <= i + off < ncols
    const int64_t lo = std::max<int64_t>(0, -off);
    const int64_t hi = std::min<int64_t>(nrows, ncols - off);
    return std::max<int64_t>(0, hi - lo);
}

mxs_status check_dia(const mxs_mat_s *A, hipStream_t s)
{
    if (A->ndiag == 0) return MXS_OK;
    std::vector<int32_t> h(A->ndiag);
    MXS_HIP(hipMemcpyAsync(h.data(), A->idx0, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    for (size_t d = 0; d < h.size(); ++d) {
        if (h[d] < -(int64_t)(A->nrows - 1) || h[d] > (int64_t)A->ncols - 1)
            return MXS_ERR_INDEX_RANGE;
    }
    for (size_t d = 1; d < h.size(); ++d)
        if (h[d] <= h[d - 1]) return MXS_ERR_UNSORTED;
    return MXS_OK;
}

mxs_status dia_slot_count(const mxs_mat_s *A, int64_t *slots, hipStream_t s)
{
    *slots = 0;
    if (A->ndiag == 0) return MXS_OK;
    std::vector<int32_t> h(A->ndiag);
    MXS_HIP(hipMemcpyAsync(h.data(), A->idx0, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    int64_t c = 0;
    for (int32_t o : h) c += offset_slots(A->nrows, A->ncols, o);
    *slots = c;
    return MXS_OK;
}

// ---------------------------------------------------------------------------
// COO <-> CSR
// ---------------------------------------------------------------------------
// irp[r] = number of entries with row < r: for each k in [0, nnz] the rows
// (ai[k-1], ai[k]] start at k (ai[-1] = -1, ai[nnz] = nrows).
__global__ void coo_to_irp_kernel(int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai,
                                  int32_t *__restrict__ irp)
{
    GRID_STRIDE(k, nnz + 1)
    {
        const int32_t lo = k == 0 ? -1 : ai[k - 1];
        const int32_t hi = k == nnz ? nrows : ai[k];
        for (int32_t r = lo + 1; r <= hi; ++r) irp[r] = (int32_t)k;
    }
}

mxs_status coo_irp_launch(int64_t nnz, int32_t nrows, const int32_t *ai, int32_t *irp,
                          hipStream_t s)
{
    coo_to_irp_kernel<<<grid1d(nnz + 1), 256, 0, s>>>(nnz, nrows, ai, irp);
    return launch_status();
}

__global__ void csr_to_ai_kernel(int32_t nrows, const int32_t *__restrict__ irp,
                                 int32_t *__restrict__ ai)
{
    GRID_STRIDE(r, nrows)
    {
        const int32_t e = irp[r + 1];
        for (int32_t k = irp[r]; k < e; ++k) ai[k] = (int32_t)r;
    }
}

mxs_status csr_row_index(const int32_t *irp, int32_t nrows, int64_t nnz, int32_t *ai, hipStream_t s)
{
    if (nnz == 0 || nrows == 0) return MXS_OK;
    csr_to_ai_kernel<<<grid1d(nrows), 256, 0, s>>>(nrows, irp, ai);
    return launch_status();
}

// ---------------------------------------------------------------------------
// -> DIA
// ---------------------------------------------------------------------------
__global__ void dia_flag_kernel(int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai,
                                const int32_t *__restrict__ aj, int32_t *__restrict__ flag)
{
    GRID_STRIDE(k, nnz)
    {
        flag[(int64_t)aj[k] - ai[k] + nrows - 1] = 1;
    }
}

__global__ void dia_offsets_kernel(int64_t span, int32_t nrows, const int32_t *__restrict__ flag,
                                   const int32_t *__restrict__ map, int32_t *__restrict__ doff)
{
    GRID_STRIDE(i, span)
    {
        if (flag[i]) doff[map[i]] = (int32_t)(i - (nrows - 1));
    }
}

template <typename T>
__global__ void dia_scatter_kernel(int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai,
                                   const int32_t *__restrict__ aj, const T *__restrict__ av,
                                   const int32_t *__restrict__ map, T *__restrict__ out)
{
    GRID_STRIDE(k, nnz)
    {
        const int32_t r = ai[k];
        const int64_t d = map[(int64_t)aj[k] - r + nrows - 1];
        out[d * nrows + r] = av[k];
    }
}

// Row indices of a COO/CSR source (borrowed for COO, a temporary for CSR).
static mxs_status source_rows(const mxs_mat_s *A, const int32_t **ai, int32_t **tmp, hipStream_t s)
{
    *tmp = nullptr;
    if (A->fmt == MXS_COO) {
        *ai = A->idx0;
        return MXS_OK;
    }
    MXS_HIP(hipMallocAsync((void **)tmp, sizeof(int32_t) * (size_t)std::max<int64_t>(A->nnz, 1), s));
    mxs_status st = csr_row_index(A->idx0, A->nrows, A->nnz, *tmp, s);
    *ai = *tmp;
    return st;
}

// Offset flags over the 2N-1 candidate diagonals and their prefix sum.
struct DiaMap {
    int32_t *flag = nullptr, *map = nullptr;
    int64_t span = 0;
    int32_t ndiag = 0;
};

static mxs_status build_dia_map(const mxs_mat_s *A, const int32_t *ai, DiaMap *m, hipStream_t s)
{
    m->span = (int64_t)A->nrows + A->ncols - 1;
    if (m->span <= 0 || A->nnz == 0) {
        m->ndiag = 0;
        return MXS_OK;
    }
    MXS_HIP(hipMallocAsync((void **)&m->flag, sizeof(int32_t) * (size_t)m->span, s));
    MXS_HIP(hipMallocAsync((void **)&m->map, sizeof(int32_t) * ((size_t)m->span + 1), s));
    mxs_status st = fill_i32(m->flag, 0, m->span, s);
    if (st != MXS_OK) return st;
    dia_flag_kernel<<<grid1d(A->nnz), 256, 0, s>>>(A->nnz, A->nrows, ai, A->idx1, m->flag);
    MXS_HIP(hipGetLastError());
    if ((st = scan_i32(m->flag, m->map, m->span, s)) != MXS_OK) return st; // syncs
    MXS_HIP(hipMemcpyAsync(&m->ndiag, m->map + m->span, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipStreamSynchronize(s));
    return MXS_OK;
}

static void free_dia_map(DiaMap *m, hipStream_t s)
{
    if (m->flag) (void)hipFreeAsync(m->flag, s);
    if (m->map) (void)hipFreeAsync(m->map, s);
    m->flag = m->map = nullptr;
}

// ---------------------------------------------------------------------------
// DIA -> COO/CSR
// ---------------------------------------------------------------------------
template <typename T>
__global__ void dia_row_count_kernel(int32_t nrows, int32_t ncols, int32_t ndiag,
                                     const int32_t *__restrict__ doff, const T *__restrict__ av,
                                     int32_t *__restrict__ cnt)
{
    GRID_STRIDE(i, nrows)
    {
        int32_t c = 0;
        for (int d = 0; d < ndiag; ++d) {
            const int64_t k = i + (int64_t)doff[d];
            if (k >= 0 && k < ncols && av[(int64_t)d * nrows + i] != T(0)) ++c;
        }
        cnt[i] = c;
    }
}

template <typename T>
__global__ void dia_emit_kernel(int32_t nrows, int32_t ncols, int32_t ndiag,
                                const int32_t *__restrict__ doff, const T *__restrict__ av,
                                const int32_t *__restrict__ pos, int32_t *__restrict__ ai,
                                int32_t *__restrict__ aj, T *__restrict__ out)
{
    GRID_STRIDE(i, nrows)
    {
        int32_t p = pos[i];
        for (int d = 0; d < ndiag; ++d) {
            const int64_t k = i + (int64_t)doff[d];
            if (k < 0 || k >= ncols) continue;
            const T v = av[(int64_t)d * nrows + i];
            if (v != T(0)) {
                if (ai) ai[p] = (int32_t)i;
                aj[p] = (int32_t)k;
                out[p] = v;
                ++p;
            }
        }
    }
}

template <typename T>
static mxs_status dia_counts(const mxs_mat_s *A, int32_t *pos, hipStream_t s)
{
    int32_t *cnt = nullptr;
    MXS_HIP(hipMallocAsync((void **)&cnt, sizeof(int32_t) * (size_t)std::max(A->nrows, 1), s));
    if (A->nrows > 0) {
        dia_row_count_kernel<T><<<grid1d(A->nrows), 256, 0, s>>>(A->nrows, A->ncols, A->ndiag,
                                                                 A->idx0, (const T *)A->vals, cnt);
        MXS_HIP(hipGetLastError());
    }
    mxs_status st = scan_i32(cnt, pos, A->nrows, s);
    MXS_HIP(hipFreeAsync(cnt, s));
    return st;
}

// ---------------------------------------------------------------------------
// Sizes and conversion drivers
// ---------------------------------------------------------------------------
mxs_status convert_size(const mxs_mat_s *A, mxs_format dst, int64_t *count, int32_t *ndiag,
                        hipStream_t s)
{
    *count = 0;
    *ndiag = 0;
    if (dst == MXS_SELL) return MXS_ERR_UNSUPPORTED; // needs sigma: sell_size
    if (A->fmt == MXS_ELL || A->fmt == MXS_SELL) {
        if (dst == MXS_ELL && A->fmt == MXS_ELL) {
            *ndiag = A->ndiag;
            *count = (int64_t)A->ndiag * A->nrows;
            return MXS_OK;
        }
        if (dst != MXS_COO && dst != MXS_CSR) return MXS_ERR_UNSUPPORTED;
        *count = A->nnz;
        return MXS_OK;
    }
    if (dst == MXS_ELL) {
        if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
        int32_t K = 0;
        mxs_status st = ell_width(A, &K, s);
        if (st != MXS_OK) return st;
        *ndiag = K;
        *count = (int64_t)K * A->nrows;
        return MXS_OK;
    }
    if (dst == MXS_DIA) {
        if (A->fmt == MXS_DIA) {
            *ndiag = A->ndiag;
            *count = (int64_t)A->ndiag * A->nrows;
            return MXS_OK;
        }
        const int32_t *ai;
        int32_t *tmp;
        mxs_status st = source_rows(A, &ai, &tmp, s);
        if (st != MXS_OK) return st;
        DiaMap m;
        st = build_dia_map(A, ai, &m, s);
        free_dia_map(&m, s);
        if (tmp) MXS_HIP(hipFreeAsync(tmp, s));
        MXS_HIP(hipStreamSynchronize(s));
        if (st != MXS_OK) return st;
        if ((int64_t)m.ndiag * A->nrows > 8 * A->nnz) return MXS_ERR_DIA_TOO_SPARSE;
        *ndiag = m.ndiag;
        *count = (int64_t)m.ndiag * A->nrows;
        return MXS_OK;
    }
    if (A->fmt != MXS_DIA) {
        *count = A->nnz;
        return MXS_OK;
    }
    int32_t *pos = nullptr;
    MXS_HIP(hipMallocAsync((void **)&pos, sizeof(int32_t) * ((size_t)A->nrows + 1), s));
    mxs_status st = A->dtype == MXS_F64 ? dia_counts<double>(A, pos, s) : dia_counts<float>(A, pos, s);
    int32_t total = 0;
    if (st == MXS_OK)
        MXS_HIP(hipMemcpyAsync(&total, pos + A->nrows, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MXS_HIP(hipFreeAsync(pos, s));
    MXS_HIP(hipStreamSynchronize(s));
    *count = total;
    return st;
}

template <typename T>
static mxs_status convert_typed(const mxs_mat_s *A, mxs_format dst, int32_t *idx0, int32_t *idx1,
                                T *vals, int64_t count, int32_t ndiag, hipStream_t s)
{
    const size_t vb = sizeof(T);
    mxs_status st = MXS_OK;
    if (dst == MXS_ELL) {
        if (A->fmt == MXS_ELL) {
            if (count) {
                MXS_HIP(hipMemcpyAsync(idx0, A->idx0, sizeof(int32_t) * count, hipMemcpyDeviceToDevice, s));
                MXS_HIP(hipMemcpyAsync(vals, A->vals, vb * count, hipMemcpyDeviceToDevice, s));
            }
            return MXS_OK;
        }
        return ell_build(A, ndiag, idx0, vals, s);
    }
    if (A->fmt == MXS_ELL || A->fmt == MXS_SELL) return padded_to_rows(A, dst, idx0, idx1, vals, s);
    if (A->fmt == dst) {
        if (dst == MXS_DIA) {
            if (ndiag) MXS_HIP(hipMemcpyAsync(idx0, A->idx0, sizeof(int32_t) * ndiag, hipMemcpyDeviceToDevice, s));
        } else {
            const size_t n0 = dst == MXS_CSR ? (size_t)A->nrows + 1 : (size_t)count;
            if (n0) MXS_HIP(hipMemcpyAsync(idx0, A->idx0, sizeof(int32_t) * n0, hipMemcpyDeviceToDevice, s));
            if (count) MXS_HIP(hipMemcpyAsync(idx1, A->idx1, sizeof(int32_t) * count, hipMemcpyDeviceToDevice, s));
        }
        if (count) MXS_HIP(hipMemcpyAsync(vals, A->vals, vb * count, hipMemcpyDeviceToDevice, s));
        return MXS_OK;
    }
    if (A->fmt != MXS_DIA && dst != MXS_DIA) {
        // COO <-> CSR: columns and values carry over unchanged
        if (count) {
            MXS_HIP(hipMemcpyAsync(idx1, A->idx1, sizeof(int32_t) * count, hipMemcpyDeviceToDevice, s));
            MXS_HIP(hipMemcpyAsync(vals, A->vals, vb * count, hipMemcpyDeviceToDevice, s));
        }
        if (dst == MXS_CSR) {
            coo_to_irp_kernel<<<grid1d(A->nnz + 1), 256, 0, s>>>(A->nnz, A->nrows, A->idx0, idx0);
            return launch_status();
        }
        return csr_row_index(A->idx0, A->nrows, A->nnz, idx0, s);
    }
    if (dst == MXS_DIA) {
        const int32_t *ai;
        int32_t *tmp;
        if ((st = source_rows(A, &ai, &tmp, s)) != MXS_OK) return st;
        DiaMap m;
        if ((st = build_dia_map(A, ai, &m, s)) == MXS_OK) {
            if (m.ndiag != ndiag) st = MXS_ERR_INVALID_ARG;
        }
        if (st == MXS_OK && count > 0) {
            st = fill_bytes0(vals, vb * (size_t)count, s);
            if (st == MXS_OK && m.ndiag > 0) {
                dia_offsets_kernel<<<grid1d(m.span), 256, 0, s>>>(m.span, A->nrows, m.flag, m.map, idx0);
                dia_scatter_kernel<T><<<grid1d(A->nnz), 256, 0, s>>>(A->nnz, A->nrows, ai, A->idx1,
                                                                     (const T *)A->vals, m.map, vals);
                st = launch_status();
            }
        }
        free_dia_map(&m, s);
        if (tmp) MXS_HIP(hipFreeAsync(tmp, s));
        return st;
    }
    // DIA -> COO / CSR
    int32_t *pos = nullptr;
    if (dst == MXS_CSR) {
        pos = idx0;
    } else {
        MXS_HIP(hipMallocAsync((void **)&pos, sizeof(int32_t) * ((size_t)A->nrows + 1), s));
    }
    st = dia_counts<T>(A, pos, s);
    if (st == MXS_OK && A->nrows > 0 && count > 0) {
        dia_emit_kernel<T><<<grid1d(A->nrows), 256, 0, s>>>(A->nrows, A->ncols, A->ndiag, A->idx0,
                                                            (const T *)A->vals, pos,
                                                            dst == MXS_COO ? idx0 : nullptr, idx1,
                                                            vals);
        st = launch_status();
    }
    if (dst != MXS_CSR) MXS_HIP(hipFreeAsync(pos, s));
    return st;
}

mxs_status convert(const mxs_mat_s *A, mxs_format dst, int32_t *idx0, int32_t *idx1, void *vals,
                   int64_t count, int32_t ndiag, hipStream_t s)
{
    if (A->dtype == MXS_F64)
        return convert_typed<double>(A, dst, idx0, idx1, (double *)vals, count, ndiag, s);
    return convert_typed<float>(A, dst, idx0, idx1, (float *)vals, count, ndiag, s);
}

// ---------------------------------------------------------------------------
// Value casts (FP64 -> FP32 rounds to nearest even)
// ---------------------------------------------------------------------------
template <typename S, typename D>
__global__ void cast_kernel(const S *__restrict__ in, D *__restrict__ out, int64_t n)
{
    GRID_STRIDE(i, n) { out[i] = (D)in[i]; }
}

mxs_status cast_values(const void *src, mxs_dtype from, void *dst, mxs_dtype to, int64_t n,
                       hipStream_t s)
{
    if (n == 0) return MXS_OK;
    if (from == to) {
        MXS_HIP(hipMemcpyAsync(dst, src, dsize(from) * (size_t)n, hipMemcpyDeviceToDevice, s));
        return MXS_OK;
    }
    if (from == MXS_F64)
        cast_kernel<double, float><<<grid1d(n), 256, 0, s>>>((const double *)src, (float *)dst, n);
    else
        cast_kernel<float, double><<<grid1d(n), 256, 0, s>>>((const float *)src, (double *)dst, n);
    return launch_status();
}

}  // namespace mxs
