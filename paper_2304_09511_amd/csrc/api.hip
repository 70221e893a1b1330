// The C ABI of libmxs (declared in mxs.h): argument validation, handle
// lifecycle and dispatch to the kernels.  Validation that needs no device
// data runs before any HIP call, so invalid arguments are reported without
// touching the GPU.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.h"

using namespace mxs;

namespace mxs {

// Detail of the last failed HIP call on this thread (see mxs_last_error).
thread_local char g_last_error[512];
thread_local char g_stale_error[160];

mxs_status note_hip_error(hipError_t e, const char *where)
{
    snprintf(g_last_error, sizeof g_last_error, "%s: %s at %s%s", hipGetErrorName(e),
             hipGetErrorString(e), where, g_stale_error);
    return from_hip(e);
}

void release(mxs_mat_s *A)
{
    if (!A) return;
    release(A->band);
    release(A->rest);
    for (mxs_mat_s *B : A->cblk) release(B);
    for (void *p : A->owned)
        if (p) (void)hipFree(p);
    delete A;
}

}  // namespace mxs

namespace {

hipStream_t S(void *stream) { return (hipStream_t)stream; }

bool valid_dtype(mxs_dtype t) { return t == MXS_F64 || t == MXS_F32; }
bool valid_format(mxs_format f)
{
    return f == MXS_COO || f == MXS_CSR || f == MXS_DIA || f == MXS_ELL || f == MXS_SELL || f == MXS_HYB;
}

// Every entry point that touches the GPU runs its body through guarded():
// an error another library left pending in HIP's per-thread error slot is
// cleared first (and named in the detail of a later failure), so launch
// checks report only this call's own launches.
template <typename F>
mxs_status guarded(F &&f)
{
    const hipError_t stale = hipGetLastError();
    if (stale != hipSuccess)
        snprintf(g_stale_error, sizeof g_stale_error, " [an earlier %s pending before this call was cleared]",
                 hipGetErrorName(stale));
    else
        g_stale_error[0] = 0;
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return MXS_ERR_OUT_OF_MEMORY;
    } catch (...) {
        snprintf(g_last_error, sizeof g_last_error, "C++ exception inside libmxs%s", g_stale_error);
        return MXS_ERR_HIP;
    }
}


// Copies `bytes` from a caller array into memory the handle owns.
mxs_status own_copy(mxs_mat_s *A, const void *src, size_t bytes, void **dst, hipStream_t s)
{
    *dst = nullptr;
    if (bytes == 0) return MXS_OK;
    MXS_HIP(hipMalloc(dst, bytes));
    A->owned.push_back(*dst);
    MXS_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyDeviceToDevice, s));
    return MXS_OK;
}

int64_t value_count(const mxs_mat_s *A)
{
    if (A->fmt == MXS_DIA || A->fmt == MXS_ELL) return (int64_t)A->ndiag * A->nrows;
    if (A->fmt == MXS_SELL) return A->slots;
    return A->nnz;
}

// Calls that run SpMV kernels need the plan mxs_optimize builds: it is
// never built implicitly.
inline mxs_status need_plan(const mxs_mat_s *A) { return A->optimized ? MXS_OK : MXS_ERR_NO_PLAN; }

// Sizing pass of A's plan (see PlanCtx); `tiny` holds the measurement counters.
mxs_status plan_layout(mxs_mat_s *A, unsigned opts, void *tiny, PlanCtx *out, hipStream_t s)
{
    PlanCtx c;
    c.opts = opts;
    c.tiny = tiny;
    const mxs_status st = plan_walk(A, c, s);
    *out = c;
    return st;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return na && nb && x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

const char *mxs_status_string(mxs_status s)
{
    switch (s) {
    case MXS_OK: return "MXS_OK";
    case MXS_NOT_CONVERGED: return "MXS_NOT_CONVERGED";
    case MXS_ERR_INVALID_ARG: return "MXS_ERR_INVALID_ARG";
    case MXS_ERR_INDEX_RANGE: return "MXS_ERR_INDEX_RANGE";
    case MXS_ERR_UNSORTED: return "MXS_ERR_UNSORTED";
    case MXS_ERR_DUPLICATE: return "MXS_ERR_DUPLICATE";
    case MXS_ERR_DIA_TOO_SPARSE: return "MXS_ERR_DIA_TOO_SPARSE";
    case MXS_ERR_OUT_OF_MEMORY: return "MXS_ERR_OUT_OF_MEMORY";
    case MXS_ERR_HIP: return "MXS_ERR_HIP";
    case MXS_ERR_BREAKDOWN: return "MXS_ERR_BREAKDOWN";
    case MXS_ERR_NONFINITE: return "MXS_ERR_NONFINITE";
    case MXS_ERR_UNSUPPORTED: return "MXS_ERR_UNSUPPORTED";
    case MXS_ERR_NO_PLAN: return "MXS_ERR_NO_PLAN";
    }
    return "MXS_UNKNOWN_STATUS";
}

int32_t mxs_version(void) { return 10000; }

const char *mxs_last_error(void) { return g_last_error; }

// ---------------------------------------------------------------------------
// Containers
// ---------------------------------------------------------------------------
mxs_status mxs_coo_create(mxs_mat *out, int32_t nrows, int32_t ncols, int64_t nnz,
                          const int32_t *ai, const int32_t *aj, const void *av, mxs_dtype dtype,
                          unsigned flags, void *stream)
{
    if (!out || nrows < 0 || ncols < 0 || nnz < 0 || !valid_dtype(dtype) ||
        (flags & ~MXS_BORROW))
        return MXS_ERR_INVALID_ARG;
    if (nnz > 0 && (!ai || !aj || !av)) return MXS_ERR_INVALID_ARG;
    if (nnz > INT32_MAX) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_mat_s *A = new mxs_mat_s;
        A->fmt = MXS_COO;
        A->dtype = dtype;
        A->nrows = nrows;
        A->ncols = ncols;
        A->nnz = nnz;
        MXS_HIP(hipGetDevice(&A->device));
        mxs_status st = MXS_OK;
        if (flags & MXS_BORROW) {
            A->idx0 = ai;
            A->idx1 = aj;
            A->vals = av;
        } else {
            void *p0, *p1, *p2;
            if ((st = own_copy(A, ai, sizeof(int32_t) * nnz, &p0, s)) != MXS_OK ||
                (st = own_copy(A, aj, sizeof(int32_t) * nnz, &p1, s)) != MXS_OK ||
                (st = own_copy(A, av, dsize(dtype) * nnz, &p2, s)) != MXS_OK)
                return release(A), st;
            A->idx0 = (const int32_t *)p0;
            A->idx1 = (const int32_t *)p1;
            A->vals = p2;
        }
        st = check_coo(A, s);
        if (st == MXS_ERR_UNSORTED && !(flags & MXS_BORROW)) {
            st = sort_coo(nrows, ncols, nnz, (int32_t *)A->idx0, (int32_t *)A->idx1,
                          (void *)A->vals, dtype, s);
            if (st == MXS_OK) st = check_coo(A, s);
        }
        if (st != MXS_OK) return release(A), st;
        *out = A;
        return MXS_OK;
    });
}

mxs_status mxs_csr_create(mxs_mat *out, int32_t nrows, int32_t ncols, int64_t nnz,
                          const int32_t *irp, const int32_t *aj, const void *av, mxs_dtype dtype,
                          unsigned flags, void *stream)
{
    if (!out || nrows < 0 || ncols < 0 || nnz < 0 || !valid_dtype(dtype) ||
        (flags & ~MXS_BORROW) || !irp)
        return MXS_ERR_INVALID_ARG;
    if (nnz > 0 && (!aj || !av)) return MXS_ERR_INVALID_ARG;
    if (nnz > INT32_MAX) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_mat_s *A = new mxs_mat_s;
        A->fmt = MXS_CSR;
        A->dtype = dtype;
        A->nrows = nrows;
        A->ncols = ncols;
        A->nnz = nnz;
        MXS_HIP(hipGetDevice(&A->device));
        mxs_status st = MXS_OK;
        if (flags & MXS_BORROW) {
            A->idx0 = irp;
            A->idx1 = aj;
            A->vals = av;
        } else {
            void *p0, *p1, *p2;
            if ((st = own_copy(A, irp, sizeof(int32_t) * ((size_t)nrows + 1), &p0, s)) != MXS_OK ||
                (st = own_copy(A, aj, sizeof(int32_t) * nnz, &p1, s)) != MXS_OK ||
                (st = own_copy(A, av, dsize(dtype) * nnz, &p2, s)) != MXS_OK)
                return release(A), st;
            A->idx0 = (const int32_t *)p0;
            A->idx1 = (const int32_t *)p1;
            A->vals = p2;
        }
        if ((st = check_csr(A, s)) != MXS_OK) return release(A), st;
        *out = A;
        return MXS_OK;
    });
}

mxs_status mxs_dia_create(mxs_mat *out, int32_t nrows, int32_t ncols, int32_t ndiag,
                          const int32_t *doff, const void *av, mxs_dtype dtype, unsigned flags,
                          void *stream)
{
    if (!out || nrows < 0 || ncols < 0 || ndiag < 0 || !valid_dtype(dtype) ||
        (flags & ~MXS_BORROW))
        return MXS_ERR_INVALID_ARG;
    if (ndiag > 0 && (!doff || (nrows > 0 && !av))) return MXS_ERR_INVALID_ARG;
    if ((int64_t)ndiag > (int64_t)nrows + ncols - 1 && ndiag > 0) return MXS_ERR_INDEX_RANGE;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_mat_s *A = new mxs_mat_s;
        A->fmt = MXS_DIA;
        A->dtype = dtype;
        A->nrows = nrows;
        A->ncols = ncols;
        A->ndiag = ndiag;
        MXS_HIP(hipGetDevice(&A->device));
        mxs_status st = MXS_OK;
        if (flags & MXS_BORROW) {
            A->idx0 = doff;
            A->vals = av;
        } else {
            void *p0, *p2;
            if ((st = own_copy(A, doff, sizeof(int32_t) * ndiag, &p0, s)) != MXS_OK ||
                (st = own_copy(A, av, dsize(dtype) * (size_t)ndiag * nrows, &p2, s)) != MXS_OK)
                return release(A), st;
            A->idx0 = (const int32_t *)p0;
            A->vals = p2;
        }
        if ((st = check_dia(A, s)) != MXS_OK || (st = dia_slot_count(A, &A->nnz, s)) != MXS_OK)
            return release(A), st;
        *out = A;
        return MXS_OK;
    });
}

mxs_status mxs_destroy(mxs_mat A)
{
    if (!A) return MXS_OK;
    if (A->part) return MXS_ERR_INVALID_ARG; // released with its split matrix
    return guarded([&] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipSetDevice(A->device);
        const hipError_t e = hipDeviceSynchronize();
        release(A);
        (void)hipSetDevice(dev);
        return from_hip(e);
    });
}

mxs_status mxs_info(mxs_mat A, mxs_format *fmt, mxs_dtype *dtype, int32_t *nrows, int32_t *ncols,
                    int64_t *nnz, int32_t *ndiag)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    if (fmt) *fmt = A->fmt;
    if (dtype) *dtype = A->dtype;
    if (nrows) *nrows = A->nrows;
    if (ncols) *ncols = A->ncols;
    if (nnz) *nnz = A->nnz;
    if (ndiag) *ndiag = A->ndiag;
    return MXS_OK;
}

mxs_status mxs_arrays(mxs_mat A, const int32_t **idx0, const int32_t **idx1, const void **vals)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    if (is_split(A)) return MXS_ERR_UNSUPPORTED;
    if (idx0) *idx0 = A->idx0;
    if (idx1) *idx1 = A->idx1;
    if (vals) *vals = A->vals;
    return MXS_OK;
}

// ---------------------------------------------------------------------------
// Conversion
// ---------------------------------------------------------------------------
mxs_status mxs_convert_size(mxs_mat src, mxs_format dst, int64_t *count, int32_t *ndiag,
                            void *stream)
{
    if (!src || !valid_format(dst)) return MXS_ERR_INVALID_ARG;
    if (is_split(src)) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        int64_t c = 0;
        int32_t nd = 0;
        mxs_status st = convert_size(src, dst, &c, &nd, S(stream));
        if (st != MXS_OK) return st;
        if (count) *count = c;
        if (ndiag) *ndiag = nd;
        return MXS_OK;
    });
}

mxs_status mxs_convert(mxs_mat src, mxs_format dst, int32_t *idx0, int32_t *idx1, void *vals,
                       mxs_mat *out, void *stream)
{
    if (!src || !valid_format(dst) || !out) return MXS_ERR_INVALID_ARG;
    if (is_split(src)) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        hipStream_t s = S(stream);
        int64_t count = 0;
        int32_t nd = 0;
        mxs_status st = convert_size(src, dst, &count, &nd, s);
        if (st != MXS_OK) return st;
        const bool need0 = dst == MXS_CSR || ((dst == MXS_COO || dst == MXS_ELL) && count > 0) ||
                           (dst == MXS_DIA && nd > 0);
        const bool need1 = (dst == MXS_COO || dst == MXS_CSR) && count > 0;
        if ((need0 && !idx0) || (need1 && !idx1) || (count > 0 && !vals))
            return MXS_ERR_INVALID_ARG;
        if ((st = convert(src, dst, idx0, idx1, vals, count, nd, s)) != MXS_OK) return st;
        mxs_mat_s *B = new mxs_mat_s;
        B->fmt = dst;
        B->dtype = src->dtype;
        B->nrows = src->nrows;
        B->ncols = src->ncols;
        B->device = src->device;
        B->idx0 = idx0;
        B->idx1 = dst == MXS_COO || dst == MXS_CSR ? idx1 : nullptr;
        B->vals = vals;
        if (dst == MXS_DIA) {
            B->ndiag = nd;
            if ((st = dia_slot_count(B, &B->nnz, s)) != MXS_OK) return release(B), st;
        } else if (dst == MXS_ELL) {
            B->ndiag = nd;
            B->nnz = src->nnz; // entries (COO/CSR/ELL source)
        } else {
            B->nnz = count;
        }
        MXS_HIP(hipStreamSynchronize(s));
        *out = B;
        return MXS_OK;
    });
}

mxs_status mxs_cast(mxs_mat src, mxs_dtype dtype, void *vals, mxs_mat *out, void *stream)
{
    if (!src || !valid_dtype(dtype) || !out) return MXS_ERR_INVALID_ARG;
    if (is_split(src)) return MXS_ERR_UNSUPPORTED;
    const int64_t n = value_count(src);
    if (n > 0 && !vals) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        mxs_status st = cast_values(src->vals, src->dtype, vals, dtype, n, S(stream));
        if (st != MXS_OK) return st;
        mxs_mat_s *B = new mxs_mat_s;
        B->fmt = src->fmt;
        B->dtype = dtype;
        B->nrows = src->nrows;
        B->ncols = src->ncols;
        B->nnz = src->nnz;
        B->ndiag = src->ndiag;
        B->device = src->device;
        B->idx0 = src->idx0;
        B->idx1 = src->idx1;
        B->vals = vals;
        B->sell_cs = src->sell_cs;
        B->slots = src->slots;
        B->sigma = src->sigma;
        *out = B;
        return MXS_OK;
    });
}

mxs_status mxs_hyb_size(mxs_mat A, int32_t K, int32_t *K_out, int64_t *rest_nnz, void *stream)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        int32_t k = K;
        int64_t r = 0;
        mxs_status st = hyb_size(A, &k, &r, S(stream));
        if (st != MXS_OK) return st;
        if (K_out) *K_out = k;
        if (rest_nnz) *rest_nnz = r;
        return MXS_OK;
    });
}

mxs_status mxs_to_hyb(mxs_mat A, int32_t K, int32_t *ell_col, void *ell_val, int32_t *rest_ai,
                      int32_t *rest_aj, void *rest_av, mxs_mat *out, void *stream)
{
    if (!A || !out) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        hipStream_t s = S(stream);
        int32_t k = K;
        int64_t r = 0;
        mxs_status st = hyb_size(A, &k, &r, s);
        if (st != MXS_OK) return st;
        if ((k > 0 && A->nrows > 0 && (!ell_col || !ell_val)) || (r > 0 && (!rest_ai || !rest_aj || !rest_av)))
            return MXS_ERR_INVALID_ARG;
        if ((st = hyb_build(A, k, ell_col, ell_val, rest_ai, rest_aj, rest_av, s)) != MXS_OK) return st;
        MXS_HIP(hipStreamSynchronize(s));
        auto *band = new mxs_mat_s;
        band->fmt = MXS_ELL;
        band->dtype = A->dtype;
        band->nrows = A->nrows;
        band->ncols = A->ncols;
        band->ndiag = k;
        band->nnz = A->nnz - r;
        band->idx0 = ell_col;
        band->vals = ell_val;
        band->device = A->device;
        band->part = band->sub = true;
        auto *rest = new mxs_mat_s;
        rest->fmt = MXS_COO;
        rest->dtype = A->dtype;
        rest->nrows = A->nrows;
        rest->ncols = A->ncols;
        rest->nnz = r;
        rest->idx0 = rest_ai;
        rest->idx1 = rest_aj;
        rest->vals = rest_av;
        rest->device = A->device;
        rest->part = rest->sub = true;
        auto *h = new mxs_mat_s;
        h->fmt = MXS_HYB;
        h->dtype = A->dtype;
        h->nrows = A->nrows;
        h->ncols = A->ncols;
        h->nnz = A->nnz;
        h->ndiag = k;
        h->device = A->device;
        h->band = band;
        h->rest = rest;
        *out = h;
        return MXS_OK;
    });
}

mxs_status mxs_sell_size(mxs_mat A, int32_t sigma, int64_t *slots, int32_t *nslices, void *stream)
{
    if (!A || sigma < 1) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        int64_t h = 0;
        mxs_status st = sell_size(A, sigma, &h, S(stream));
        if (st != MXS_OK) return st;
        if (slots) *slots = h;
        if (nslices) *nslices = (int32_t)(((int64_t)A->nrows + 63) / 64);
        return MXS_OK;
    });
}

mxs_status mxs_to_sell(mxs_mat A, int32_t sigma, int32_t *perm, int64_t *cs, int32_t *col, void *vals,
                       mxs_mat *out, void *stream)
{
    if (!A || sigma < 1 || !out || !cs || (A->nrows > 0 && !perm)) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        hipStream_t s = S(stream);
        int64_t slots = 0;
        mxs_status st = sell_size(A, sigma, &slots, s);
        if (st != MXS_OK) return st;
        if (slots > 0 && (!col || !vals)) return MXS_ERR_INVALID_ARG;
        if ((st = sell_build(A, sigma, perm, cs, col, vals, s)) != MXS_OK) return st;
        mxs_mat_s *B = new mxs_mat_s;
        B->fmt = MXS_SELL;
        B->dtype = A->dtype;
        B->nrows = A->nrows;
        B->ncols = A->ncols;
        B->nnz = A->nnz;
        B->ndiag = (int32_t)(((int64_t)A->nrows + 63) / 64);
        B->device = A->device;
        B->idx0 = col;
        B->idx1 = perm;
        B->vals = vals;
        B->sell_cs = cs;
        B->slots = slots;
        B->sigma = sigma;
        MXS_HIP(hipStreamSynchronize(s));
        *out = B;
        return MXS_OK;
    });
}

// ---------------------------------------------------------------------------
// SpMV and BLAS-1
// ---------------------------------------------------------------------------
constexpr unsigned kPlanOpts = MXS_PLAN_NO_ELL | MXS_PLAN_NO_COLBLK | MXS_PLAN_DIA_BLOCKED;

mxs_status mxs_plan_size(mxs_mat A, unsigned opts, size_t *bytes, void *stream)
{
    if (!A || !bytes || (opts & ~kPlanOpts) || A->sub) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        std::lock_guard<std::mutex> lk(A->mu);
        void *tiny = nullptr;
        MXS_HIP(hipMallocAsync(&tiny, kTinyBytes, s));
        PlanCtx c;
        mxs_status st = plan_layout(A, opts, tiny, &c, s);
        (void)hipFreeAsync(tiny, s);
        if (hipStreamSynchronize(s) != hipSuccess && st == MXS_OK) st = MXS_ERR_HIP;
        if (st == MXS_OK) *bytes = c.total();
        return st;
    });
}

mxs_status mxs_optimize(mxs_mat A, unsigned opts, void *workspace, size_t bytes, void *stream)
{
    if (!A || (opts & ~kPlanOpts) || A->sub || (bytes > 0 && !workspace)) return MXS_ERR_INVALID_ARG;
    if ((uintptr_t)workspace % kPlanAlign != 0) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        std::lock_guard<std::mutex> lk(A->mu);
        // the earlier plan (if any) is dropped first: the workspace may be its memory
        plan_reset(A);
        // the layout, its counters in the workspace's first bytes
        PlanCtx z;
        mxs_status st = plan_layout(A, opts, bytes >= kTinyBytes ? workspace : nullptr, &z, s);
        if (st != MXS_OK) return st;
        if (bytes < z.total()) return MXS_ERR_INVALID_ARG;
        // then the plan itself
        PlanCtx c;
        c.opts = opts;
        c.build = true;
        c.keep_base = (char *)workspace;
        char *t = (char *)workspace + PlanCtx::up(z.keep_used);
        c.tiny = z.tiny_used ? (void *)t : nullptr;
        c.tmp_base = t + (z.tiny_used ? kTinyBytes : 0);
        st = plan_walk(A, c, s);
        if (st == MXS_OK && hipStreamSynchronize(s) != hipSuccess) st = MXS_ERR_HIP;
        if (st == MXS_OK && (c.keep_used != z.keep_used || c.total() > z.total())) {
            snprintf(g_last_error, sizeof g_last_error,
                     "plan layout differs between its sizing and build passes");
            st = MXS_ERR_HIP;
        }
        if (st != MXS_OK) plan_reset(A);
        return st;
    });
}

mxs_status mxs_plan_info(mxs_mat A, int32_t *optimized, unsigned *opts)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    if (optimized) *optimized = A->optimized ? 1 : 0;
    if (opts) *opts = A->plan_opts;
    return MXS_OK;
}

mxs_status mxs_split_parts(mxs_mat H, mxs_mat *band, mxs_mat *rest)
{
    if (!H) return MXS_ERR_INVALID_ARG;
    if (!is_split(H)) return MXS_ERR_UNSUPPORTED;
    if (band) *band = H->band;
    if (rest) *rest = H->rest;
    return MXS_OK;
}

int32_t mxs_impl_count(mxs_mat A)
{
    return A ? impl_count(A) : 0;
}

mxs_status mxs_set_impl(mxs_mat A, int32_t impl, void *stream)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    if (is_split(A)) return MXS_ERR_UNSUPPORTED;
    return guarded([&] {
        mxs_status st = need_plan(A);
        if (st != MXS_OK) return st;
        std::lock_guard<std::mutex> lk(A->mu);
        if (!impl_ok(A, impl)) return MXS_ERR_UNSUPPORTED;
        set_impl(A, impl);
        return MXS_OK;
    });
}

mxs_status mxs_get_impl(mxs_mat A, int32_t *impl, void *stream)
{
    if (!A || !impl) return MXS_ERR_INVALID_ARG;
    if (is_split(A)) return MXS_ERR_UNSUPPORTED;
    (void)stream;
    return guarded([&] {
        mxs_status st = need_plan(A);
        if (st == MXS_OK) *impl = A->impl;
        return st;
    });
}

mxs_status mxs_tune(mxs_mat A, const void *x, void *y, int32_t reps, int32_t *impl, double *ms,
                    void *stream)
{
    if (!A || reps < 1 || reps > 10000) return MXS_ERR_INVALID_ARG;
    if (is_split(A)) return MXS_ERR_UNSUPPORTED;
    const size_t es = dsize(A->dtype);
    if ((A->ncols > 0 && !x) || (A->nrows > 0 && !y)) return MXS_ERR_INVALID_ARG;
    if (overlaps(x, es * A->ncols, y, es * A->nrows)) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_status st = need_plan(A);
        if (st != MXS_OK) return st;
        std::lock_guard<std::mutex> lk(A->mu);
        return tune(A, x, y, reps, impl, ms, s);
    });
}

mxs_status mxs_spmv(mxs_mat A, const void *x, void *y, void *stream)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    const size_t es = dsize(A->dtype);
    if ((A->ncols > 0 && !x) || (A->nrows > 0 && !y)) return MXS_ERR_INVALID_ARG;
    if (overlaps(x, es * A->ncols, y, es * A->nrows)) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        mxs_status st = need_plan(A);
        if (st != MXS_OK) return st;
        return spmv_launch(A, x, y, nullptr, nullptr, S(stream));
    });
}

mxs_status mxs_spmv_scratch_size(mxs_mat A, size_t *bytes)
{
    if (!A || !bytes) return MXS_ERR_INVALID_ARG;
    if (!A->optimized) return MXS_ERR_NO_PLAN;
    *bytes = spmv_scratch_bytes(A);
    return MXS_OK;
}

mxs_status mxs_spmv_ws(mxs_mat A, const void *x, void *y, void *scratch, size_t bytes, void *stream)
{
    if (!A) return MXS_ERR_INVALID_ARG;
    const size_t es = dsize(A->dtype);
    if ((A->ncols > 0 && !x) || (A->nrows > 0 && !y)) return MXS_ERR_INVALID_ARG;
    if (overlaps(x, es * A->ncols, y, es * A->nrows)) return MXS_ERR_INVALID_ARG;
    if (!A->optimized) return MXS_ERR_NO_PLAN;
    const size_t need = spmv_scratch_bytes(A);
    if (bytes < need || (need > 0 && !scratch)) return MXS_ERR_INVALID_ARG;
    if (scratch && (overlaps(scratch, need, x, es * A->ncols) || overlaps(scratch, need, y, es * A->nrows)))
        return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        return spmv_launch(A, x, y, nullptr, nullptr, S(stream), need > 0 ? scratch : nullptr);
    });
}

mxs_status mxs_dot(int64_t n, mxs_dtype dtype, const void *a, const void *b, double *result,
                   void *stream)
{
    if (n < 0 || !valid_dtype(dtype) || !result || (n > 0 && (!a || !b)))
        return MXS_ERR_INVALID_ARG;
    return guarded([&] { return dot_launch(n, dtype, a, b, result, S(stream)); });
}

mxs_status mxs_dot_noalloc(int64_t n, mxs_dtype dtype, const void *a, const void *b, double *result,
                           void *stream)
{
    if (n < 0 || !valid_dtype(dtype) || !result || (n > 0 && (!a || !b)))
        return MXS_ERR_INVALID_ARG;
    return guarded([&] { return dot_noalloc_launch(n, dtype, a, b, result, S(stream)); });
}

mxs_status mxs_axpby(int64_t n, mxs_dtype dtype, double alpha, const void *x, double beta, void *y,
                     void *stream)
{
    if (n < 0 || !valid_dtype(dtype) || (n > 0 && (!x || !y))) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return axpby_launch(n, dtype, alpha, x, beta, y, S(stream)); });
}

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------
mxs_status mxs_cg_workspace_size(mxs_mat A, int32_t mixed, size_t *bytes)
{
    if (!A || !bytes) return MXS_ERR_INVALID_ARG;
    *bytes = cg_workspace_bytes(A->nrows, mixed ? 1 : 0, 0, 0);
    return MXS_OK;
}

mxs_status mxs_cg_solve(mxs_mat A, mxs_mat A32, const double *b, double *x, const mxs_cg_opts *opts,
                        mxs_cg_result *res, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!A || !opts || !res || A->dtype != MXS_F64 || A->nrows != A->ncols)
        return MXS_ERR_INVALID_ARG;
    if (A->nrows > 0 && (!b || !x || !workspace)) return MXS_ERR_INVALID_ARG;
    if (overlaps(b, 8 * (size_t)A->nrows, x, 8 * (size_t)A->nrows)) return MXS_ERR_INVALID_ARG;
    if (opts->mixed && (!A32 || A32->dtype != MXS_F32 || A32->nrows != A->nrows ||
                        A32->ncols != A->ncols))
        return MXS_ERR_INVALID_ARG;
    if (opts->mixed < 0 || opts->mixed > 2) return MXS_ERR_INVALID_ARG;
    if (opts->mixed && is_split(A)) return MXS_ERR_UNSUPPORTED;
    if (!(opts->rtol >= 0.0) || opts->maxit < 0 || (opts->mixed == 1 && opts->max_outer < 0))
        return MXS_ERR_INVALID_ARG;
    if (opts->mixed == 2 && !(opts->ru_delta >= 0.0 && opts->ru_delta <= 1.0))
        return MXS_ERR_INVALID_ARG;
    if (workspace_bytes < cg_workspace_bytes(A->nrows, opts->mixed ? 1 : 0, 0, 0))
        return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_status st = need_plan(A);
        if (st == MXS_OK && opts->mixed) st = need_plan(A32);
        if (st != MXS_OK) return st;
        if (A->nrows == 0) {
            *res = mxs_cg_result{};
            return MXS_OK;
        }
        return cg_solve(A, opts->mixed ? A32 : nullptr, b, x, opts, res, workspace,
                        workspace_bytes, s);
    });
}

// ---------------------------------------------------------------------------
// HPCG's preconditioner
// ---------------------------------------------------------------------------
static mxs_status mg_shape_ok(int32_t n, int32_t levels)
{
    if (n < 1 || levels < 1 || levels > 12) return MXS_ERR_INVALID_ARG;
    if (n % (1 << (levels - 1)) != 0) return MXS_ERR_INVALID_ARG;
    if ((int64_t)n * n * n > INT32_MAX || mxs_stencil_nnz(n, 27) > INT32_MAX)
        return MXS_ERR_UNSUPPORTED;
    return MXS_OK;
}

mxs_status mxs_mg_size(int32_t n, int32_t levels, size_t *bytes)
{
    if (!bytes) return MXS_ERR_INVALID_ARG;
    const mxs_status st = mg_shape_ok(n, levels);
    if (st != MXS_OK) return st;
    return guarded([&] {
        *bytes = mg_bytes(n, levels);
        return *bytes > 0 ? MXS_OK : MXS_ERR_UNSUPPORTED;
    });
}

mxs_status mxs_mg_create(int32_t n, int32_t levels, void *workspace, size_t bytes, mxs_mg *out,
                         void *stream)
{
    if (!out || !workspace || (uintptr_t)workspace % kPlanAlign != 0) return MXS_ERR_INVALID_ARG;
    const mxs_status st = mg_shape_ok(n, levels);
    if (st != MXS_OK) return st;
    return guarded([&] { return mg_create(n, levels, workspace, bytes, out, S(stream)); });
}

mxs_status mxs_mg_destroy(mxs_mg M)
{
    if (!M) return MXS_OK;
    return guarded([&] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipSetDevice(M->device);
        const hipError_t e = hipDeviceSynchronize();
        mg_release(M);
        (void)hipSetDevice(dev);
        return from_hip(e);
    });
}

mxs_status mxs_mg_level(mxs_mg M, int32_t level, int32_t *n, mxs_mat *A)
{
    if (!M || level < 0 || level >= (int32_t)M->lv.size()) return MXS_ERR_INVALID_ARG;
    if (n) *n = M->lv[(size_t)level].n;
    if (A) *A = M->lv[(size_t)level].A;
    return MXS_OK;
}

mxs_status mxs_symgs(mxs_mg M, int32_t level, const double *r, double *x, void *stream)
{
    if (!M || level < 0 || level >= (int32_t)M->lv.size()) return MXS_ERR_INVALID_ARG;
    const size_t rows = (size_t)M->lv[(size_t)level].rows;
    if (!r || !x || overlaps(r, 8 * rows, x, 8 * rows)) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return symgs_launch(M, level, r, x, S(stream)); });
}

mxs_status mxs_mg_apply(mxs_mg M, const double *r, double *z, void *stream)
{
    if (!M) return MXS_ERR_INVALID_ARG;
    const size_t rows = (size_t)M->lv[0].rows;
    if (!r || !z || overlaps(r, 8 * rows, z, 8 * rows)) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mg_apply(M, r, z, nullptr, S(stream)); });
}

mxs_status mxs_pcg_workspace_size(mxs_mg M, size_t *bytes)
{
    if (!M || !bytes) return MXS_ERR_INVALID_ARG;
    *bytes = pcg_workspace_bytes(M->lv[0].rows);
    return MXS_OK;
}

mxs_status mxs_pcg_solve(mxs_mg M, mxs_mat A, const double *b, double *x, const mxs_cg_opts *opts,
                         mxs_cg_result *res, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!M || !opts || !res) return MXS_ERR_INVALID_ARG;
    if (!A) A = M->lv[0].A;
    const int64_t n = M->lv[0].rows;
    if (A->dtype != MXS_F64 || A->nrows != n || A->ncols != n) return MXS_ERR_INVALID_ARG;
    if (!b || !x || !workspace || overlaps(b, 8 * (size_t)n, x, 8 * (size_t)n))
        return MXS_ERR_INVALID_ARG;
    if (opts->mixed != 0 || !(opts->rtol >= 0.0) || opts->maxit < 0) return MXS_ERR_INVALID_ARG;
    if (workspace_bytes < pcg_workspace_bytes(n)) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        mxs_status st = need_plan(A);
        if (st != MXS_OK) return st;
        return pcg_solve(M, A, b, x, opts, res, workspace, workspace_bytes, s);
    });
}

// ---------------------------------------------------------------------------
// Split matrices
// ---------------------------------------------------------------------------
mxs_status mxs_split_size(mxs_mat A, double min_fill, int32_t *band_ndiag, int64_t *rest_nnz,
                          void *stream)
{
    if (!A || !band_ndiag || !rest_nnz || !(min_fill >= 0.0)) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    return guarded([&] { return split_size(A, min_fill, band_ndiag, rest_nnz, S(stream)); });
}

mxs_status mxs_split(mxs_mat A, double min_fill, mxs_format rest_format, int32_t *band_doff,
                     void *band_vals, int32_t *rest_idx0, int32_t *rest_idx1, void *rest_vals,
                     mxs_mat *out, void *stream)
{
    if (!A || !out || !(min_fill >= 0.0) || (rest_format != MXS_COO && rest_format != MXS_CSR))
        return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR) return MXS_ERR_UNSUPPORTED;
    if (rest_format == MXS_CSR && A->nrows > 0 && !rest_idx0) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        int32_t nd = 0;
        int64_t rn = 0;
        mxs_status st = split_size(A, min_fill, &nd, &rn, s);
        if (st != MXS_OK) return st;
        if ((nd > 0 && (!band_doff || !band_vals)) ||
            (rn > 0 && (!rest_idx0 || !rest_idx1 || !rest_vals)))
            return MXS_ERR_INVALID_ARG;
        mxs_mat_s *h = nullptr;
        st = split(A, min_fill, rest_format, band_doff, band_vals, rest_idx0, rest_idx1, rest_vals,
                   &h, s);
        if (st == MXS_OK) *out = h;
        return st;
    });
}

// ---------------------------------------------------------------------------
// Problem setup
// ---------------------------------------------------------------------------
int64_t mxs_stencil_nnz(int32_t n, int32_t points)
{
    if (n < 0) return -1;
    const int64_t m = n;
    if (points == 27) return (3 * m - 2) * (3 * m - 2) * (3 * m - 2) * (m > 0);
    if (points == 7) return m * m * m + 6 * (m - 1) * m * m * (m > 0);
    return -1;
}

mxs_status mxs_stencil_coo(int32_t n, int32_t points, double diag, double offdiag, int32_t *ai,
                           int32_t *aj, void *av, mxs_dtype dtype, void *stream)
{
    if (n < 0 || (points != 7 && points != 27) || !valid_dtype(dtype)) return MXS_ERR_INVALID_ARG;
    const int64_t nnz = mxs_stencil_nnz(n, points);
    if ((int64_t)n * n * n > INT32_MAX || nnz > INT32_MAX) return MXS_ERR_UNSUPPORTED;
    if (nnz > 0 && (!ai || !aj || !av)) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return stencil_coo(n, points, diag, offdiag, ai, aj, av, dtype, S(stream)); });
}

// ---------------------------------------------------------------------------
// Format selection
// ---------------------------------------------------------------------------
mxs_status mxs_features(mxs_mat A, double out[8], void *stream)
{
    if (!A || !out) return MXS_ERR_INVALID_ARG;
    if (A->fmt != MXS_COO && A->fmt != MXS_CSR && A->fmt != MXS_DIA) return MXS_ERR_UNSUPPORTED;
    return guarded([&] { return features(A, out, S(stream)); });
}

mxs_status mxs_mlp_inputs(const double *raw, int32_t n, const float *mu, const float *sd, float *X,
                          void *stream)
{
    if (n < 0 || (n > 0 && (!raw || !mu || !sd || !X))) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_inputs(raw, n, mu, sd, X, S(stream)); });
}

mxs_status mxs_mlp_norm_stats(const double *raw, int32_t n, float *mu, float *sd, void *stream)
{
    if (n < 0 || !mu || !sd || (n > 0 && !raw)) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_norm_stats(raw, n, mu, sd, S(stream)); });
}

mxs_status mxs_mlp_forward(const float *w, const float *X, int32_t n, float *logits, void *stream)
{
    if (n < 0 || !w || (n > 0 && (!X || !logits))) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_forward(w, X, n, logits, S(stream)); });
}

mxs_status mxs_mlp_predict(const float *w, const float *X, int32_t n, const uint8_t *feasible,
                           int32_t *fmt_out, void *stream)
{
    if (n < 0 || !w || (n > 0 && (!X || !fmt_out))) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_predict(w, X, n, feasible, fmt_out, S(stream)); });
}

size_t mxs_mlp_workspace_size(int32_t n)
{
    // per-sample scratch, then (for mxs_mlp_train_step) the gradient
    return (mlp_ws_bytes(n) + 255) / 256 * 256 + sizeof(float) * MXS_MLP_NPARAM;
}

mxs_status mxs_mlp_grad(const float *w, const float *X, const int32_t *labels, int32_t n,
                        float *grad, float *loss, void *workspace, size_t bytes, void *stream)
{
    if (n < 0 || !w || !grad || !loss || (n > 0 && (!X || !labels || !workspace)))
        return MXS_ERR_INVALID_ARG;
    if (n > 0 && bytes < mlp_ws_bytes(n)) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_grad(w, X, labels, n, grad, loss, workspace, S(stream)); });
}

mxs_status mxs_mlp_adam(float *w, float *m, float *v, const float *grad, float lr, int32_t t,
                        float beta1, float beta2, float eps, void *stream)
{
    if (!w || !m || !v || !grad || t < 1) return MXS_ERR_INVALID_ARG;
    return guarded([&] { return mlp_adam(w, m, v, grad, lr, t, beta1, beta2, eps, S(stream)); });
}

mxs_status mxs_mlp_train_step(float *w, float *m, float *v, const float *X, const int32_t *labels,
                              int32_t n, float lr, int32_t t, float *loss, void *workspace,
                              size_t bytes, void *stream)
{
    if (!w || !m || !v || !loss || t < 1 || n < 0 || (n > 0 && (!X || !labels || !workspace)))
        return MXS_ERR_INVALID_ARG;
    if (bytes < mxs_mlp_workspace_size(n)) return MXS_ERR_INVALID_ARG;
    return guarded([&] {
        hipStream_t s = S(stream);
        const size_t off = (mlp_ws_bytes(n) + 255) / 256 * 256;
        float *grad = (float *)((char *)workspace + off);
        mxs_status st = mlp_grad(w, X, labels, n, grad, loss, workspace, s);
        if (st != MXS_OK) return st;
        return mlp_adam(w, m, v, grad, lr, t, 0.9f, 0.999f, 1e-8f, s);
    });
}

}  // extern "C"
