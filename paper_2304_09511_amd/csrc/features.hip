// Matrix features for format selection: row-length statistics from the row
// pointers and the distinct-diagonal count and bandwidth from the entries.
// Integer reductions only (exact and order-independent); the few divisions
// happen on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "common.h"

namespace mxs {

struct FeatAcc {
    unsigned long long sumsq; // sum of squared row lengths
    unsigned long long ndiag; // distinct offsets
    int maxlen;               // longest row
    int bandwidth;            // max |j - i|
};

#define GRID_STRIDE(i, n)                                                          \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

__global__ void row_stats_kernel(int32_t nrows, const int32_t *__restrict__ irp, FeatAcc *acc)
{
    unsigned long long sq = 0;
    int mx = 0;
    GRID_STRIDE(r, nrows)
    {
        const long long l = irp[r + 1] - irp[r];
        sq += (unsigned long long)(l * l);
        mx = max(mx, (int)l);
    }
    if (sq) atomicAdd(&acc->sumsq, sq);
    if (mx) atomicMax(&acc->maxlen, mx);
}

__global__ void entry_stats_kernel(int64_t nnz, int32_t nrows, const int32_t *__restrict__ ai,
                                   const int32_t *__restrict__ aj, int32_t *__restrict__ flag,
                                   FeatAcc *acc)
{
    int bw = 0;
    GRID_STRIDE(k, nnz)
    {
        const int32_t d = aj[k] - ai[k];
        flag[(int64_t)d + nrows - 1] = 1;
        bw = max(bw, abs(d));
    }
    if (bw) atomicMax(&acc->bandwidth, bw);
}

__global__ void count_flags_kernel(int64_t n, const int32_t *__restrict__ flag, FeatAcc *acc)
{
    unsigned long long c = 0;
    GRID_STRIDE(i, n) c += flag[i] != 0;
    if (c) atomicAdd(&acc->ndiag, c);
}

static uint32_t grid_of(int64_t n)
{
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}


mxs_status features(const mxs_mat_s *A, double out[8], hipStream_t s)
{
    mxs_status st = MXS_OK;
    const int32_t nrows = A->nrows, ncols = A->ncols;
    std::vector<void *> tmp;
    auto talloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMallocAsync(&p, std::max<size_t>(bytes, 4), s) != hipSuccess) return nullptr;
        tmp.push_back(p);
        return p;
    };
    auto release = [&]() {
        for (void *p : tmp) (void)hipFreeAsync(p, s);
        (void)hipStreamSynchronize(s);
    };
    // A CSR + COO view of the stored (non-zero for DIA) entries.
    const int32_t *irp = nullptr, *ai = nullptr, *aj = nullptr;
    int64_t nnz = A->nnz;
    if (A->fmt == MXS_DIA) {
        int64_t cnt;
        int32_t nd;
        if ((st = convert_size(A, MXS_CSR, &cnt, &nd, s)) != MXS_OK) return st;
        int32_t *c_irp = (int32_t *)talloc(sizeof(int32_t) * ((size_t)nrows + 1));
        int32_t *c_aj = (int32_t *)talloc(sizeof(int32_t) * (size_t)cnt);
        void *c_av = talloc(dsize(A->dtype) * (size_t)cnt);
        if (!c_irp || !c_aj || !c_av) return release(), MXS_ERR_OUT_OF_MEMORY;
        if ((st = convert(A, MXS_CSR, c_irp, c_aj, c_av, cnt, 0, s)) != MXS_OK) return release(), st;
        irp = c_irp;
        aj = c_aj;
        nnz = cnt;
    } else if (A->fmt == MXS_CSR) {
        irp = A->idx0;
        aj = A->idx1;
    } else {
        ai = A->idx0;
        aj = A->idx1;
        int32_t *c_irp = (int32_t *)talloc(sizeof(int32_t) * ((size_t)nrows + 1));
        if (!c_irp) return release(), MXS_ERR_OUT_OF_MEMORY;
        if ((st = coo_irp_launch(nnz, nrows, ai, c_irp, s)) != MXS_OK) return release(), st;
        irp = c_irp;
    }
    if (!ai) {
        int32_t *c_ai = (int32_t *)talloc(sizeof(int32_t) * (size_t)nnz);
        if (!c_ai) return release(), MXS_ERR_OUT_OF_MEMORY;
        if ((st = csr_row_index(irp, nrows, nnz, c_ai, s)) != MXS_OK) return release(), st;
        ai = c_ai;
    }
    const int64_t span = std::max<int64_t>((int64_t)nrows + ncols - 1, 1);
    FeatAcc *acc = (FeatAcc *)talloc(sizeof(FeatAcc));
    int32_t *flag = (int32_t *)talloc(sizeof(int32_t) * (size_t)span);
    if (!acc || !flag) return release(), MXS_ERR_OUT_OF_MEMORY;
    if ((st = fill_bytes0(acc, sizeof(FeatAcc), s)) != MXS_OK) return release(), st;
    if ((st = fill_i32(flag, 0, span, s)) != MXS_OK) return release(), st;
    if (nrows > 0) row_stats_kernel<<<grid_of(nrows), 256, 0, s>>>(nrows, irp, acc);
    if (nnz > 0) entry_stats_kernel<<<grid_of(nnz), 256, 0, s>>>(nnz, nrows, ai, aj, flag, acc);
    count_flags_kernel<<<grid_of(span), 256, 0, s>>>(span, flag, acc);
    if (hipGetLastError() != hipSuccess) return release(), MXS_ERR_HIP;
    FeatAcc h;
    if (hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
        return release(), MXS_ERR_HIP;
    release();
    const double n = (double)nrows;
    out[0] = n;
    out[1] = (double)nnz;
    out[2] = nrows ? (double)nnz / n : 0.0;
    if (nrows) {
        // population variance from exact integer moments: (n*S2 - S1^2) / n^2
        const __int128 num = (__int128)nrows * (__int128)h.sumsq - (__int128)nnz * (__int128)nnz;
        out[3] = (double)((long double)num / ((long double)nrows * (long double)nrows));
    } else {
        out[3] = 0.0;
    }
    out[4] = (double)h.maxlen;
    out[5] = (double)h.ndiag;
    out[6] = (h.ndiag > 0 && nrows > 0) ? (double)nnz / ((double)h.ndiag * n) : 0.0;
    out[7] = ncols > 0 ? (double)h.bandwidth / (double)ncols : 0.0;
    return MXS_OK;
}

}  // namespace mxs
