// Sparse H times a dense block: W = H V (the product the whole method is built
// on; the paper performs every such product with a CPU SpMM library).
//
// Layout: H in CSR (int32 row pointers and columns, FP64 or FP32 values);
// V and W row-major n x ld, so one orbital's b entries are contiguous. A group
// of LPR lanes owns one row of W and lane j of the group owns columns
// j, j+LPR, ..., j+(C-1)*LPR (ld = C*LPR), so every V row is read as C
// coalesced LPR-wide segments. The row's nonzeros are walked four at a time
// to keep several V-row loads in flight.

#include <hip/hip_runtime.h>

#include <mutex>

#include "css_common.h"
#include "spmm.h"

namespace css {
namespace {

template <typename T, int LPR, int C>
__global__ __launch_bounds__(256) void k_spmm_csr(int n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ V,
                                                  T* __restrict__ W, int ld) {
    const int lane = threadIdx.x % LPR;
    const int64_t row = (int64_t)blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
    if (row >= n) return;
    T acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = T(0);
    const int s = rp[row], e = rp[row + 1];
    const T* __restrict__ vb = V + lane;
    int t = s;
    for (; t + 4 <= e; t += 4) {
        const int64_t c0 = col[t], c1 = col[t + 1], c2 = col[t + 2], c3 = col[t + 3];
        const T h0 = val[t], h1 = val[t + 1], h2 = val[t + 2], h3 = val[t + 3];
        const T* p0 = vb + c0 * ld;
        const T* p1 = vb + c1 * ld;
        const T* p2 = vb + c2 * ld;
        const T* p3 = vb + c3 * ld;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            T a = p0[k * LPR], b = p1[k * LPR], c = p2[k * LPR], d = p3[k * LPR];
            acc[k] += h0 * a;
            acc[k] += h1 * b;
            acc[k] += h2 * c;
            acc[k] += h3 * d;
        }
    }
    for (; t < e; ++t) {
        const int64_t c0 = col[t];
        const T h0 = val[t];
        const T* p0 = vb + c0 * ld;
#pragma unroll
        for (int k = 0; k < C; ++k) acc[k] += h0 * p0[k * LPR];
    }
    T* __restrict__ wr = W + row * ld + lane;
#pragma unroll
    for (int k = 0; k < C; ++k) wr[k * LPR] = acc[k];
}

template <typename T, int LPR, int C>
void launch_one(const SpmmArgs<T>& a, hipStream_t s) {
    constexpr int rows_per_block = 256 / LPR;
    const unsigned grid = static_cast<unsigned>((a.n + rows_per_block - 1) / rows_per_block);
    k_spmm_csr<T, LPR, C><<<grid, 256, 0, s>>>(a.n, a.row_ptr, a.col, a.val, a.V, a.W, a.ld);
}

template <typename T, int LPR>
bool dispatch_c(const SpmmArgs<T>& a, int c, hipStream_t s) {
    switch (c) {
#define CSS_CASE(CC) case CC: launch_one<T, LPR, CC>(a, s); return true;
        CSS_CASE(1) CSS_CASE(2) CSS_CASE(3) CSS_CASE(4) CSS_CASE(5) CSS_CASE(6) CSS_CASE(7) CSS_CASE(8)
        CSS_CASE(9) CSS_CASE(10) CSS_CASE(11) CSS_CASE(12) CSS_CASE(13) CSS_CASE(14) CSS_CASE(15) CSS_CASE(16)
#undef CSS_CASE
        default: return false;
    }
}

// state[1] |= 1 for a malformed CSR structure.
__global__ void k_validate_csr(int n, int64_t nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int* __restrict__ state) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const int32_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || b > nnz) atomicOr(&state[1], 1);
        if (i == 0 && a != 0) atomicOr(&state[1], 1);
        if (i == n - 1 && (int64_t)b != nnz) atomicOr(&state[1], 1);
    }
    if (i < nnz) {
        const int32_t c = col[i];
        if (c < 0 || c >= n) atomicOr(&state[1], 1);
    }
}

__global__ void k_zero_ints(int* __restrict__ p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

}  // namespace

void csr_validate_launch(int n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, int* state,
                         hipStream_t s) {
    k_validate_csr<<<grid_for(std::max<int64_t>(n, nnz), 256), 256, 0, s>>>(n, nnz, row_ptr, col, state);
}

template <typename T>
bool spmm_launch(const SpmmArgs<T>& a, hipStream_t s) {
    if (a.ld % 16 != 0 || a.ld > kMaxColors) return false;
    if (a.ld <= 256) return dispatch_c<T, 16>(a, a.ld / 16, s);
    if (a.ld <= 512 && a.ld % 32 == 0) return dispatch_c<T, 32>(a, a.ld / 32, s);
    if (a.ld % 64 == 0) return dispatch_c<T, 64>(a, a.ld / 64, s);
    return false;
}

template bool spmm_launch<double>(const SpmmArgs<double>&, hipStream_t);
template bool spmm_launch<float>(const SpmmArgs<float>&, hipStream_t);

namespace {

std::mutex g_tune_mu;
Tuning g_tune;

constexpr size_t kSpmmHeader = 256;     // 16 status ints ahead of the group arrays

SpmmGroups groups_in(void* ws, int n, int64_t nnz, size_t elem) {
    Arena a;
    a.base = static_cast<char*>(ws) + kSpmmHeader;
    a.cap = ~size_t(0);
    SpmmGroups g;
    carve_groups(a, n, nnz, elem, g);
    return g;
}

bool csr_shape_ok(const css_csr* H) {
    return H && H->n >= 1 && H->row_ptr && H->col && H->val && H->nnz >= 0 && H->nnz < (int64_t(1) << 31) &&
           (H->val_dtype == CSS_F64 || H->val_dtype == CSS_F32);
}

size_t elem_of(const css_csr* H) { return H->val_dtype == CSS_F32 ? 4 : 8; }

// The product on a workspace filled by css_spmm_prepare (16-row groups) unless the
// tuning asks for the CSR kernel, or the CSR kernel without a workspace.
css_status spmm_dispatch(const css_csr* H, const void* V, void* W, int32_t ld, const void* ws, const Tuning& tu,
                         hipStream_t s) {
    SpmmGroups g = ws ? groups_in(const_cast<void*>(ws), H->n, H->nnz, elem_of(H)) : SpmmGroups{};
    g.blocks_ready = ws != nullptr && tu.kernel != 2;
    bool ok;
    if (H->val_dtype == CSS_F64) {
        SpmmArgs<double> a{H->n, H->row_ptr, H->col, static_cast<const double*>(H->val),
                           static_cast<const double*>(V), static_cast<double*>(W), ld};
        ok = spmm_grp_launch(a, g, tu, s) || spmm_launch(a, s);
    } else {
        SpmmArgs<float> a{H->n, H->row_ptr, H->col, static_cast<const float*>(H->val),
                          static_cast<const float*>(V), static_cast<float*>(W), ld};
        ok = spmm_grp_launch(a, g, tu, s) || spmm_launch(a, s);
    }
    if (!ok) return CSS_E_UNSUPPORTED;
    return hipGetLastError() == hipSuccess ? CSS_OK : CSS_E_DEVICE;
}

css_status tuning_from(const css_tuning* t, Tuning& v) {
    if (t->spmm_kernel < 0 || t->spmm_kernel > 2 || t->spmm_run < 0 ||
        (t->spmm_depth != 0 && t->spmm_depth != 4 && t->spmm_depth != 8) ||
        (t->gram_chunks != 0 && t->gram_chunks != 1 && t->gram_chunks != 2 && t->gram_chunks != 4) ||
        (t->update_rows != 0 && t->update_rows != 64 && t->update_rows != 128) || t->cholqr2_series < 0 ||
        t->cholqr2_series > 2)
        return CSS_E_ARG;
    v.kernel = t->spmm_kernel;
    v.run = t->spmm_run;
    v.depth = t->spmm_depth;
    v.gram_chunks = t->gram_chunks;
    v.update_rows = t->update_rows;
    v.chol_series = t->cholqr2_series;
    return CSS_OK;
}

}  // namespace

size_t spmm_workspace_bytes(int n, int64_t nnz) {
    Arena a;
    SpmmGroups g;
    carve_groups(a, n, nnz, 8, g);
    return kSpmmHeader + a.used;
}

Tuning tuning() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune;
}

}  // namespace css

using namespace css;

extern "C" css_status css_spmm_prepare(const css_csr* H, void* ws, size_t ws_bytes, void* stream) {
    if (!csr_shape_ok(H) || !ws) return CSS_E_ARG;
    if (ws_bytes < spmm_workspace_bytes(H->n, H->nnz)) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    int* state = static_cast<int*>(ws);
    const SpmmGroups g = groups_in(ws, H->n, H->nnz, elem_of(H));
    k_zero_ints<<<1, 64, 0, s>>>(state, 16);
    csr_validate_launch(H->n, H->nnz, H->row_ptr, H->col, state, s);
    int hst[16];
    CSS_HIP_TRY(hipGetLastError());
    CSS_HIP_TRY(hipMemcpyAsync(hst, state, sizeof(hst), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (hst[1]) return CSS_E_CSR;
    spmm_grp_prepare(H->n, H->row_ptr, H->col, g, state + 4, s);
    CSS_HIP_TRY(hipGetLastError());
    CSS_HIP_TRY(hipMemcpyAsync(hst, state, sizeof(hst), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (!spmm_grp_worthwhile(H->nnz, hst[4], hst[5])) return CSS_E_UNSUPPORTED;
    if (H->val_dtype == CSS_F64)
        spmm_grp_fill<double>(H->n, H->row_ptr, static_cast<const double*>(H->val), g, s);
    else
        spmm_grp_fill<float>(H->n, H->row_ptr, static_cast<const float*>(H->val), g, s);
    CSS_HIP_TRY(hipGetLastError());
    return CSS_OK;
}

extern "C" css_status css_spmm(const css_csr* H, const void* V, void* W, int32_t b, int32_t ld, const void* ws,
                               size_t ws_bytes, void* stream) {
    if (!csr_shape_ok(H) || !V || !W || b < 1 || ld < b) return CSS_E_ARG;
    if (ws && ws_bytes < spmm_workspace_bytes(H->n, H->nnz)) return CSS_E_WORKSPACE;
    return spmm_dispatch(H, V, W, ld, ws, tuning(), as_stream(stream));
}

extern "C" css_status css_spmm_time(const css_csr* H, const void* V, void* W, int32_t b, int32_t ld, const void* ws,
                                    size_t ws_bytes, const css_tuning* cfg, int32_t reps, float* avg_ms,
                                    void* stream) {
    if (!csr_shape_ok(H) || !V || !W || b < 1 || ld < b || reps < 1 || !avg_ms) return CSS_E_ARG;
    if (ws && ws_bytes < spmm_workspace_bytes(H->n, H->nnz)) return CSS_E_WORKSPACE;
    Tuning tu = tuning();
    if (cfg) CSS_TRY(tuning_from(cfg, tu));
    hipStream_t s = as_stream(stream);
    CSS_TRY(spmm_dispatch(H, V, W, ld, ws, tu, s));          // untimed
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CSS_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CSS_E_DEVICE;
    }
    css_status st = hipEventRecord(e0, s) == hipSuccess ? CSS_OK : CSS_E_DEVICE;
    for (int r = 0; r < reps && st == CSS_OK; ++r) st = spmm_dispatch(H, V, W, ld, ws, tu, s);
    if (st == CSS_OK && hipEventRecord(e1, s) != hipSuccess) st = CSS_E_DEVICE;
    if (st == CSS_OK && hipEventSynchronize(e1) != hipSuccess) st = CSS_E_DEVICE;
    float ms = 0.f;
    if (st == CSS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = CSS_E_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == CSS_OK) *avg_ms = ms / (float)reps;
    return st;
}

extern "C" css_status css_set_tuning(const css_tuning* t) {
    Tuning v;
    if (t) CSS_TRY(tuning_from(t, v));
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = v;
    return CSS_OK;
}

extern "C" css_status css_get_tuning(css_tuning* t) {
    if (!t) return CSS_E_ARG;
    const Tuning v = tuning();
    *t = css_tuning{};
    t->spmm_kernel = v.kernel;
    t->spmm_run = v.run;
    t->spmm_depth = v.depth;
    t->gram_chunks = v.gram_chunks;
    t->update_rows = v.update_rows;
    t->cholqr2_series = v.chol_series;
    return CSS_OK;
}
