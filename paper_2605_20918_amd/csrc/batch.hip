// Many independent systems (clusters, fragments, snapshots of uneven size), each
// the computation of css_density_matrix, in one call.
//
// A small system cannot fill the GPU: its Cholesky factorisations and pole solves
// are N-independent chains that occupy a few compute units, and its SpMM and
// block products have few workgroups. The systems are therefore run side by side
// on library-created streams (default priority), one host worker per stream
// taking systems largest first from a shared counter. Every system goes through
// the single-system path with its own slice of the caller's workspace, so each
// result is bitwise the one css_density_matrix gives for that system alone.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <numeric>
#include <thread>
#include <vector>

#include "css.h"
#include "css_common.h"

namespace css {
namespace {

constexpr size_t kSliceAlign = 256;

size_t slice_bytes(const css_system* sys, int32_t count, int32_t depth, uint32_t flags, css_status* st) {
    size_t per = 0;
    *st = CSS_OK;
    for (int32_t k = 0; k < count; ++k) {
        size_t b = 0;
        const css_status s = css_workspace_size(CSS_ENTRY_DENSITY, sys[k].H.n, sys[k].H.nnz, sys[k].n_colors, depth,
                                                flags, &b);
        if (s != CSS_OK) {
            *st = s;
            return 0;
        }
        per = std::max(per, b);
    }
    return (per + kSliceAlign - 1) / kSliceAlign * kSliceAlign;
}

}  // namespace
}  // namespace css

using namespace css;

extern "C" css_status css_batched_workspace_size(const css_system* systems, int32_t count, int32_t depth,
                                                 uint32_t flags, int32_t concurrency, size_t* bytes) {
    if (!systems || count < 1 || !bytes || concurrency < 1 || concurrency > CSS_MAX_BATCH_STREAMS) return CSS_E_ARG;
    css_status st;
    const size_t per = slice_bytes(systems, count, depth, flags, &st);
    if (st != CSS_OK) return st;
    *bytes = per * (size_t)std::min(concurrency, count);
    return CSS_OK;
}

extern "C" css_status css_density_matrix_batched(css_system* systems, int32_t count, double kT, int32_t depth,
                                                 double spin_deg, uint32_t flags, int32_t concurrency, void* ws,
                                                 size_t ws_bytes, void* stream) {
    if (!systems || count < 1 || !ws || concurrency < 1 || concurrency > CSS_MAX_BATCH_STREAMS) return CSS_E_ARG;
    if (flags & CSS_SUBSPACE_EIG) return CSS_E_UNSUPPORTED;     // one solver handle per device
    css_status st;
    const size_t per = slice_bytes(systems, count, depth, flags, &st);
    if (st != CSS_OK) return st;
    const int C = std::min(concurrency, count);
    if (ws_bytes < per * (size_t)C) return CSS_E_WORKSPACE;
    int dev = 0;
    CSS_HIP_TRY(hipGetDevice(&dev));
    hipStream_t caller = as_stream(stream);

    // the batch starts after the caller's stream has reached this point
    hipEvent_t start = nullptr;
    CSS_HIP_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    std::vector<hipStream_t> st_w(C, nullptr);
    css_status setup = hipEventRecord(start, caller) == hipSuccess ? CSS_OK : CSS_E_DEVICE;
    for (int w = 0; w < C && setup == CSS_OK; ++w) {
        if (hipStreamCreateWithFlags(&st_w[w], hipStreamNonBlocking) != hipSuccess ||
            hipStreamWaitEvent(st_w[w], start, 0) != hipSuccess)
            setup = CSS_E_DEVICE;
    }
    if (setup == CSS_OK) {
        for (int32_t k = 0; k < count; ++k) systems[k].status = CSS_E_DEVICE;   // until run
        std::vector<int32_t> order(count);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return (int64_t)systems[a].H.n * systems[a].n_colors > (int64_t)systems[b].H.n * systems[b].n_colors;
        });
        std::atomic<int32_t> next{0};
        auto work = [&](int w) {
            if (hipSetDevice(dev) != hipSuccess) return;
            char* slice = static_cast<char*>(ws) + (size_t)w * per;
            for (;;) {
                const int32_t i = next.fetch_add(1);
                if (i >= count) break;
                css_system& s = systems[order[i]];
                s.status = css_density_matrix(&s.H, s.color, s.sign, s.n_colors, s.mu, kT, depth, spin_deg,
                                              s.p_row_ptr, s.p_col, s.p_nnz, flags, s.p_val, &s.e_band, &s.trace,
                                              &s.info, slice, per, st_w[w]);
            }
        };
        std::vector<std::thread> threads;
        for (int w = 1; w < C; ++w) threads.emplace_back(work, w);
        work(0);
        for (auto& t : threads) t.join();
    }
    // a system that stopped on an error may have left work queued on its stream
    for (hipStream_t s : st_w)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    (void)hipEventDestroy(start);
    if (setup != CSS_OK) return setup;
    for (int32_t k = 0; k < count; ++k)
        if (systems[k].status != CSS_OK) return systems[k].status;
    return CSS_OK;
}
