// Many independent systems (clusters, fragments, snapshots of uneven size), each
// the computation of css_density_matrix (or of css_color), in one call.
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

size_t color_workspace_bytes(int n);

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

// Runs job(i, worker_stream, worker_index) for i in 0..count-1 on `concurrency`
// library streams (default priority) after the caller's stream has reached this
// point, largest jobs first (`weight`). Every stream is synchronised at the end.
template <class Job>
css_status run_side_by_side(int32_t count, int32_t concurrency, const std::vector<int64_t>& weight,
                            hipStream_t caller, Job job) {
    const int C = std::min(concurrency, count);
    int dev = 0;
    CSS_HIP_TRY(hipGetDevice(&dev));
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
        std::vector<int32_t> order(count);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return weight[a] > weight[b]; });
        std::atomic<int32_t> next{0};
        auto work = [&](int w) {
            if (hipSetDevice(dev) != hipSuccess) return;
            for (;;) {
                const int32_t i = next.fetch_add(1);
                if (i >= count) break;
                job(order[i], st_w[w], w);
            }
        };
        std::vector<std::thread> threads;
        for (int w = 1; w < C; ++w) threads.emplace_back(work, w);
        work(0);
        for (auto& t : threads) t.join();
    }
    // a job that stopped on an error may have left work queued on its stream
    for (hipStream_t st : st_w)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    (void)hipEventDestroy(start);
    return setup;
}

size_t color_slice_bytes(const css_color_job* jobs, int32_t count) {
    size_t per = 0;
    for (int32_t k = 0; k < count; ++k) per = std::max(per, color_workspace_bytes(std::max(1, jobs[k].n)));
    return (per + kSliceAlign - 1) / kSliceAlign * kSliceAlign;
}

}  // namespace
}  // namespace css

using namespace css;

extern "C" css_status css_color_batched_workspace_size(const css_color_job* jobs, int32_t count,
                                                       int32_t concurrency, size_t* bytes) {
    if (!jobs || count < 1 || !bytes || concurrency < 1 || concurrency > CSS_MAX_BATCH_STREAMS) return CSS_E_ARG;
    *bytes = color_slice_bytes(jobs, count) * (size_t)std::min(concurrency, count);
    return CSS_OK;
}

extern "C" css_status css_color_batched(css_color_job* jobs, int32_t count, int32_t concurrency, void* ws,
                                        size_t ws_bytes, void* stream) {
    if (!jobs || count < 1 || !ws || concurrency < 1 || concurrency > CSS_MAX_BATCH_STREAMS) return CSS_E_ARG;
    const size_t per = color_slice_bytes(jobs, count);
    if (ws_bytes < per * (size_t)std::min(concurrency, count)) return CSS_E_WORKSPACE;
    std::vector<int64_t> weight(count);
    for (int32_t k = 0; k < count; ++k) {
        weight[k] = jobs[k].n;
        jobs[k].status = CSS_E_DEVICE;                           // until run
    }
    const css_status setup = run_side_by_side(count, concurrency, weight, as_stream(stream),
                                              [&](int32_t k, hipStream_t st, int w) {
        css_color_job& j = jobs[k];
        j.status = css_color(j.xyz, j.n, j.box, j.r_cut, j.color, &j.n_colors, j.p_row_ptr, j.p_col, &j.p_nnz,
                             &j.rounds, static_cast<char*>(ws) + (size_t)w * per, per, st);
    });
    if (setup != CSS_OK) return setup;
    for (int32_t k = 0; k < count; ++k)
        if (jobs[k].status != CSS_OK) return jobs[k].status;
    return CSS_OK;
}

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
    if (ws_bytes < per * (size_t)std::min(concurrency, count)) return CSS_E_WORKSPACE;
    std::vector<int64_t> weight(count);
    for (int32_t k = 0; k < count; ++k) {
        weight[k] = (int64_t)systems[k].H.n * systems[k].n_colors;
        systems[k].status = CSS_E_DEVICE;                        // until run
    }
    const css_status setup = run_side_by_side(count, concurrency, weight, as_stream(stream),
                                              [&](int32_t k, hipStream_t st, int w) {
        css_system& sy = systems[k];
        sy.status = css_density_matrix(&sy.H, sy.color, sy.sign, sy.n_colors, sy.mu, kT, depth, spin_deg,
                                       sy.p_row_ptr, sy.p_col, sy.p_nnz, flags, sy.p_val, &sy.e_band, &sy.trace,
                                       &sy.info, static_cast<char*>(ws) + (size_t)w * per, per, st);
    });
    if (setup != CSS_OK) return setup;
    for (int32_t k = 0; k < count; ++k)
        if (systems[k].status != CSS_OK) return systems[k].status;
    return CSS_OK;
}
