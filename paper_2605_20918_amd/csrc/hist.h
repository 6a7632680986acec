// Internal: colour histogram count[c] += #{m : color[m] == c}, c in [0, b).
//
// Each work-group counts its share in LDS and adds one global atomic per
// (work-group, colour): a global atomic per orbital would serialise on the few
// colour counters, all work-groups of the device queueing on the same addresses.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "css_common.h"

namespace css {

constexpr int kHistThreads = 1024;
constexpr int kHistMaxBins = 8192;     // LDS bins (32 KB); more colours count directly
constexpr int kHistBlocks = 64;

// count must be zero beforehand. Colours outside [0, b) are not counted and set
// *bad |= bad_bit when bad is not null.
__global__ __launch_bounds__(kHistThreads) inline void k_colour_hist(const int32_t* __restrict__ color, int n, int b,
                                                                    int* __restrict__ count, int* __restrict__ bad,
                                                                    int bad_bit) {
    extern __shared__ int bins[];
    const bool lds = b <= kHistMaxBins;
    if (lds) {
        for (int c = threadIdx.x; c < b; c += kHistThreads) bins[c] = 0;
        __syncthreads();
    }
    bool out = false;
    for (int64_t m = blockIdx.x * (int64_t)kHistThreads + threadIdx.x; m < n; m += (int64_t)gridDim.x * kHistThreads) {
        const int c = color[m];
        if (c < 0 || c >= b) out = true;
        else if (lds) atomicAdd(&bins[c], 1);
        else atomicAdd(&count[c], 1);
    }
    if (out && bad) atomicOr(bad, bad_bit);
    if (lds) {
        __syncthreads();
        for (int c = threadIdx.x; c < b; c += kHistThreads)
            if (bins[c]) atomicAdd(&count[c], bins[c]);
    }
}

inline void colour_hist(const int32_t* color, int n, int b, int* count, int* bad, int bad_bit, hipStream_t s) {
    const unsigned grid = std::min<unsigned>(kHistBlocks, grid_for(n, kHistThreads));
    const size_t lds = b <= kHistMaxBins ? sizeof(int) * (size_t)b : 0;
    k_colour_hist<<<grid, kHistThreads, lds, s>>>(color, n, b, count, bad, bad_bit);
}

}  // namespace css
