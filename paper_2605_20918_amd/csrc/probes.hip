// CSS probe vectors: one +-1 probe per colour (Eq.(2), Fig.1(c)).
//
// The probes are never stored densely: probe c is sign[m] on the orbitals m of
// colour c. Signs come from a counter-based SplitMix64 (Steele, Lea and Flood,
// 2014): the (m+1)-th output from state `seed` is mix(seed + (m+1)*gamma),
// gamma = 0x9E3779B97F4A7C15, mix the published two-multiply finaliser.

#include <hip/hip_runtime.h>

#include <vector>

#include "css_common.h"
#include "hist.h"

namespace css {
namespace {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t m) {
    uint64_t z = seed + (m + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_probes(int n, uint64_t seed, int ones, int8_t* __restrict__ sign) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    sign[m] = ones ? int8_t(1) : ((splitmix64_at(seed, (uint64_t)m) >> 63) ? int8_t(-1) : int8_t(1));
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0;
}

}  // namespace
}  // namespace css

using namespace css;

extern "C" css_status css_build_probes(const int32_t* color, int32_t n, int32_t n_colors, uint64_t seed,
                                       uint32_t flags, int8_t* sign, int32_t* color_count, void* stream) {
    if (n < 1 || n_colors < 1 || n_colors > n || !color || !sign || !color_count) return CSS_E_ARG;
    hipStream_t s = as_stream(stream);
    k_zero_i32<<<grid_for(n_colors, 256), 256, 0, s>>>(color_count, n_colors);
    k_probes<<<grid_for(n, 256), 256, 0, s>>>(n, seed, (flags & CSS_SIGNS_ONES) ? 1 : 0, sign);
    colour_hist(color, n, n_colors, color_count, nullptr, 0, s);     // out-of-range colours show in the sum
    std::vector<int32_t> h(n_colors);
    CSS_HIP_TRY(hipMemcpyAsync(h.data(), color_count, sizeof(int32_t) * n_colors, hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    int64_t total = 0;
    for (int32_t c : h) {
        if (c <= 0) return CSS_E_CSR;                  // a colour owns no orbital
        total += c;
    }
    return total == n ? CSS_OK : CSS_E_CSR;           // some colour was out of range
}
