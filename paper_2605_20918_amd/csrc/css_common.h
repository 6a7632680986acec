// Internal helpers shared by the HIP sources of libcss (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/css.h"

namespace css {

#define CSS_HIP_TRY(expr)                                  \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return CSS_E_DEVICE;         \
    } while (0)

#define CSS_TRY(expr)                                      \
    do {                                                   \
        css_status _s = (expr);                            \
        if (_s != CSS_OK) return _s;                       \
    } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Leading dimension of an n x b block: b rounded up so that 16-wide MFMA tiles
// and the SpMM lane groups cover it exactly.
inline int32_t block_ld(int32_t b) {
    if (b <= 256) return (b + 15) / 16 * 16;
    if (b <= 512) return (b + 31) / 32 * 32;
    return (b + 63) / 64 * 64;
}
constexpr int32_t kMaxColors = 1024;

// Rows of every dense N x ld block are padded to a multiple of this so that
// row tiles need no bounds checks; padded rows are kept at zero.
constexpr int32_t kRowPad = 256;
inline int64_t padded_rows(int64_t n) { return (n + kRowPad - 1) / kRowPad * kRowPad; }

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace. With base == nullptr it only
// counts bytes (used by css_workspace_size with the same call sequence).
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    bool overflow = false;
    template <class T>
    T* take(size_t count) {
        size_t off = align_up(used);
        used = off + align_up(count * sizeof(T));
        if (base == nullptr) return nullptr;
        if (used > cap) { overflow = true; return nullptr; }
        return reinterpret_cast<T*>(base + off);
    }
};

// Launch choices (process-wide, set by css_set_tuning; zero fields mean the built-in
// default). None changes the arithmetic beyond the order of FP32 sums.
struct Tuning {
    int kernel = 0;        // SpMM: 0 automatic (16-row groups where prepared), 1 16-row groups, 2 CSR
    int run = 0;           // SpMM: groups per XCD run (default 512)
    int depth = 0;         // SpMM: k-steps in flight per wave, 4 or 8 (default 4)
    int gram_chunks = 0;   // FP32 split Gram: work-groups per compute unit and product set, 1, 2 or 4 (default 1)
    int update_rows = 0;   // FP32 split block update: rows per work-group, 64 or 128 (default 128)
    int chol_series = 0;   // second CholQR factor: 0 or 1 series near the identity, 2 always factorise
};
Tuning tuning();

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(g);
}

// p[i] = v for i < n. Flags and counters are cleared with this ordinary kernel rather
// than hipMemsetAsync, so that a stream capture holds only kernel nodes.
template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
template <typename T>
inline void fill_launch(T* p, T v, int64_t n, hipStream_t s) {
    k_fill<T><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

}  // namespace css
