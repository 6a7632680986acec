// Internal SpMM launcher shared by the Lanczos driver and css_spmm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace css {

template <typename T>
struct SpmmArgs {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* col;
    const T* val;
    const T* V;
    T* W;
    int32_t ld;
};

// Enqueues W = H V on stream s; false if ld has no kernel instance.
template <typename T>
bool spmm_launch(const SpmmArgs<T>& a, hipStream_t s);

}  // namespace css
