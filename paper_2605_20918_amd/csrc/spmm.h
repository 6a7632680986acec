// Internal SpMM launcher shared by the Lanczos driver and css_spmm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "css_common.h"

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

// state[1] |= 1 (device int) if row_ptr / col do not form a valid n-row CSR of nnz entries.
void csr_validate_launch(int n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, int* state,
                         hipStream_t s);

// Row-group (16 rows) MFMA SpMM: per group the sorted union U_g of its rows'
// columns (once per pattern) and H's values as a dense k-major 16 x round4(|U_g|)
// block (once per set of values).
constexpr int kSpmmGroup = 16;
constexpr int kSpmmGroupCap = 8192;   // nonzeros of one group the union kernel can sort
constexpr int kGroupFill = 4;         // grouped kernel if sum 16 |U_g| <= kGroupFill nnz
struct SpmmGroups {
    int32_t* U = nullptr;        // nnz: group g's union at U[row_ptr[16 g] ..]
    int32_t* ucount = nullptr;   // groups: |U_g|
    int32_t* pos = nullptr;      // nnz: (row in group) << 16 | position of the entry's column in U_g
    int64_t* boff = nullptr;     // groups + 1: element offset of each group's block
    void* hblk = nullptr;        // cap elements of H's value type
    int64_t cap = 0;
    bool blocks_ready = false;   // blocks filled for the current H
};


int spmm_groups(int n);
// Elements reserved for the blocks: enough whenever spmm_grp_worthwhile holds.
int64_t spmm_grp_block_cap(int n, int64_t nnz);
// Takes the group arrays from an arena (elem = bytes per H value).
void carve_groups(Arena& a, int n, int64_t nnz, size_t elem, SpmmGroups& g);
// Builds the unions and block offsets of a validated CSR (reads row_ptr and col
// only). Device ints: stats[0] |= 1 if a group has more than kSpmmGroupCap nonzeros
// (its union is left empty and the grouped kernel must not be used); stats[1] = sum
// of |U_g| (capped at INT_MAX).
void spmm_grp_prepare(int n, const int32_t* row_ptr, const int32_t* col, const SpmmGroups& gp, int* stats,
                      hipStream_t s);
// Host decision from the two stats: no oversized group and blocks within kGroupFill nnz.
bool spmm_grp_worthwhile(int64_t nnz, int too_long, int64_t sum_union);
// The dense blocks from H's values (after spmm_grp_prepare, and only when
// spmm_grp_worthwhile holds, so that the blocks fit in cap).
template <typename T>
void spmm_grp_fill(int n, const int32_t* row_ptr, const T* val, const SpmmGroups& gp, hipStream_t s);
// false if ld is not a multiple of 16 up to 128, or V / W are not 16-byte aligned.
// V must be finite: a block's explicit zeros multiply V rows of other rows' columns.
template <typename T>
bool spmm_grp_launch(const SpmmArgs<T>& a, const SpmmGroups& gp, const Tuning& tu, hipStream_t s);

// The grouped product where the tuning allows it and the blocks are filled; false
// otherwise (the caller then runs the CSR kernel).
template <typename T>
bool spmm_grouped_launch(const SpmmArgs<T>& a, const SpmmGroups& gp, hipStream_t s);

// Workspace of css_spmm_prepare / css_spmm: status ints and the group arrays.
size_t spmm_workspace_bytes(int n, int64_t nnz);

}  // namespace css
