// Sparse H times a dense block on MFMA, by groups of 16 rows.
//
// W = H V with V, W row-major n x ld. Rows are taken 16 at a time. For group g
// the sorted union U_g of its rows' column indices is computed once per sparsity
// pattern (k_grp_union), and H's values once per call (k_grp_fill) as a dense
// 16 x |U_g| block, k-major (Hg[k][row]), zero-padded to a multiple of 4 columns.
// The product of the group is then the small dense product
//   W[16g .. 16g+15, :] = Hg (16 x |U_g|) * V[U_g, :] (|U_g| x ld)
// on MFMA: every V row in U_g is read once per group instead of once per nonzero
// (the cost of a row-per-lane CSR kernel, where each nonzero re-reads a b-wide V
// row). The blocks' zeros cost MFMA work and block bytes only; on water-like H
// the blocks hold about 2.3 times the nonzeros.
//
// MFMA 16x16x4 layout (gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// result register r of lane l holds D[4(l/16)+r][l%16] (FP32) or D[(l/16)+4r][l%16] (FP64).
// The 16 columns of one MFMA tile need not be adjacent columns of W: a segment of
// q tiles starting at tile t gives lane column lc of its e-th tile the W column
// 16t + q lc + e, so each lane reads (and writes) q adjacent elements at once.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "css_common.h"
#include "mfma_util.h"
#include "spmm.h"

namespace css {
namespace {

template <typename T>
using GMF = Mfma<T>;

// Per group: U_g (sorted unique columns) at U[rp[16g] ..], |U_g| in ucount[g], and for
// every CSR entry t of the group pos[t] = (row - 16g) << 16 | (position of col[t] in U_g).
// stats[0] |= 1 if a group holds more than kSpmmGroupCap entries.
// The group's entries are sorted in LDS: with sorted rows by four levels of pairwise
// merges of the 16 rows (an entry's place in the merged run is its place in its own
// run plus the number of entries of the partner run before it, ties to the left
// run), otherwise by a bitonic sort.
__device__ __forceinline__ int lower_in(const int32_t* a, int lo, int hi, int x) {   // first a[i] >= x
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int upper_in(const int32_t* a, int lo, int hi, int x) {   // first a[i] > x
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

constexpr int kUnionThreads = 1024;

__global__ __launch_bounds__(kUnionThreads) void k_grp_union(int n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, int32_t* __restrict__ U,
                                                   int32_t* __restrict__ ucount, int32_t* __restrict__ pos,
                                                   int* __restrict__ stats) {
    __shared__ int32_t buf0[kSpmmGroupCap];
    __shared__ int32_t buf1[kSpmmGroupCap];
    __shared__ uint8_t rowof[kSpmmGroupCap];
    __shared__ int32_t scan[kUnionThreads];
    __shared__ int32_t grp[kSpmmGroup + 1];       // group-relative row starts
    __shared__ int unsorted;
    const int g = blockIdx.x;
    const int r0 = g * kSpmmGroup;
    const int r1 = min(n, r0 + kSpmmGroup);
    const int t0 = rp[r0], t1 = rp[r1];
    const int cnt = t1 - t0;
    if (cnt > kSpmmGroupCap) {
        if (threadIdx.x == 0) {
            ucount[g] = 0;
            atomicOr(&stats[0], 1);
        }
        return;
    }
    if (threadIdx.x <= kSpmmGroup) grp[threadIdx.x] = rp[min(r0 + (int)threadIdx.x, r1)] - t0;
    if (threadIdx.x == 0) unsorted = 0;
    for (int i = threadIdx.x; i < cnt; i += kUnionThreads) buf0[i] = col[t0 + i];
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kUnionThreads) {
        int r = 0;
        while (grp[r + 1] <= i) ++r;
        rowof[i] = static_cast<uint8_t>(r);
        if (i > grp[r] && buf0[i - 1] > buf0[i]) unsorted = 1;
    }
    __syncthreads();
    int32_t* srt = buf0;
    int32_t* tmp = buf1;
    if (!unsorted) {
        for (int lev = 0; lev < 4; ++lev) {
            for (int i = threadIdx.x; i < cnt; i += kUnionThreads) {
                const int run = rowof[i] >> lev;
                const int left = run & ~1;
                const int ls = grp[min(kSpmmGroup, left << lev)];          // left run [ls, ms)
                const int ms = grp[min(kSpmmGroup, (left + 1) << lev)];    // right run [ms, re)
                const int re = grp[min(kSpmmGroup, (left + 2) << lev)];
                const int x = srt[i];
                const int at = (run & 1) ? (i - ms) + upper_in(srt, ls, ms, x) - ls
                                         : (i - ls) + lower_in(srt, ms, re, x) - ms;
                tmp[ls + at] = x;
            }
            __syncthreads();
            int32_t* t = srt;
            srt = tmp;
            tmp = t;
        }
    } else {
        int len = 1;
        while (len < cnt) len <<= 1;
        for (int i = cnt + threadIdx.x; i < len; i += kUnionThreads) srt[i] = 0x7fffffff;
        __syncthreads();
        for (int k = 2; k <= len; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < len; i += kUnionThreads) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const int a = srt[i], b = srt[ixj];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) { srt[i] = b; srt[ixj] = a; }
                    }
                }
                __syncthreads();
            }
    }
    // unique: each thread handles a contiguous span, block scan of the span counts
    int32_t* uq = tmp;
    const int per = (cnt + kUnionThreads - 1) / kUnionThreads;
    const int a0 = min(cnt, (int)threadIdx.x * per), a1 = min(cnt, a0 + per);
    int mine = 0;
    for (int i = a0; i < a1; ++i) mine += (i == 0 || srt[i] != srt[i - 1]);
    scan[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 1; off < kUnionThreads; off <<= 1) {
        const int v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int w = scan[threadIdx.x] - mine;
    for (int i = a0; i < a1; ++i)
        if (i == 0 || srt[i] != srt[i - 1]) {
            U[t0 + w] = srt[i];
            uq[w] = srt[i];
            ++w;
        }
    const int nu = scan[kUnionThreads - 1];
    if (threadIdx.x == 0) ucount[g] = nu;
    __syncthreads();
    // positions by binary search in U_g
    for (int t = t0 + threadIdx.x; t < t1; t += kUnionThreads)
        pos[t] = (static_cast<int>(rowof[t - t0]) << 16) | lower_in(uq, 0, nu, col[t]);
}

// Offsets of the groups' blocks (in elements): boff[g] = 16 * sum_{h<g} round4(|U_h|),
// boff[ngroups] = total; stats[1] = sum_g |U_g| (capped at INT_MAX). One work-group;
// each thread sums a contiguous span.
__global__ __launch_bounds__(1024) void k_grp_offsets(int ngroups, const int32_t* __restrict__ ucount,
                                                      int64_t* __restrict__ boff, int* __restrict__ stats) {
    __shared__ int64_t scan[1024];
    __shared__ unsigned long long usum;
    if (threadIdx.x == 0) usum = 0;
    const int per = (ngroups + 1023) / 1024;
    const int a0 = min(ngroups, (int)threadIdx.x * per), a1 = min(ngroups, a0 + per);
    int64_t mine = 0, mine_u = 0;
    for (int g = a0; g < a1; ++g) {
        mine += 16 * (int64_t)((ucount[g] + 3) & ~3);
        mine_u += ucount[g];
    }
    scan[threadIdx.x] = mine;
    __syncthreads();
    atomicAdd(&usum, (unsigned long long)mine_u);       // LDS atomic: one work-group only
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = scan[threadIdx.x] - mine;
    for (int g = a0; g < a1; ++g) {
        boff[g] = run;
        run += 16 * (int64_t)((ucount[g] + 3) & ~3);
    }
    if (threadIdx.x == 1023) boff[ngroups] = scan[1023];
    if (threadIdx.x == 0) stats[1] = (int)min<unsigned long long>(usum, 0x7fffffffull);
}

// Dense k-major block of group g: zero, then each CSR entry at [pos][row].
template <typename T>
__global__ __launch_bounds__(256) void k_grp_fill(int n, const int32_t* __restrict__ rp, const T* __restrict__ val,
                                                  const int32_t* __restrict__ ucount, const int32_t* __restrict__ pos,
                                                  const int64_t* __restrict__ boff, T* __restrict__ hblk) {
    const int g = blockIdx.x;
    const int r0 = g * kSpmmGroup;
    const int r1 = min(n, r0 + kSpmmGroup);
    T* B = hblk + boff[g];
    const int len = 16 * ((ucount[g] + 3) & ~3);
    for (int i = threadIdx.x; i < len; i += 256) B[i] = T(0);
    __syncthreads();
    for (int t = rp[r0] + threadIdx.x; t < rp[r1]; t += 256) {
        const int pp = pos[t];
        B[(pp & 0xffff) * kSpmmGroup + (pp >> 16)] = val[t];
    }
}

// Reads step st of this lane: A = Hg[4 st + lane/16][lane%16] and the V values of
// row U_g[c0 + 4 st + lane/16] (the q-element runs of every tile segment).
template <typename T, int NT>
__device__ inline void load_step(const T* __restrict__ Hb, const T* __restrict__ V, const int32_t* uidx, int ld,
                                 int st, int lane, int lr, int lc, T& a, T (&x)[NT]) {
    a = Hb[64 * st + lane];
    load_run<T, NT>(V + (int64_t)uidx[4 * st + lr] * ld, lc, x);
}

// One wavefront per group of 16 rows: W rows = Hg * V[U_g]. The union is walked in
// chunks of UC columns whose indices are staged in LDS; the A values and V values
// of each k-step (4 union columns) are fetched D steps ahead of their use. Loads
// past the chunk's last step repeat that step (in bounds) and are multiplied by
// zero. Work-groups are dealt round-robin to the 8 XCDs; XCD x takes the runs of
// `run` consecutive groups x, x + 8, x + 16, ... (block b: run (b / 8) / run * 8 + b % 8,
// group (b / 8) % run within it): an XCD's L2 sees neighbouring rows, and the eight
// XCDs sweep the rows together, so the V rows in use at any time stay in the MALL.
template <typename T, int NT, int UC, int D>
__global__ __launch_bounds__(64) void k_spmm_grp(int n, int ngroups, int run, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ U, const int32_t* __restrict__ ucount,
                                                 const int64_t* __restrict__ boff, const T* __restrict__ hblk,
                                                 const T* __restrict__ V, T* __restrict__ W, int ld) {
    typedef GMF<T> M;
    __shared__ int32_t uidx[UC];
    const int lane = threadIdx.x, lr = lane >> 4, lc = lane & 15;
    const int xi = (int)(blockIdx.x / 8);
    const int g = ((xi / run) * 8 + (int)(blockIdx.x % 8)) * run + xi % run;
    if (g >= ngroups) return;
    const int r0 = g * kSpmmGroup;
    const int r1 = min(n, r0 + kSpmmGroup);
    const int nu = ucount[g];
    const int32_t* Ug = U + rp[r0];
    typename M::acc c[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) c[t] = M::zero();
    for (int c0 = 0; c0 < nu; c0 += UC) {
        const int uc = min(UC, nu - c0);
        const int nst = (uc + 3) >> 2;
        const T* Hb = hblk + boff[g] + 16 * (int64_t)c0;
        int iv[UC / 64];
#pragma unroll
        for (int j = 0; j < UC / 64; ++j) iv[j] = Ug[c0 + min(lane + 64 * j, uc - 1)];
#pragma unroll
        for (int j = 0; j < UC / 64; ++j) uidx[lane + 64 * j] = iv[j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        T a[D];
        T x[D][NT];
#pragma unroll
        for (int d = 0; d < D; ++d) load_step<T, NT>(Hb, V, uidx, ld, min(d, nst - 1), lane, lr, lc, a[d], x[d]);
        for (int s0 = 0; s0 < nst; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const T av = (s0 + d < nst) ? a[d] : T(0);
#pragma unroll
                for (int t = 0; t < NT; ++t) c[t] = M::mma(av, x[d][t], c[t]);
                load_step<T, NT>(Hb, V, uidx, ld, min(s0 + d + D, nst - 1), lane, lr, lc, a[d], x[d]);
                __builtin_amdgcn_sched_barrier(0);   // keep each step's loads D steps ahead of their use
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = r0 + M::row(lane, r);
        if (row >= r1) continue;
        T y[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) y[t] = c[t][r];
        store_run<T, NT>(W + (int64_t)row * ld, lc, y);
    }
}

template <typename T, int NT>
void launch_grp(const SpmmArgs<T>& a, const SpmmGroups& gp, const Tuning& tu, hipStream_t s) {
    constexpr int UC = 256;                           // union columns per index chunk
    // groups per XCD run: at most 512 by default (on 10^6 water 512 beat one contiguous
    // range per XCD by 7%; at 10k, 469 groups per XCD, one range per XCD moved the
    // fewest bytes)
    const int ngroups = spmm_groups(a.n);
    const int run = std::max(1, std::min(tu.run > 0 ? tu.run : 512, (ngroups + 7) / 8));
    const int nruns = (ngroups + run - 1) / run;
    const int blocks = 8 * ((nruns + 7) / 8) * run;
    // k-steps in flight per wave: 4 by default (10k water 47.1 against 49.6 us with 8,
    // 10^6 water 3.61 against 3.72 ms)
    if (tu.depth == 8)
        k_spmm_grp<T, NT, UC, 8><<<blocks, 64, 0, s>>>(a.n, ngroups, run, a.row_ptr, gp.U, gp.ucount, gp.boff,
                                                       static_cast<const T*>(gp.hblk), a.V, a.W, a.ld);
    else
        k_spmm_grp<T, NT, UC, 4><<<blocks, 64, 0, s>>>(a.n, ngroups, run, a.row_ptr, gp.U, gp.ucount, gp.boff,
                                                       static_cast<const T*>(gp.hblk), a.V, a.W, a.ld);
}

}  // namespace

int spmm_groups(int n) { return (n + kSpmmGroup - 1) / kSpmmGroup; }

int64_t spmm_grp_block_cap(int n, int64_t nnz) { return (int64_t)kGroupFill * nnz + 48 * (int64_t)spmm_groups(n); }

void carve_groups(Arena& a, int n, int64_t nnz, size_t elem, SpmmGroups& g) {
    const int ng = spmm_groups(n);
    g.U = a.take<int32_t>(std::max<int64_t>(1, nnz));
    g.pos = a.take<int32_t>(std::max<int64_t>(1, nnz));
    g.ucount = a.take<int32_t>(ng);
    g.boff = a.take<int64_t>(ng + 1);
    g.cap = spmm_grp_block_cap(n, nnz);
    g.hblk = a.take<char>((size_t)g.cap * elem);
}

void spmm_grp_prepare(int n, const int32_t* row_ptr, const int32_t* col, const SpmmGroups& gp, int* stats,
                      hipStream_t s) {
    k_grp_union<<<spmm_groups(n), kUnionThreads, 0, s>>>(n, row_ptr, col, gp.U, gp.ucount, gp.pos, stats);
    k_grp_offsets<<<1, 1024, 0, s>>>(spmm_groups(n), gp.ucount, gp.boff, stats);
}

bool spmm_grp_worthwhile(int64_t nnz, int too_long, int64_t sum_union) {
    return too_long == 0 && (int64_t)kSpmmGroup * sum_union <= (int64_t)kGroupFill * std::max<int64_t>(1, nnz);
}

template <typename T>
void spmm_grp_fill(int n, const int32_t* row_ptr, const T* val, const SpmmGroups& gp, hipStream_t s) {
    const int ng = spmm_groups(n);
    k_grp_fill<T><<<ng, 256, 0, s>>>(n, row_ptr, val, gp.ucount, gp.pos, gp.boff, static_cast<T*>(gp.hblk));
}

template <typename T>
bool spmm_grp_launch(const SpmmArgs<T>& a, const SpmmGroups& gp, const Tuning& tu, hipStream_t s) {
    if (!gp.blocks_ready || a.ld % 16 != 0 ||
        (reinterpret_cast<uintptr_t>(a.V) | reinterpret_cast<uintptr_t>(a.W)) % 16 != 0)
        return false;
    switch (a.ld / 16) {
        case 1: launch_grp<T, 1>(a, gp, tu, s); return true;
        case 2: launch_grp<T, 2>(a, gp, tu, s); return true;
        case 3: launch_grp<T, 3>(a, gp, tu, s); return true;
        case 4: launch_grp<T, 4>(a, gp, tu, s); return true;
        case 5: launch_grp<T, 5>(a, gp, tu, s); return true;
        case 6: launch_grp<T, 6>(a, gp, tu, s); return true;
        case 7: launch_grp<T, 7>(a, gp, tu, s); return true;
        case 8: launch_grp<T, 8>(a, gp, tu, s); return true;
        default: return false;      // wider blocks use the CSR kernel
    }
}

template <typename T>
bool spmm_grouped_launch(const SpmmArgs<T>& a, const SpmmGroups& gp, hipStream_t s) {
    const Tuning tu = tuning();
    return tu.kernel != 2 && spmm_grp_launch(a, gp, tu, s);
}

template void spmm_grp_fill<double>(int, const int32_t*, const double*, const SpmmGroups&, hipStream_t);
template void spmm_grp_fill<float>(int, const int32_t*, const float*, const SpmmGroups&, hipStream_t);
template bool spmm_grp_launch<double>(const SpmmArgs<double>&, const SpmmGroups&, const Tuning&, hipStream_t);
template bool spmm_grp_launch<float>(const SpmmArgs<float>&, const SpmmGroups&, const Tuning&, hipStream_t);
template bool spmm_grouped_launch<double>(const SpmmArgs<double>&, const SpmmGroups&, hipStream_t);
template bool spmm_grouped_launch<float>(const SpmmArgs<float>&, const SpmmGroups&, hipStream_t);

}  // namespace css
