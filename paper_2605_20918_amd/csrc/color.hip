// Conflict graph (= sparsity pattern of P) and greedy multicolouring on the GPU.
//
// Method: the text around Eq.(2) colours orbitals greedily in the manner of
// Welsh and Powell so that any two orbitals closer than the cutoff differ
// (Fig.1(b)). The sequential algorithm visits orbitals by degree descending
// (ties: smaller index first) and gives each the smallest colour not used by
// its already coloured neighbours. Those are exactly its higher-priority
// neighbours (Welsh-Powell rank), so the greedy colours are the unique solution
// of c(v) = mex{ c(u) : u a higher-priority neighbour of v }. It is found here by
// in-place fixed-point sweeps that re-evaluate only orbitals whose inputs
// changed; the first sweep without a change certifies the solution. On water
// the sweeps needed stay near a hundred at any size, while the dependency depth
// that a round-by-round (Jones-Plassmann) colouring has to walk grows with the
// system (about a thousand levels at 60 000 orbitals, ten thousand at 6 million).
//
// The distance predicate is evaluated with separately rounded products and
// sums (no fused multiply-add) so that every conflict decision is identical
// to a plain IEEE evaluation of ((dx*dx + dy*dy) + dz*dz) <= r_cut*r_cut.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "css_common.h"

namespace css {
namespace {

constexpr int kMaxRowLds = 8192;     // longest pattern row the LDS row sort handles

struct Grid {
    int nc[3];          // cells per dimension
    double w[3];        // cell width (>= r_cut)
    double lo[3];       // origin (open directions) / 0 (periodic)
    double L[3];        // box edge, 0 = open
    double invL[3];     // 1 / L (0 for open directions)
};

__device__ __forceinline__ int cell_coord(double x, int k, const Grid& g) {
    double t;
    if (g.L[k] > 0.0) {
        t = x - g.L[k] * floor(x / g.L[k]);
    } else {
        t = x - g.lo[k];
    }
    int c = static_cast<int>(floor(t / g.w[k]));
    return c < 0 ? 0 : (c >= g.nc[k] ? g.nc[k] - 1 : c);
}

// Bounding box in two levels: every work-group's min and max per coordinate to
// part[6 blockIdx.x ..], then one work-group over the parts (min and max are
// order independent).
constexpr int kBboxBlocks = 256;

__global__ __launch_bounds__(256) void k_bbox(const double* __restrict__ xyz, int64_t n, int stride,
                                              double* __restrict__ out) {
    __shared__ double smin[3][256], smax[3][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], xyz[stride * i + k]);
            mx[k] = fmax(mx[k], xyz[stride * i + (stride == 3 ? k : 3 + k)]);
        }
    for (int k = 0; k < 3; ++k) { smin[k][threadIdx.x] = mn[k]; smax[k][threadIdx.x] = mx[k]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
                smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) { out[6 * blockIdx.x + k] = smin[k][0]; out[6 * blockIdx.x + 3 + k] = smax[k][0]; }
}

__global__ void k_finite_check(const double* __restrict__ xyz, int64_t cnt, int* __restrict__ bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt && !isfinite(xyz[i])) atomicOr(bad, 1);
}

__global__ void k_bin(const double* __restrict__ xyz, int n, Grid g, int* __restrict__ cell_of,
                      int* __restrict__ cell_count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(xyz[3 * (int64_t)i], 0, g);
    int cy = cell_coord(xyz[3 * (int64_t)i + 1], 1, g);
    int cz = cell_coord(xyz[3 * (int64_t)i + 2], 2, g);
    int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = c;
    atomicAdd(&cell_count[c], 1);
}

__global__ void k_place(int n, const int* __restrict__ cell_of, const int* __restrict__ cell_start,
                        int* __restrict__ cell_fill, int* __restrict__ cell_list) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int pos = cell_start[c] + atomicAdd(&cell_fill[c], 1);
    cell_list[pos] = i;
}

// Stencil offsets along one dimension: all distinct neighbouring cells.
__device__ __forceinline__ int stencil(int nc, bool periodic, int c, int o[3]) {
    if (nc == 1) { o[0] = 0; return 1; }
    if (periodic) {
        if (nc == 2) { o[0] = 0; o[1] = 1; return 2; }
        o[0] = (c + nc - 1) % nc; o[1] = c; o[2] = (c + 1) % nc; return 3;
    }
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
        int cc = c + d;
        if (cc >= 0 && cc < nc) o[k++] = cc;
    }
    return k;
}

// Minimum-image difference dk - L rint(dk / L). The integer rint(dk / L) is taken
// from dk * (1/L) unless that product lies within a relative 1e-9 of a
// half-integer (then from the IEEE quotient): away from ties both round to the
// same integer, so the result is bitwise the plain formula's.
__device__ __forceinline__ double min_image(double dk, double L, double invL) {
#pragma clang fp contract(off)
    const double t = dk * invL;
    double q = rint(t);
    if (fabs(fabs(t - q) - 0.5) <= 1e-9 * fmax(1.0, fabs(t))) q = rint(dk / L);
    const double s = L * q;
    return dk - s;
}

// Conflict pairs, one work-group per cell: the cell's orbitals are taken 64 at a
// time (one per lane) and the orbitals of the (up to 27) neighbouring cells are
// staged through LDS kCandChunk at a time, the four wavefronts taking every
// fourth candidate (a broadcast read). Every conflict decision is the plain
// ((dx*dx + dy*dy) + dz*dz) <= r_cut^2, products and sums rounded separately.
// COUNT = true: deg[m] = number of conflicting partners (self excluded), and, when
// rows_tmp is given, the row (self included, unsorted) in the first kRowTmp slots of
// rows_tmp[m kRowTmp ..]; when every row fits there, the second pass is not run and
// the sort reads the rows from rows_tmp (water at r_cut = 6 A: rows of 169 entries
// on average and at most 206 at 10^4 molecules, where the two passes took 214 +
// 226 us). The slots are kept for up to kRowTmpMaxN orbitals (1 GB), so larger
// systems take the second pass and no more memory.
// COUNT = false: write the row (self included) at p_col[p_row_ptr[m] ...] unsorted.
constexpr int kPairThreads = 256;
constexpr int kRowTmp = 256;
constexpr int kRowTmpMaxN = 1 << 20;
constexpr int kCandChunk = 1024;

template <bool COUNT>
__global__ __launch_bounds__(kPairThreads) void k_cell_pairs(const double* __restrict__ xyz, Grid g, double rc2,
                                                             const int* __restrict__ cell_start,
                                                             const int* __restrict__ cell_list, int* __restrict__ deg,
                                                             const int64_t* __restrict__ p_row_ptr,
                                                             int32_t* __restrict__ p_col, int32_t* __restrict__ rows_tmp) {
#pragma clang fp contract(off)
    __shared__ double sx[kCandChunk], sy[kCandChunk], sz[kCandChunk];
    __shared__ int sid[kCandChunk];
    __shared__ int ncells, ccell[27], cpre[28];
    __shared__ int cnt[64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x;
    const int os = cell_start[c], oe = cell_start[c + 1];
    if (os == oe) return;
    if (threadIdx.x == 0) {
        const int kz = c % g.nc[2], ky = (c / g.nc[2]) % g.nc[1], kx = c / (g.nc[2] * g.nc[1]);
        int ox[3], oy[3], oz[3];
        const int nx = stencil(g.nc[0], g.L[0] > 0.0, kx, ox);
        const int ny = stencil(g.nc[1], g.L[1] > 0.0, ky, oy);
        const int nz = stencil(g.nc[2], g.L[2] > 0.0, kz, oz);
        int k = 0;
        cpre[0] = 0;
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < ny; ++b)
                for (int d = 0; d < nz; ++d) {
                    const int cc = (ox[a] * g.nc[1] + oy[b]) * g.nc[2] + oz[d];
                    ccell[k] = cc;
                    cpre[k + 1] = cpre[k] + (cell_start[cc + 1] - cell_start[cc]);
                    ++k;
                }
        ncells = k;
    }
    __syncthreads();
    const int total = cpre[ncells];
    for (int o0 = os; o0 < oe; o0 += 64) {
        const int on = min(64, oe - o0);
        const bool own = lane < on;
        const int m = cell_list[o0 + (own ? lane : 0)];
        const double mx = xyz[3 * (int64_t)m], my = xyz[3 * (int64_t)m + 1], mz = xyz[3 * (int64_t)m + 2];
        const int64_t rbase = COUNT ? 0 : p_row_ptr[m];
        if (threadIdx.x < 64) cnt[threadIdx.x] = 0;
        for (int j0 = 0; j0 < total; j0 += kCandChunk) {
            const int jn = min(kCandChunk, total - j0);
            __syncthreads();                       // counters zeroed / previous chunk consumed
            for (int q = threadIdx.x; q < jn; q += kPairThreads) {
                const int gj = j0 + q;
                int k = 0;
                while (cpre[k + 1] <= gj) ++k;
                const int nb = cell_list[cell_start[ccell[k]] + (gj - cpre[k])];
                sid[q] = nb;
                sx[q] = xyz[3 * (int64_t)nb];
                sy[q] = xyz[3 * (int64_t)nb + 1];
                sz[q] = xyz[3 * (int64_t)nb + 2];
            }
            __syncthreads();
            if (own)
                for (int q = w; q < jn; q += kPairThreads / 64) {
                    const int nb = sid[q];
                    bool hit = nb == m;
                    if (!hit) {
                        double dx = sx[q] - mx, dy = sy[q] - my, dz = sz[q] - mz;
                        if (g.L[0] > 0.0) dx = min_image(dx, g.L[0], g.invL[0]);
                        if (g.L[1] > 0.0) dy = min_image(dy, g.L[1], g.invL[1]);
                        if (g.L[2] > 0.0) dz = min_image(dz, g.L[2], g.invL[2]);
                        const double a = dx * dx;
                        const double b = dy * dy;
                        const double e = dz * dz;
                        const double ab = a + b;
                        hit = ab + e <= rc2;
                    }
                    if (hit) {
                        const int slot = atomicAdd(&cnt[lane], 1);
                        if (!COUNT) p_col[rbase + slot] = nb;
                        else if (rows_tmp && slot < kRowTmp) rows_tmp[(int64_t)m * kRowTmp + slot] = nb;
                    }
                }
        }
        __syncthreads();
        if (COUNT && threadIdx.x < on) deg[cell_list[o0 + threadIdx.x]] = cnt[threadIdx.x] - 1;   // self once
        __syncthreads();
    }
}

// Sort each pattern row ascending by rank (entries are distinct): one wavefront per
// row, the row in a per-wavefront LDS slice of kSortWaveRow entries, each lane
// placing its entries by counting the smaller ones. Used when every row fits; one
// work-group per row with a kMaxRowLds slice otherwise (k_sort_rows). The row is
// padded to 16 entries and compared 16 at a time from four 16-byte LDS reads in
// flight. At 10^4 water molecules (60 000 rows of about 169 entries): 112 us, against
// 185 us for the work-group-per-row sort (five 32 KB work-groups per compute unit)
// and 247 us for this one comparing one entry per LDS read and wait.
constexpr int kSortWaveRow = 512;

// Orders the wavefront's LDS accesses across its lanes (fences on LDS only: a
// wavefront-scope release on all memory would also wait for its global stores).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__global__ __launch_bounds__(256) void k_sort_rows_wave(int n, const int64_t* __restrict__ p_row_ptr,
                                                        const int32_t* __restrict__ rows_tmp, int32_t* __restrict__ p_col) {
    // rows_tmp: the rows in slots of kRowTmp per orbital (every row fits, checked by the
    // host), or nullptr: the rows are read from p_col in place
    static_assert(kSortWaveRow % 16 == 0, "rows are padded to 16 entries");
    __shared__ int4 rows[4][kSortWaveRow / 4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    int32_t* row = reinterpret_cast<int32_t*>(rows[w]);
    for (int m = blockIdx.x * 4 + w; m < n; m += gridDim.x * 4) {
        const int64_t s = p_row_ptr[m];
        // <= kSortWaveRow (checked by the host); the padding INT_MAX is never smaller
        // than an entry (entries are column indices below n)
        const int len = __builtin_amdgcn_readfirstlane(static_cast<int>(p_row_ptr[m + 1] - s));
        const int len16 = (len + 15) & ~15;
        const int32_t* src = rows_tmp ? rows_tmp + (int64_t)m * kRowTmp : p_col + s;
        for (int i = lane; i < len16; i += 64) row[i] = i < len ? src[i] : INT_MAX;
        wave_sync_lds();
        for (int i = lane; i < len; i += 64) {
            const int32_t x = row[i];
            int r = 0;
            for (int k = 0; k < len16 / 4; k += 4) {        // 16 entries, four 16-byte reads in flight
                const int4 a = rows[w][k], b = rows[w][k + 1], c = rows[w][k + 2], d = rows[w][k + 3];
                r += (a.x < x) + (a.y < x) + (a.z < x) + (a.w < x) + (b.x < x) + (b.y < x) + (b.z < x) +
                     (b.w < x) + (c.x < x) + (c.y < x) + (c.z < x) + (c.w < x) + (d.x < x) + (d.y < x) +
                     (d.z < x) + (d.w < x);
            }
            p_col[s + r] = x;
        }
        wave_sync_lds();                                                // row[] is reused for the next row
    }
}

__global__ void k_sort_rows(int n, const int64_t* __restrict__ p_row_ptr, int32_t* __restrict__ p_col) {
    __shared__ int32_t row[kMaxRowLds];
    int m = blockIdx.x;
    if (m >= n) return;
    int64_t s = p_row_ptr[m];
    int len = static_cast<int>(p_row_ptr[m + 1] - s);
    for (int i = threadIdx.x; i < len; i += blockDim.x) row[i] = p_col[s + i];
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        int32_t x = row[i];
        int r = 0;
        for (int k = 0; k < len; ++k) r += (row[k] < x);
        p_col[s + r] = x;
    }
}

__device__ __forceinline__ bool higher_priority(int du, int u, int dv, int v) {
    return du > dv || (du == dv && u < v);
}

// Pattern entries of higher-priority neighbours carry this flag in the sign bit of
// their column index while the colouring runs; k_clear_flags removes it.
constexpr int32_t kHpFlag = int32_t(0x80000000u);

// Flags every row's higher-priority entries, starts every colour at 0 and makes
// every orbital due in sweep 0 (stamp 0). One wavefront per orbital.
__global__ __launch_bounds__(256) void k_fp_init(int n, const int64_t* __restrict__ p_row_ptr,
                                                 int32_t* __restrict__ p_col, const int* __restrict__ deg,
                                                 int* __restrict__ color, int* __restrict__ stamp) {
    const int lane = threadIdx.x & 63;
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    const int dv = deg[v];
    for (int64_t t = p_row_ptr[v] + lane; t < p_row_ptr[v + 1]; t += 64) {
        const int u = p_col[t];
        if (u != v && higher_priority(deg[u], u, dv, v)) p_col[t] = u | kHpFlag;
    }
    if (lane == 0) {
        color[v] = 0;
        stamp[v] = 0;
    }
}

__global__ void k_clear_flags(int32_t* __restrict__ p_col, int64_t nnz) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nnz) p_col[t] &= ~kHpFlag;
}

// One sweep k of the fixed-point iteration c(v) = mex{ c(u) : u a higher-priority
// neighbour of v }. Its solution is unique (the priority relation is acyclic,
// so it is fixed level by level) and it is the sequential greedy colouring:
// there, v receives the smallest colour absent from its already coloured
// neighbours, which are exactly its higher-priority ones. Only orbitals with
// stamp k are evaluated; one whose colour changes stamps its lower-priority
// neighbours k + 1 (plain stores: every writer writes the same value, and a
// stamp only grows). Updates are in place; an orbital read before a neighbour's
// change in the same sweep is stamped and evaluated again in the next one, so
// the first sweep in which nothing changes leaves every orbital satisfying its
// equation: the iteration has converged to the greedy colouring.
// A wavefront owns kFpChunk consecutive orbitals (one load per lane brings their
// stamps, colours, degrees and row bounds) and evaluates the due ones one after
// the other in priority order, so that an orbital can already see the new colour
// of a higher-priority neighbour of the same chunk (consecutive orbitals are
// mostly on one molecule). A row is read kFpLoads entries per lane at a time; the
// first batch of every due orbital's row is requested before the first is used.
// Water colourings, whole call, 64 sweeps per host check: 4 orbitals per
// wavefront 2.77 ms at 10^4 molecules and 14.6 ms at 10^5; 8 orbitals 2.69 and
// 17.1 ms (fewer sweeps, 63 and 67 against 66 and 80, but a longer serial chain per
// wavefront); 2 loads per lane instead of 4, 2.87 and 15.2 ms. With the mex masks
// reduced by LDS lane permutes instead of the VALU moves of wave_or: 3.16 and
// 17.1 ms; with stamps read before they are written as well, and 8 orbitals, 3.12
// and 21.1 ms. Issuing the colour gathers of the due orbitals' first 64 entries
// before the first evaluation was slower: 3.45 against 2.41 ms at 10^4 (80 sweeps
// per host check), more sweeps and dearer ones.
constexpr int kFpChunk = 4;
// Colouring sweeps per host check. A call whose sweeps run past a batch pays for
// a whole further batch (launches that return at once, one more host round trip):
// water needs about 66 sweeps at 10^4 molecules, where 80 per check gave 2.40 ms
// per colouring against 2.62 ms with 64.
constexpr int kFpBatch = 80;
constexpr int kFpLoads = 4;
constexpr int kFpSpan = 64 * kFpLoads;               // row entries per batch

__device__ __forceinline__ void mex_mark(int cu, int base, unsigned long long (&m)[4]) {
    const int cc = cu - base;
    const bool in = cu >= 0 && cc >= 0 && cc < 256;
    const unsigned long long bit = in ? 1ull << (cc & 63) : 0ull;
    const int word = cc >> 6;
    m[0] |= word == 0 ? bit : 0ull;
    m[1] |= word == 1 ? bit : 0ull;
    m[2] |= word == 2 ? bit : 0ull;
    m[3] |= word == 3 ? bit : 0ull;
}

// OR of x over the 64 lanes of the wavefront, in every lane, on VALU cross-lane
// moves only: within each 16-lane row by DPP (swap neighbours, swap pairs, mirror
// the half rows, mirror the rows), then across the four rows by the two lane-swap
// instructions (the 32-lane swap pairs rows 0-2 and 1-3, the 16-lane swap 0-1 and 2-3).
__device__ __forceinline__ unsigned wave_or(unsigned x) {
    x |= static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0xB1, 0xf, 0xf, false));
    x |= static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x4E, 0xf, 0xf, false));
    x |= static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x141, 0xf, 0xf, false));
    x |= static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x140, 0xf, 0xf, false));
    const auto h = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    x = static_cast<unsigned>(h[0]) | static_cast<unsigned>(h[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return static_cast<unsigned>(q[0]) | static_cast<unsigned>(q[1]);
}

// Smallest colour >= base absent from the wave's masks (-1 if all 256 are present).
__device__ __forceinline__ int mex_of(unsigned long long (&m)[4], int base) {
#pragma unroll
    for (int wd = 0; wd < 4; ++wd)
        m[wd] = static_cast<unsigned long long>(wave_or(static_cast<unsigned>(m[wd]))) |
                static_cast<unsigned long long>(wave_or(static_cast<unsigned>(m[wd] >> 32))) << 32;
    if (~m[0]) return base + __builtin_ctzll(~m[0]);
    if (~m[1]) return base + 64 + __builtin_ctzll(~m[1]);
    if (~m[2]) return base + 128 + __builtin_ctzll(~m[2]);
    if (~m[3]) return base + 192 + __builtin_ctzll(~m[3]);
    return -1;
}

// v of lane `src` (uniform) in every lane
__device__ __forceinline__ int lane_int(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ int64_t lane_i64(int64_t v, int src) {
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v & 0xffffffffLL), src));
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), src);
    return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | lo);
}

// Stamps the lower-priority neighbours among a batch of row entries (entry q of
// this lane at index t + 64 q) with `next`. Plain stores, not read first: every
// writer in this sweep writes the same value and no stamp is larger during it, so
// a store loses nothing (reading the stamp first, to skip the stores most
// neighbours do not need, took longer: 3.12 against 2.99 ms per 10k colouring).
__device__ __forceinline__ void mark_lower(const int (&u)[kFpLoads], int v, int64_t t, int64_t e, int next,
                                           int* stamp) {
#pragma unroll
    for (int q = 0; q < kFpLoads; ++q)
        if (u[q] >= 0 && u[q] != v && t + 64 * q < e) stamp[u[q]] = next;
}

__global__ __launch_bounds__(256) void k_fp_sweep(int n, const int64_t* __restrict__ p_row_ptr,
                                                  const int32_t* __restrict__ p_col, const int* __restrict__ deg,
                                                  int* color, int* stamp, int k, int* __restrict__ changed,
                                                  const int* __restrict__ prev_changed) {
    // changed: set to 1 if this sweep changed a colour (cleared by the host before).
    // prev_changed (may be nullptr): the previous sweep's flag; if it changed nothing,
    // no orbital carries stamp k and this sweep is a no-op, so it returns at once
    if (prev_changed && *prev_changed == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    int nchanged = 0;
    for (int64_t v0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kFpChunk; v0 < n; v0 += nwaves * kFpChunk) {
        const int64_t vl = min<int64_t>(v0 + lane % kFpChunk, n - 1);
        const int st = stamp[vl], cl = color[vl], dl = deg[vl];
        __builtin_amdgcn_sched_barrier(0);
        const bool due = lane < kFpChunk && v0 + lane < n && st == k;
        const unsigned long long dm = __ballot(due);
        if (!dm) continue;
        const int64_t rs = p_row_ptr[vl], re = p_row_ptr[vl + 1];
        // rank among the due orbitals of the chunk: the number of higher-priority ones
        int rank = 0;
#pragma unroll
        for (int j = 0; j < kFpChunk; ++j) {
            const int dj = lane_int(dl, j);
            rank += ((dm >> j) & 1) && (dj > dl || (dj == dl && j < lane));
        }
        const int ndue = __popcll(dm);
        // first batch of every due orbital's row, in evaluation order, all in flight at once
        int src[kFpChunk];
        int u[kFpChunk][kFpLoads];
#pragma unroll
        for (int r = 0; r < kFpChunk; ++r) {
            const unsigned long long b = __ballot(due && rank == r);
            src[r] = b ? __builtin_ctzll(b) : 0;
            const int64_t sr = lane_i64(rs, src[r]), er = lane_i64(re, src[r]);
#pragma unroll
            for (int q = 0; q < kFpLoads; ++q) u[r][q] = p_col[min(sr + lane + 64 * q, er - 1)];
        }
        for (int r = 0; r < ndue; ++r) {
            const int v = static_cast<int>(v0) + src[0];
            const int cur = lane_int(cl, src[0]);
            const int64_t s = lane_i64(rs, src[0]), e = lane_i64(re, src[0]);
            int cu[kFpLoads];
#pragma unroll
            for (int q = 0; q < kFpLoads; ++q) {
                const bool hp = u[0][q] < 0 && s + lane + 64 * q < e;
                cu[q] = hp ? color[u[0][q] & ~kHpFlag] : -1;
            }
            unsigned long long m[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
            for (int q = 0; q < kFpLoads; ++q) mex_mark(cu[q], 0, m);
            // the rest of a long row
            for (int64_t tb = s + lane + kFpSpan; __ballot(tb < e); tb += kFpSpan) {
                int w[kFpLoads], cw[kFpLoads];
#pragma unroll
                for (int q = 0; q < kFpLoads; ++q) w[q] = p_col[min(tb + 64 * q, e - 1)];
#pragma unroll
                for (int q = 0; q < kFpLoads; ++q) cw[q] = (w[q] < 0 && tb + 64 * q < e) ? color[w[q] & ~kHpFlag] : -1;
#pragma unroll
                for (int q = 0; q < kFpLoads; ++q) mex_mark(cw[q], 0, m);
            }
            int chosen = mex_of(m, 0);
            // colours beyond 255: further windows over the whole row
            for (int base = 256; chosen < 0 && base <= e - s; base += 256) {
                unsigned long long mb[4] = {0ull, 0ull, 0ull, 0ull};
                for (int64_t tb = s + lane; __ballot(tb < e); tb += kFpSpan) {
                    int w[kFpLoads], cw[kFpLoads];
#pragma unroll
                    for (int q = 0; q < kFpLoads; ++q) w[q] = p_col[min(tb + 64 * q, e - 1)];
#pragma unroll
                    for (int q = 0; q < kFpLoads; ++q) cw[q] = (w[q] < 0 && tb + 64 * q < e) ? color[w[q] & ~kHpFlag] : -1;
#pragma unroll
                    for (int q = 0; q < kFpLoads; ++q) mex_mark(cw[q], base, mb);
                }
                chosen = mex_of(mb, base);
            }
            chosen = chosen < 0 ? 0 : chosen;            // unreachable: the mex of L colours is <= L
            if (chosen != cur) {
                if (lane == 0) color[v] = chosen;
                ++nchanged;
                mark_lower(u[0], v, s + lane, e, k + 1, stamp);
                for (int64_t tb = s + lane + kFpSpan; __ballot(tb < e); tb += kFpSpan) {
                    int w[kFpLoads];
#pragma unroll
                    for (int q = 0; q < kFpLoads; ++q) w[q] = p_col[min(tb + 64 * q, e - 1)];
                    mark_lower(w, v, tb, e, k + 1, stamp);
                }
            }
            // next orbital's row to the front
#pragma unroll
            for (int i = 0; i + 1 < kFpChunk; ++i) {
                src[i] = src[i + 1];
#pragma unroll
                for (int q = 0; q < kFpLoads; ++q) u[i][q] = u[i + 1][q];
            }
        }
    }
    // a plain store of the same value by every wave that changed something: device-wide
    // atomics on one address would serialise thousands of waves
    if (lane == 0 && nchanged > 0) *changed = 1;
}

// Exclusive scan of the n cell counts into start[0 .. n] (start[n] = total) by one
// work-group: each thread adds a contiguous segment, the segment sums are scanned in
// LDS, then each thread writes its segment's prefixes.
constexpr int kCellScanThreads = 256;
__global__ __launch_bounds__(kCellScanThreads) void k_cell_scan(const int* __restrict__ count, int n,
                                                                int* __restrict__ start) {
    __shared__ int part[kCellScanThreads];
    const int t = threadIdx.x;
    const int per = (n + kCellScanThreads - 1) / kCellScanThreads;
    const int a = min(n, t * per), e = min(n, a + per);
    int sum = 0;
    for (int c = a; c < e; ++c) sum += count[c];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int q = 0; q < kCellScanThreads; ++q) {
            const int v = part[q];
            part[q] = run;
            run += v;
        }
        start[n] = run;
    }
    __syncthreads();
    int run = part[t];
    for (int c = a; c < e; ++c) {
        start[c] = run;
        run += count[c];
    }
}

__global__ void k_fill_int(int* __restrict__ p, int64_t cnt, int v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

__global__ void k_max_color(const int* __restrict__ color, int n, int* __restrict__ out, int* __restrict__ maxrow,
                            const int64_t* __restrict__ p_row_ptr) {
    __shared__ int sc[256], sr[256];
    int mc = -1, mr = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (color) mc = max(mc, color[i]);
        mr = max(mr, static_cast<int>(min<int64_t>(p_row_ptr[i + 1] - p_row_ptr[i], INT_MAX)));
    }
    sc[threadIdx.x] = mc;
    sr[threadIdx.x] = mr;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sc[threadIdx.x] = max(sc[threadIdx.x], sc[threadIdx.x + s]);
            sr[threadIdx.x] = max(sr[threadIdx.x], sr[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { atomicMax(out, sc[0]); atomicMax(maxrow, sr[0]); }
}

// ---- exclusive scan of (deg[i] + 1) into int64 row pointers -----------------

constexpr int kScanBlock = 1024;

__global__ void k_scan_blocks(const int* __restrict__ deg, int n, int64_t* __restrict__ out,
                              int64_t* __restrict__ block_sum) {
    __shared__ int64_t s[kScanBlock];
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    int64_t v = (i < n) ? (int64_t)deg[i] + 1 : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t t = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i + 1] = s[threadIdx.x];          // inclusive within block, shifted
    if (threadIdx.x == kScanBlock - 1) block_sum[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_sums(int64_t* __restrict__ block_sum, int nb) {
    // single block: exclusive scan of the block sums in place (sequential chunks)
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    __shared__ int64_t s[kScanBlock];
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        int64_t v = (i < nb) ? block_sum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            int64_t t = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) block_sum[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry += s[threadIdx.x];
        __syncthreads();
    }
}

__global__ void k_scan_add(int64_t* __restrict__ out, int n, const int64_t* __restrict__ block_sum) {
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    if (i == 0) out[0] = 0;
    if (i < n) out[i + 1] += block_sum[blockIdx.x];
}

Grid make_grid(int n, const double box[3], double r_cut, const double bb[6]) {
    Grid g;
    const double wmin = r_cut * (1.0 + 1e-9);
    for (int k = 0; k < 3; ++k) {
        g.L[k] = box[k] > 0.0 ? box[k] : 0.0;
        double extent = g.L[k] > 0.0 ? g.L[k] : (bb[3 + k] - bb[k]);
        g.lo[k] = g.L[k] > 0.0 ? 0.0 : bb[k];
        long long c = extent > 0.0 ? static_cast<long long>(std::floor(extent / wmin)) : 1;
        g.nc[k] = static_cast<int>(std::max<long long>(1, std::min<long long>(c, 1 << 20)));
    }
    // cap the number of cells so the workspace stays O(n)
    const long long cap = 2LL * n + 64;
    while ((long long)g.nc[0] * g.nc[1] * g.nc[2] > cap) {
        int k = (g.nc[0] >= g.nc[1] && g.nc[0] >= g.nc[2]) ? 0 : (g.nc[1] >= g.nc[2] ? 1 : 2);
        g.nc[k] = std::max(1, g.nc[k] / 2);
    }
    for (int k = 0; k < 3; ++k) {
        double extent = g.L[k] > 0.0 ? g.L[k] : (bb[3 + k] - bb[k]);
        g.w[k] = extent > 0.0 ? extent / g.nc[k] : 1.0;
        if (g.w[k] < wmin) g.w[k] = wmin;   // open direction: cells may overhang the box
        g.invL[k] = g.L[k] > 0.0 ? 1.0 / g.L[k] : 0.0;
    }
    return g;
}

struct ColorWs {
    int *cell_of, *cell_count, *cell_start, *cell_fill, *cell_list, *deg, *scalars, *stamp;
    int32_t* rows_tmp;
    int64_t* block_sum;
    double *bbox, *bbox_part;
};

ColorWs carve_color(Arena& a, int n) {
    ColorWs w;
    int64_t ncell = 2LL * n + 64;
    w.cell_of = a.take<int>(n);
    w.cell_count = a.take<int>(ncell);
    w.cell_start = a.take<int>(ncell + 1);
    w.cell_fill = a.take<int>(ncell);
    w.cell_list = a.take<int>(n);
    w.deg = a.take<int>(n);
    w.stamp = a.take<int>(n);
    w.rows_tmp = n <= kRowTmpMaxN ? a.take<int32_t>(static_cast<size_t>(n) * kRowTmp) : nullptr;
    w.scalars = a.take<int>(16 + kFpBatch);
    w.block_sum = a.take<int64_t>((n + kScanBlock - 1) / kScanBlock + 1);
    w.bbox = a.take<double>(8);
    w.bbox_part = a.take<double>(6 * kBboxBlocks);
    return w;
}

}  // namespace

size_t color_workspace_bytes(int n) {
    Arena a;
    carve_color(a, n);
    return a.used + 256;
}

}  // namespace css

using namespace css;

extern "C" css_status css_color(const double* xyz, int32_t n, const double box[3], double r_cut,
                                int32_t* color, int32_t* n_colors, int64_t* p_row_ptr,
                                int32_t* p_col, int64_t* p_nnz, int32_t* rounds, void* ws,
                                size_t ws_bytes, void* stream) {
    if (n < 1 || xyz == nullptr || box == nullptr || p_row_ptr == nullptr || p_nnz == nullptr ||
        !(r_cut > 0.0) || !std::isfinite(r_cut) || ws == nullptr)
        return CSS_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!(box[k] >= 0.0) || !std::isfinite(box[k])) return CSS_E_ARG;
    if (p_col != nullptr && (color == nullptr || n_colors == nullptr)) return CSS_E_ARG;
    if (ws_bytes < color_workspace_bytes(n)) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);

    Arena ar;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    ColorWs w = carve_color(ar, n);
    if (ar.overflow) return CSS_E_WORKSPACE;

    // finite coordinates and bounding box (open directions)
    fill_launch<int>(w.scalars, 0, 16 + kFpBatch, s);
    k_finite_check<<<grid_for(3LL * n, 256), 256, 0, s>>>(xyz, 3LL * n, w.scalars);
    {
        // per-block boxes of the n centres (stride 3), then the box of those boxes (stride 6)
        const unsigned nb = std::min<unsigned>(kBboxBlocks, grid_for(n, 256));
        k_bbox<<<nb, 256, 0, s>>>(xyz, n, 3, w.bbox_part);
        k_bbox<<<1, 256, 0, s>>>(w.bbox_part, nb, 6, w.bbox);
    }
    double hb[8];
    int hbad = 0;
    CSS_HIP_TRY(hipMemcpyAsync(hb, w.bbox, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipMemcpyAsync(&hbad, w.scalars, sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (hbad) return CSS_E_NONFINITE;
    Grid g = make_grid(n, box, r_cut, hb);
    const int ncell = g.nc[0] * g.nc[1] * g.nc[2];
    const double rc2 = r_cut * r_cut;

    // cell list
    fill_launch<int>(w.cell_count, 0, ncell, s);
    fill_launch<int>(w.cell_fill, 0, ncell, s);
    k_bin<<<grid_for(n, 256), 256, 0, s>>>(xyz, n, g, w.cell_of, w.cell_count);
    k_cell_scan<<<1, kCellScanThreads, 0, s>>>(w.cell_count, ncell, w.cell_start);   // cell_start, on the device
    k_place<<<grid_for(n, 256), 256, 0, s>>>(n, w.cell_of, w.cell_start, w.cell_fill, w.cell_list);

    // degrees and row pointers
    k_cell_pairs<true><<<ncell, kPairThreads, 0, s>>>(xyz, g, rc2, w.cell_start, w.cell_list, w.deg, nullptr,
                                                      nullptr, n <= kRowTmpMaxN ? w.rows_tmp : nullptr);
    const int nblk = (n + kScanBlock - 1) / kScanBlock;
    k_scan_blocks<<<nblk, kScanBlock, 0, s>>>(w.deg, n, p_row_ptr, w.block_sum);
    k_scan_sums<<<1, kScanBlock, 0, s>>>(w.block_sum, nblk);
    k_scan_add<<<nblk, kScanBlock, 0, s>>>(p_row_ptr, n, w.block_sum);
    // nnz, and the longest row (it must fit the LDS row sort), in one host round trip
    fill_launch<int>(w.scalars, 0, 2, s);
    k_max_color<<<64, 256, 0, s>>>(nullptr, n, w.scalars, w.scalars + 1, p_row_ptr);
    int64_t nnz = 0;
    int hmax[2];
    CSS_HIP_TRY(hipMemcpyAsync(&nnz, p_row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipMemcpyAsync(hmax, w.scalars, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    const int64_t capacity = *p_nnz;
    *p_nnz = nnz;
    if (p_col == nullptr) return CSS_OK;                 // size query
    if (capacity < nnz) return CSS_E_CAPACITY;
    if (hmax[1] > kMaxRowLds) return CSS_E_UNSUPPORTED;

    // rows (self included) of at most kRowTmp entries are already in rows_tmp
    const bool rows_kept = n <= kRowTmpMaxN && hmax[1] <= kRowTmp;
    if (!rows_kept)
        k_cell_pairs<false><<<ncell, kPairThreads, 0, s>>>(xyz, g, rc2, w.cell_start, w.cell_list, w.deg, p_row_ptr,
                                                           p_col, nullptr);
    static_assert(kRowTmp <= kSortWaveRow, "kept rows go through the wavefront sort");
    if (hmax[1] <= kSortWaveRow)
        k_sort_rows_wave<<<static_cast<unsigned>(std::min<int64_t>(8192, (n + 3) / 4)), 256, 0, s>>>(
            n, p_row_ptr, rows_kept ? w.rows_tmp : nullptr, p_col);
    else
        k_sort_rows<<<n, 256, 0, s>>>(n, p_row_ptr, p_col);

    // fixed-point sweeps, kFpBatch per host check of the change counters; a sweep after
    // one that changed nothing returns at once, so a batch costs one host round trip
    int* stamp = w.stamp;
    int* changed = w.scalars + 16;                // kFpBatch change counters
    k_fp_init<<<grid_for(n, 4), 256, 0, s>>>(n, p_row_ptr, p_col, w.deg, color, stamp);
    const unsigned sgrid = static_cast<unsigned>(std::min<int64_t>(16384, (n + 4 * kFpChunk - 1) / (4 * kFpChunk)));
    int sweeps = 0;
    for (int k0 = 0; sweeps == 0; k0 += kFpBatch) {
        if (k0 > n + kFpBatch) return CSS_E_DEVICE;       // cannot happen: sweep k fixes priority level k
        fill_launch<int>(changed, 0, kFpBatch, s);
        for (int r = 0; r < kFpBatch; ++r)
            k_fp_sweep<<<sgrid, 256, 0, s>>>(n, p_row_ptr, p_col, w.deg, color, stamp, k0 + r, changed + r,
                                             r > 0 ? changed + r - 1 : nullptr);
        int hch[kFpBatch];
        CSS_HIP_TRY(hipMemcpyAsync(hch, changed, sizeof(hch), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        for (int r = 0; r < kFpBatch && sweeps == 0; ++r)
            if (hch[r] == 0) sweeps = k0 + r + 1;
    }
    k_clear_flags<<<grid_for(nnz, 256), 256, 0, s>>>(p_col, nnz);
    fill_launch<int>(w.scalars, -1, 1, s);
    fill_launch<int>(w.scalars + 1, 0, 1, s);
    k_max_color<<<64, 256, 0, s>>>(color, n, w.scalars, w.scalars + 1, p_row_ptr);
    int hc = 0;
    CSS_HIP_TRY(hipMemcpyAsync(&hc, w.scalars, sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    *n_colors = hc + 1;
    if (rounds) *rounds = sweeps;
    return CSS_OK;
}
