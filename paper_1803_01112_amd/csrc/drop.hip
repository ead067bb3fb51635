// drop.hip -- the feasibility-seeking sweep P_T on gfx950: block-iterative
// DROP (diagonally relaxed orthogonal projections) over blocks of B
// consecutive histories (arXiv 1803.01112, Section III-D; P_T in Appendix A).
//
// For block b, from one image x:
//   r_i = (b_i - a_i . x) / ||a_i||^2          every row i of the block
//   c_j = sum_i r_i a_ij,  s_j = #entries at j
//   x_j += lambda c_j / s_j                     where s_j > 0
// Blocks are applied one after another.
//
// Tile-wise form.  The entries of a block are grouped by 16 x 16-voxel image
// tile (tile lists, rows.hip).  One workgroup owns one tile:
//   finish (block b - 1): every entry of the tile's list takes r_i from its
//     row's dot product (complete after the previous launch), and the
//     tile's c_j and s_j are summed in LDS; the tile's voxels are updated
//     in LDS and written back once;
//   dots (block b): every entry multiplies its chord by the updated voxel
//     value in LDS; within a wavefront the products of one row (consecutive
//     in the list) are summed over their run with shuffles, and one atomic
//     per run adds the run's sum to the row's dot product.
// Both halves of one step touch only the workgroup's own tile of x, so one
// launch per block does both (the launch boundary is the only device-wide
// synchronisation, and finishes every row's dot product before it is
// used).  Row dot products are summed as 64-bit integers in units of
// 2^-36, corrections in units of 2^-40: integer sums are exact, so the
// results do not depend on the order in which workgroups or lanes add.  A
// correction larger than `big` (outside the guaranteed integer range) is
// summed in float64 instead; a product |a_ij x_j| above `dot_max` raises
// an error flag (bit 0) that the host reports as a range error, and an
// entry naming a row outside its block is skipped and raises bit 1.
#include <hip/hip_ext.h>

#include "device_common.hpp"
#include "tvs_internal.hpp"

namespace tvs {
namespace {

using dev::entry_chord;
using dev::kNoRow;
using dev::row_of;

constexpr double kDotUnit = 1.0 / kDotScale;
constexpr double kCorrUnit = 1.0 / kCorrScale;

// LDS of one tile workgroup.
struct TileLds {
    double x[kTileWords];
    long long cf[kTileWords];    // fixed-point correction sums
    double cb[kTileWords];       // float64 part (large contributions)
    uint32_t hits[kTileWords];
};

// One list entry as loaded: tag (word | row << 8), chord, and whether the
// index lay inside the list.
struct Ent {
    uint32_t m = 0u;
    float a = 0.0f;
    bool ok = false;
};

template <typename CH>
__device__ inline Ent load_ent(const TileBlock &B, int64_t e, int64_t end)
{
    Ent r;
    if (e < end) {
        r.m = B.meta[e - B.base];
        r.a = entry_chord<CH>(B, e - B.base, r.m);
        r.ok = true;
    }
    return r;
}

// Row data an entry of the finished block needs: its row's WEPL, ||a||^2
// and dot product (complete since the previous launch).
struct RowData {
    double wepl = 0.0, n2 = 1.0, dot = 0.0;
};

__device__ inline RowData load_row(const TileBlock &P, const Ent &en)
{
    RowData d;
    const uint32_t q = row_of(P, en.m);
    if (en.ok && q < P.rows) {
        d.wepl = (double)P.wepl[q];
        d.n2 = (double)P.n2[q];
        d.dot = (double)P.dot[q] * kDotUnit;
    }
    return d;
}

// Adds one entry of the finished block to the tile's LDS sums.
__device__ inline void finish_one(const TileBlock &P, const Ent &en, const RowData &d, TileLds &L,
                                  double big, uint32_t *err)
{
    if (!en.ok) return;
    const uint32_t q = row_of(P, en.m);
    if (q >= P.rows) {
        atomicOr(err, 2u);
        return;
    }
    const int w = (int)(en.m & (kTileWords - 1));
    const double r = (d.wepl - d.dot) / d.n2;
    const double v = r * (double)en.a;
    atomicAdd(&L.hits[w], 1u);
    if (fabs(v) <= big)
        atomicAdd(reinterpret_cast<unsigned long long *>(&L.cf[w]),
                  (unsigned long long)__double2ll_rn(v * kCorrScale));
    else
        atomicAdd(&L.cb[w], v);
}

// Finishes block P on this tile (x in LDS and global updated in place).  The
// first round of entries (e0, with its row data d0) was loaded by the caller
// together with the tile; the LDS sums are already cleared.
template <int NT, typename CH>
__device__ void tile_finish(const TileBlock &P, int64_t p0, int64_t p1, const Ent &e0,
                            const RowData &d0, TileLds &L, double *xt, double lambda, double big,
                            uint32_t *err)
{
    finish_one(P, e0, d0, L, big, err);
    for (int64_t e = p0 + NT + threadIdx.x; e < p1; e += NT) {
        const Ent en = load_ent<CH>(P, e, p1);
        finish_one(P, en, load_row(P, en), L, big, err);
    }
    __syncthreads();
    for (int w = threadIdx.x; w < kTileWords; w += NT) {
        const uint32_t h = L.hits[w];
        if (h) {
            const double c = (double)L.cf[w] * kCorrUnit + L.cb[w];
            const double nx = L.x[w] + lambda * c / (double)h;
            L.x[w] = nx;
            xt[w] = nx;
        }
    }
    __syncthreads();
}

// Partial dot products of block C's rows on this tile, from x in LDS; e0 is
// the first round of entries, loaded by the caller.
template <int NT, typename CH>
__device__ void tile_dots(const TileBlock &C, int64_t c0, int64_t c1, const Ent &e0,
                          const TileLds &L, double dot_max, uint32_t *err)
{
    // every thread runs the same number of rounds (the shuffles are uniform)
    uint32_t m = e0.m;
    float a = e0.a;
    bool ok = e0.ok;
    for (int64_t r0 = c0; r0 < c1; r0 += NT) {
        if (r0 != c0) {
            const int64_t e = r0 + threadIdx.x;
            ok = e < c1;
            if (ok) {
                m = C.meta[e - C.base];
                a = entry_chord<CH>(C, e - C.base, m);
            }
        }
        uint32_t q = kNoRow;
        long long f = 0;
        if (ok) {
            q = row_of(C, m);
            const double p = (double)a * L.x[m & (kTileWords - 1)];
            if (q >= C.rows) {
                atomicOr(err, 2u);
                q = kNoRow;
            } else if (fabs(p) <= dot_max) {
                f = __double2ll_rn(p * kDotScale);
            } else {
                atomicOr(err, 1u);
            }
        }
        const dev::Runs runs = dev::wave_runs(q);
        f = dev::run_sum(f, runs);
        if (runs.tail && q != kNoRow)
            atomicAdd(reinterpret_cast<unsigned long long *>(C.dot + q), (unsigned long long)f);
    }
}

__device__ inline void clear_next(const DropTileArgs &A, int nt)
{
    if (!A.zero) return;
    for (int64_t q = (int64_t)blockIdx.x * nt + threadIdx.x; q < A.B; q += (int64_t)gridDim.x * nt)
        A.zero[q] = 0;
}

// List bounds of dispatch slot i (lists are laid out in slot order, so the
// bounds do not wait for the slot's tile to be looked up).
__device__ inline void list_range(const TileBlock &t, int64_t i, int64_t &a, int64_t &b)
{
    a = b = 0;
    if (t.valid) {
        a = t.toff[i];
        b = t.toff[i + 1];
    }
}

// Loads the tile into LDS and clears the finish sums (with fin); the caller
// has issued its other first-round loads before, so they overlap.
template <int NT>
__device__ inline void stage_tile(const double *xt, TileLds &L, bool fin)
{
    double xv[kTileWords / NT];
#pragma unroll
    for (int k = 0; k < kTileWords / NT; k++) xv[k] = xt[threadIdx.x + k * NT];
#pragma unroll
    for (int k = 0; k < kTileWords / NT; k++) {
        const int w = threadIdx.x + k * NT;
        L.x[w] = xv[k];
        if (fin) {
            L.hits[w] = 0u;
            L.cf[w] = 0;
            L.cb[w] = 0.0;
        }
    }
}

// The DROP steps form a chain of short dependent launches, while the rows
// of later blocks are formed beside them on another stream by long float64
// waves.  A step's waves take the highest issue priority on their SIMD so
// that the chain is not held back behind the row formation.
__device__ inline void chain_priority() { __builtin_amdgcn_s_setprio(3); }

// Fused step: finish block P, then the dot products of block C.  The list
// bounds, both lists' first round, the finished rows' data and the tile are
// all requested before the first wait.
template <int NT, typename CH>
__global__ void __launch_bounds__(NT) k_drop_tile(DropTileArgs A)
{
    __shared__ TileLds L;
    chain_priority();
    const int64_t T = A.tiles[blockIdx.x];
    int64_t p0, p1, c0, c1;
    list_range(A.P, blockIdx.x, p0, p1);
    list_range(A.C, blockIdx.x, c0, c1);
    clear_next(A, NT);
    if (p0 == p1 && c0 == c1) return;
    double *xt = A.x + (T << kTileShift);
    const Ent pe = load_ent<CH>(A.P, p0 + threadIdx.x, p1);
    const Ent ce = load_ent<CH>(A.C, c0 + threadIdx.x, c1);
    const RowData pd = load_row(A.P, pe);
    stage_tile<NT>(xt, L, p1 > p0);
    __syncthreads();
    if (p1 > p0) tile_finish<NT, CH>(A.P, p0, p1, pe, pd, L, xt, A.lambda, A.big, A.err);
    if (c1 > c0) tile_dots<NT, CH>(A.C, c0, c1, ce, L, A.dot_max, A.err);
}

// Split form, first launch: finish block P only.
template <int NT, typename CH>
__global__ void __launch_bounds__(NT) k_drop_tile_finish(DropTileArgs A)
{
    __shared__ TileLds L;
    chain_priority();
    const int64_t T = A.tiles[blockIdx.x];
    int64_t p0, p1;
    list_range(A.P, blockIdx.x, p0, p1);
    if (p0 == p1) return;
    double *xt = A.x + (T << kTileShift);
    const Ent pe = load_ent<CH>(A.P, p0 + threadIdx.x, p1);
    const RowData pd = load_row(A.P, pe);
    stage_tile<NT>(xt, L, true);
    __syncthreads();
    tile_finish<NT, CH>(A.P, p0, p1, pe, pd, L, xt, A.lambda, A.big, A.err);
}

// Split form, second launch: dot products of block C only.
template <int NT, typename CH>
__global__ void __launch_bounds__(NT) k_drop_tile_dots(DropTileArgs A)
{
    __shared__ TileLds L;
    chain_priority();
    const int64_t T = A.tiles[blockIdx.x];
    int64_t c0, c1;
    list_range(A.C, blockIdx.x, c0, c1);
    clear_next(A, NT);
    if (c0 == c1) return;
    const double *xt = A.x + (T << kTileShift);
    const Ent ce = load_ent<CH>(A.C, c0 + threadIdx.x, c1);
    stage_tile<NT>(xt, L, false);
    __syncthreads();
    tile_dots<NT, CH>(A.C, c0, c1, ce, L, A.dot_max, A.err);
}

// One lane per tile, walking the blocks (lanes of neighbouring tiles read
// neighbouring counts): the tile's list entries over all blocks, saturated
// at 2^32 - 1.
__global__ void __launch_bounds__(256) k_tile_totals(const uint32_t *cnt, int64_t nblocks,
                                                     int64_t ntiles, uint32_t *total)
{
    const int64_t T = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (T >= ntiles) return;
    uint64_t tot = 0;
    for (int64_t b = 0; b < nblocks; b++) tot += cnt[b * ntiles + T];
    total[T] = tot > 0xffffffffull ? 0xffffffffu : (uint32_t)tot;
}

// The (block, tile) counts gathered into (block, slot) order.
__global__ void __launch_bounds__(256) k_slot_counts(const uint32_t *cnt, const int32_t *act,
                                                     int64_t nact, int64_t nblocks, int64_t ntiles,
                                                     uint32_t *out)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nblocks * nact;
         q += (int64_t)gridDim.x * 256) {
        const int64_t b = q / nact, i = q - b * nact;
        out[q] = cnt[b * ntiles + act[i]];
    }
}

__global__ void __launch_bounds__(256) k_zero_i64(long long *p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * 256)
        p[q] = 0;
}

// Launches one kernel; with a timer pair the launch carries its own start and
// stop events, which take the dispatch's timestamps (no gap around it).
template <typename F, typename... Args>
void launch(F kernel, dim3 grid, dim3 block, hipStream_t stream, hipEvent_t t0, hipEvent_t t1,
            Args... args)
{
    hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, t0, t1, 0u, args...);
}

template <int NT, typename CH>
hipError_t drop_tiles(const DropTileArgs &a, int64_t ntiles, int split, hipStream_t stream,
                      const KTimer &t)
{
    const dim3 grid((unsigned)a.nact), block(NT);
    if (!split) {
        launch(k_drop_tile<NT, CH>, grid, block, stream, t.e[0], t.e[1], a);
        return hipGetLastError();
    }
    if (a.P.valid) launch(k_drop_tile_finish<NT, CH>, grid, block, stream, t.e[0], t.e[1], a);
    launch(k_drop_tile_dots<NT, CH>, grid, block, stream, t.e[2], t.e[3], a);
    return hipGetLastError();
}

template <typename CH>
hipError_t drop_tiles_nt(const DropTileArgs &a, int64_t ntiles, int threads, int split,
                         hipStream_t stream, const KTimer &t)
{
    switch (threads) {
    case 64: return drop_tiles<64, CH>(a, ntiles, split, stream, t);
    case 128: return drop_tiles<128, CH>(a, ntiles, split, stream, t);
    default: return drop_tiles<256, CH>(a, ntiles, split, stream, t);
    }
}

}  // namespace

hipError_t launch_drop_tiles(const DropTileArgs &a, int64_t ntiles, int threads, int split,
                             hipStream_t stream, const KTimer *kt)
{
    if (ntiles <= 0 || (!a.P.valid && !a.C.valid) || !a.tiles || a.nact <= 0) return hipSuccess;
    const KTimer none{};
    const KTimer &t = kt ? *kt : none;
    const TileBlock &v = a.P.valid ? a.P : a.C;
    if (v.chq) return drop_tiles_nt<uint16_t>(a, ntiles, threads, split, stream, t);
    if (v.ch16) return drop_tiles_nt<__half>(a, ntiles, threads, split, stream, t);
    return drop_tiles_nt<float>(a, ntiles, threads, split, stream, t);
}

hipError_t launch_tile_totals(const uint32_t *cnt, int64_t nblocks, int64_t ntiles,
                              uint32_t *total, hipStream_t stream)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_totals, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, stream,
                       cnt, nblocks, ntiles, total);
    return hipGetLastError();
}

hipError_t launch_slot_counts(const uint32_t *cnt, const int32_t *act, int64_t nact,
                              int64_t nblocks, int64_t ntiles, uint32_t *out, hipStream_t stream)
{
    const int64_t n = nblocks * nact;
    if (n <= 0) return hipSuccess;
    const int64_t wgs = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_slot_counts, dim3((unsigned)wgs), dim3(256), 0, stream, cnt, act, nact,
                       nblocks, ntiles, out);
    return hipGetLastError();
}

hipError_t launch_zero_i64(long long *p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    int64_t wgs = (n + 255) / 256;
    if (wgs > 1024) wgs = 1024;
    hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)wgs), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace tvs
