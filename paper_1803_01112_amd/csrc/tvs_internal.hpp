// tvs_internal.hpp -- internal declarations of the MI355X TVS library: the
// device-side parameter blocks and the kernel launchers.  Nothing here is
// part of the public ABI (include/tvs.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tvs.h"

namespace tvs {

// Voxel grid as the kernels see it.  Every device image (and every voxel
// index a row holds) uses the tiled layout below; images cross the ABI in
// plain x-fastest order and are converted on the way in and out.
struct GridDev {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double ox, oy, oz;
    int32_t ntx, nty;         // tiles per slice along x and y
    double rvx, rvy, rvz;     // 1/vx, 1/vy, 1/vz rounded to nearest
};

// Tiled layout.  Each slice is cut into 16 x 16 voxel tiles of 256
// consecutive float64 words (tiles x-fastest, then y, slices outermost);
// inside a tile, 4 x 2 (x, y) bricks of 8 words (one 64-byte line), bricks
// x-fastest.  A DROP block is processed tile by tile: one workgroup holds a
// tile's 256 voxels in LDS, so the block's corrections never leave the CU.
// Voxels past nx / ny in the last tile column / row are padding: never
// indexed by a row, zero in every image and subgradient.
constexpr int kTileShift = 8, kTileWords = 1 << kTileShift, kTileSide = 16;

__host__ __device__ inline int64_t vaddr(const GridDev &g, int64_t i, int64_t j, int64_t k)
{
    const int64_t tile = (k * g.nty + (j >> 4)) * g.ntx + (i >> 4);
    const int64_t in = ((((j & 15) >> 1) << 2 | ((i & 15) >> 2)) << 3) | ((j & 1) << 2) | (i & 3);
    return (tile << kTileShift) | in;
}

// vaddr in 32-bit arithmetic, for images of fewer than 2^31 words (every
// image a context accepts).
__host__ __device__ inline int32_t vaddr32(const GridDev &g, int32_t i, int32_t j, int32_t k)
{
    const int32_t tile = (k * g.nty + (j >> 4)) * g.ntx + (i >> 4);
    const int32_t in = ((((j & 15) >> 1) << 2 | ((i & 15) >> 2)) << 3) | ((j & 1) << 2) | (i & 3);
    return (tile << kTileShift) | in;
}

// Inverse of vaddr: voxel coordinates of tiled-layout word a.
__host__ __device__ inline void vcoord(const GridDev &g, int64_t a, int64_t &i, int64_t &j,
                                       int64_t &k)
{
    const int64_t tile = a >> kTileShift, in = a & (kTileWords - 1);
    const int64_t brick = in >> 3, w = in & 7;
    const int64_t t2 = tile / g.ntx;
    const int64_t tx = tile - t2 * g.ntx;
    k = t2 / g.nty;
    const int64_t ty = t2 - k * g.nty;
    i = tx * kTileSide + (brick & 3) * 4 + (w & 3);
    j = ty * kTileSide + (brick >> 2) * 2 + (w >> 2);
}

__host__ __device__ inline int64_t num_tiles(const GridDev &g)
{
    return (int64_t)g.ntx * g.nty * g.nz;
}

// Words of a device image (padding included).
__host__ __device__ inline int64_t padded_voxels(const GridDev &g)
{
    return num_tiles(g) << kTileShift;
}

inline GridDev make_grid_dev(const tvs_grid &g)
{
    return GridDev{g.nx, g.ny, g.nz, g.vx, g.vy, g.vz, g.ox, g.oy, g.oz,
                   (g.nx + kTileSide - 1) / kTileSide, (g.ny + kTileSide - 1) / kTileSide,
                   1.0 / g.vx, 1.0 / g.vy, 1.0 / g.vz};
}

// SoA history streams on the device: 13 float32 arrays of length n, one
// after the other from base, in the order of HistStream.  Two words of
// kernel arguments instead of thirteen pointers.
enum HistStream { kEx = 0, kEy, kEz, kQx, kQy, kQz, kEth, kEps, kQth, kQps, kUx, kUy, kWepl };
struct HistDev {
    const float *base;
    int64_t n;
    __host__ __device__ const float *s(int k) const { return base + (int64_t)k * n; }
};

struct MlpCfg {
    double step;
    int32_t log_term;
    int32_t const_power;
    const double *s1i = nullptr;   // entry-side table: (Sigma_1(j * step))^-1 as {a, b, d}
    int64_t nj = 0;                // depths j < nj in the table
    uint32_t *err = nullptr;       // raised by a depth past the table
};

// Row-major rows of histories [first, first + n) (debug copies of rows):
// CSR with offsets relative to the start of this row set.
struct RowSet {
    int64_t first = 0;        // global index of the first history
    int64_t n = 0;            // histories in the set
    int64_t base = 0;         // entries of row q start at row_off[q] - base
    int64_t *row_off = nullptr;   // n + 1 offsets
    int32_t *idx = nullptr;       // voxel indices (x-fastest order after the copy-out)
    float *chord32 = nullptr;     // chords (float32)
    float *norm2 = nullptr;       // ||a_i||^2 per history (0: the history forms no row)
};

// Tile lists.  The entries of DROP block b (rows bB .. bB+B-1) are kept
// grouped by image tile: list (b, T) holds, for every row of the block that
// crosses tile T, its entries inside T, each as
//   meta  = (word within the tile) | (row within the block) << 8,
//   chord = float32, float16, or fixed point: an unsigned code times a unit
//           (the longest chord of the loaded rows / the largest code,
//           rounded up), its low 16 bits in a 16-bit word and its high bits
//           in the tag bits above the row field, which a block of B rows
//           leaves free (24 - ceil(log2 B) of them: 12 at B = 3200).
// A row's entries inside one tile form a segment (a run of consecutive
// entries of its walk); the place of every segment in its list is fixed
// once, when the histories are loaded, so rows formed again on every sweep
// land where the sweep expects them.
struct TileFill {
    int64_t first = 0, n = 0;       // histories [first, first + n)
    int64_t B = 1;                  // block size
    const int64_t *seg_off = nullptr;   // per history: first segment (global)
    const int64_t *segdst = nullptr;    // per segment: global entry index of its first entry
    int64_t base = 0;               // global entry index of meta[0] / chord[0]
    uint32_t *meta = nullptr;
    float *ch32 = nullptr;
    __half *ch16 = nullptr;
    uint16_t *chq = nullptr;        // fixed-point store: low 16 bits of each chord's code
    double qinv = 0.0;              // fixed-point store: code = rint(length * qinv)
    uint32_t qmax = 0;              // fixed-point store: largest code
    uint32_t qshift = 31;           // fixed-point store: tag bit of the code's bit 16
    int64_t cap = 0;                // entries meta / chord can hold
    float *norm2 = nullptr;         // per history (global index)
    uint32_t *err = nullptr;        // raised if a walk disagrees with the load-time lists
    int64_t max_wgs = 0;            // > 0: at most this many workgroups (grid-stride)
    const int32_t *order = nullptr; // non-null: lane q forms history order[first + q] (the
                                    // histories of a chunk by decreasing row length)
    int32_t room = 0;               // 1 (float chords only): the kernel held at two waves per
                                    // SIMD, leaving room for DROP waves beside it
};

// ----------------------------------------------------------------- rows.hip
// Load-time passes over every history (all asynchronous on `stream`):
//   count : nnz[i] entries and nseg[i] segments of row i;
//   seg   : reserves each segment's place in its (block, tile) list with an
//           atomic on btc[b * ntiles + T] and records (T, place) in segtab;
//   dest  : turns (T, place) into the segment's global entry index, given
//           the exclusive scan bt_off of btc.
// A walk that disagrees with the count pass writes nothing and raises *err.
hipError_t launch_rows_count(const GridDev &g, const HistDev &h, const MlpCfg &m, int64_t first,
                             int64_t n, int32_t *nnz, int32_t *nseg, hipStream_t stream);
// seg also raises *chmax to the float32 bits of the longest chord (rounded
// up to float32).
hipError_t launch_rows_seg(const GridDev &g, const HistDev &h, const MlpCfg &m, int64_t n,
                           int64_t B, const int64_t *seg_off, uint32_t *btc, uint64_t *segtab,
                           uint32_t *err, uint32_t *chmax, const int32_t *order,
                           hipStream_t stream);
// bt_off: the list starts of every (block, slot), slot_of: tile -> slot.
hipError_t launch_seg_dest(const GridDev &g, int64_t n, int64_t B, const int64_t *seg_off,
                           const int64_t *bt_off, const int32_t *slot_of, int64_t nslots,
                           uint64_t *segtab, uint32_t *err, hipStream_t stream);
// Forms the rows of f.first .. f.first + f.n - 1 into their tile lists.
hipError_t launch_rows_fill_tiled(const GridDev &g, const HistDev &h, const MlpCfg &m,
                                  const TileFill &f, hipStream_t stream);
// Forms rows in row-major order (for tvs_debug_rows).
hipError_t launch_rows_fill(const GridDev &g, const HistDev &h, const MlpCfg &m, const RowSet &rs,
                            hipStream_t stream);
// Exclusive scan of n int32 (or uint32) counts into n+1 int64 offsets
// (off[n] = total).  `tmp` needs scan_tmp_elems(n) int64 elements.
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_scan(const int32_t *cnt, int64_t n, int64_t *off, int64_t *tmp,
                       hipStream_t stream);
// Counts histories with non-finite values, a degenerate beam axis,
// coordinates beyond 1e6 mm or more than 2^20 MLP vertices into *bad, and
// raises *jmax to at least every valid history's vertex count + 2.
hipError_t launch_validate(const HistDev &h, int64_t n, double step, uint32_t *bad,
                           uint32_t *jmax, hipStream_t stream);
// Hull detection (straight entry-exit lines): in_cnt / out_cnt (tiled
// layout, cleared by the caller) count the lines of WEPL >= wepl_in /
// < wepl_out through every voxel, each up to in_sat / out_sat (past which no
// decision changes); decide writes hull (x-fastest uint8) and, with mask,
// zeroes the image outside the hull.
hipError_t launch_hull_counts(const GridDev &g, const HistDev &h, int64_t n, double wepl_in,
                              double wepl_out, uint32_t *in_cnt, uint32_t *out_cnt,
                              uint32_t in_sat, uint32_t out_sat, hipStream_t stream);
hipError_t launch_hull_decide(const GridDev &g, const uint32_t *in_cnt, const uint32_t *out_cnt,
                              uint32_t min_in, uint32_t max_out, uint8_t *hull, double *mask,
                              hipStream_t stream);
// dst[b] = src[b * stride] for b < n.
// Initial iterate (fbp.hip): binning, Ram-Lak filter, backprojection,
// in-slice median (radius 0..2; 0 only narrows the image to float32).
hipError_t launch_fbp_bin(const GridDev &g, const HistDev &h, int64_t n, int32_t A, double tau,
                          int32_t nt, unsigned long long *sum, uint32_t *cnt, hipStream_t stream);
hipError_t launch_fbp_mean(const unsigned long long *sum, const uint32_t *cnt, int64_t nb, double *p,
                           hipStream_t stream);
hipError_t launch_fbp_filter(const double *p, int64_t rows, int32_t nt, double tau, double *q,
                             hipStream_t stream);
hipError_t launch_fbp_backproject(const GridDev &g, const double *q, const double *cs, int32_t A,
                                  double tau, int32_t nt, int clip, double *x, hipStream_t stream);
hipError_t launch_median(const GridDev &g, const double *x, int radius, float *out,
                         hipStream_t stream);
// cos and sin of the A beam angles a * 2 pi / A into cs (2 A doubles).
hipError_t launch_fbp_angles(int32_t A, double *cs, hipStream_t stream);
hipError_t launch_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst,
                       hipStream_t stream);
// Fills the entry-side table of m for depths j = 0 .. nj - 1 (3 doubles each).
hipError_t launch_mlp_table(const MlpCfg &m, int64_t nj, double *tab, hipStream_t stream);

// ----------------------------------------------------------------- drop.hip
// One DROP block's tile lists as a kernel sees them.
struct TileBlock {
    const uint32_t *meta = nullptr;   // entry e (global index) at meta[e - base]
    const float *ch32 = nullptr;
    const __half *ch16 = nullptr;
    const uint16_t *chq = nullptr;    // fixed-point store: low 16 bits of each chord's code
    double qunit = 0.0;               // fixed-point store: mm per unit of the code
    uint32_t qshift = 31;             // fixed-point store: the code's bits 16.. sit in tag bits qshift..
    uint32_t rowmask = 0xffffffu;     // row field of a tag: (tag >> 8) & rowmask
    const int64_t *toff = nullptr;    // nact + 1 list starts in slot order (global entry index)
    int64_t base = 0;
    const float *wepl = nullptr;      // per row of the block
    const float *n2 = nullptr;        // ||a_i||^2 per row of the block
    long long *dot = nullptr;         // fixed-point row dot products (x S for batches)
    uint32_t rows = 0;                // rows of the block; an entry naming another raises err
    int valid = 0;
};

// Fixed-point units: row dot products are summed as integers in units of
// 2^-36 (exact and order-free), block corrections in units of 2^-40.
constexpr double kDotScale = 68719476736.0;          // 2^36
constexpr double kCorrScale = 1099511627776.0;       // 2^40

struct DropTileArgs {
    TileBlock P;            // block b - 1: its update is finished on every tile
    TileBlock C;            // block b: partial dot products of its rows per tile
    double *x = nullptr;    // image (tiled layout, float64)
    double lambda = 0.0;
    double big = 0.0;       // |r a| above this is summed in float64 (keeps the fixed sum in range)
    double dot_max = 0.0;   // |a x| above this cannot be summed in fixed point: error flag
    long long *zero = nullptr;  // dot accumulators to clear for block b + 1
    int64_t B = 0;
    uint32_t *err = nullptr;
    // tiles that some block's lists cross (the others have no work in any
    // step), the busiest first; non-null: workgroup i takes tile tiles[i],
    // nact workgroups
    const int32_t *tiles = nullptr;
    int64_t nact = 0;
};

// Start/stop events of the kernels of one block (first and second launch);
// null events are not recorded.
struct KTimer {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
};

// One step of the tile-wise DROP chain: finish block b - 1 and form the dot
// products of block b (either may be absent) on every tile.  threads: 64,
// 128 or 256 per tile workgroup; split: 0 one fused launch, 1 two launches.
hipError_t launch_drop_tiles(const DropTileArgs &a, int64_t ntiles, int threads, int split,
                             hipStream_t stream, const KTimer *kt = nullptr);
hipError_t launch_zero_i64(long long *p, int64_t n, hipStream_t stream);
// total[T] = entries of tile T over the lists of every block (list starts
// bt_off of nblocks x ntiles lists), saturated at 2^32 - 1.
hipError_t launch_slot_counts(const uint32_t *cnt, const int32_t *act, int64_t nact,
                              int64_t nblocks, int64_t ntiles, uint32_t *out, hipStream_t stream);
hipError_t launch_tile_totals(const uint32_t *cnt, int64_t nblocks, int64_t ntiles,
                              uint32_t *total, hipStream_t stream);

// ----------------------------------------------------------------- tv.hip
struct TvBuffers {
    double *g;           // subgradient
    double *part;        // per-workgroup partial sums
    uint32_t *ticket;    // last-workgroup counter
    double *scal;        // [0] = ||g||^2, [1] = phi value
    int64_t nparts;
};
int64_t tv_num_parts(const GridDev &g);
// Schedule of checked cycles, held on the device while a checked
// tvs_iterate call runs (ell and the SplitMix64 state).
struct SchedDev {
    int64_t ell;
    uint64_t rng;
};
// Scratch of the device-side TV check: partial sums of TV(x) and of the
// trial images per tile workgroup (tv_check_parts doubles), a last-workgroup
// ticket, and the decision {scale, accepted}.
struct CheckBuffers {
    double *part;
    uint32_t *ticket;
    double *dec;
};
int64_t tv_check_parts(const GridDev &g);
// One checked step: decides on the device (first try t with
// TV(x + s_t g) <= TV(x), s_t = -alpha^(ell + t) / sqrt(scal[0]), at most
// max_tries tries), advances sd->ell by the tries and writes *rec.
hipError_t launch_tv_check(const GridDev &g, const double *x, double eps, double alpha,
                           int32_t max_tries, int32_t k, int32_t n, SchedDev *sd,
                           tvs_step_log *rec, const CheckBuffers &c, const TvBuffers &t,
                           hipStream_t stream);
// x += s g with the decided scale (nothing when the step gave up).
hipError_t launch_tv_apply(const GridDev &g, double *x, const TvBuffers &t, const CheckBuffers &c,
                           hipStream_t stream);
// ell = rand(k, ell) with the device SplitMix64 state; sets the state.
hipError_t launch_sched_draw(SchedDev *sd, int64_t k, hipStream_t stream);
hipError_t launch_sched_set(SchedDev *sd, int64_t ell, uint64_t rng, hipStream_t stream);
// g = grad TV(x); scal[0] = ||g||^2 (fixed-order reduction).
hipError_t launch_tv_grad(const GridDev &g, const double *x, double eps, const TvBuffers &t,
                          hipStream_t stream);
// x = x + s * g with s = -beta / sqrt(scal[0]) (0 when the norm is 0).
hipError_t launch_tv_step(const GridDev &g, double *x, double beta, const TvBuffers &t,
                          hipStream_t stream);
// Image conversion between the ABI's x-fastest float32 and the device's
// float64 tiled layout (the padding of dst is left untouched by widen).
hipError_t launch_widen(const GridDev &g, const float *src, double *dst, hipStream_t stream);
hipError_t launch_narrow(const GridDev &g, const double *src, float *dst, hipStream_t stream);

// ----------------------------------------------------------------- batch.hip
// S images interleaved by voxel (x[p*S + s]).
struct BatchBuffers {
    int S = 0;
    int64_t nvox = 0;
    double *x = nullptr;        // nvox * S
    double *g = nullptr;        // nvox * S
    double *part = nullptr;     // batch_num_parts * S
    uint32_t *ticket = nullptr;
    double *norm2 = nullptr;    // S
    double *lambda = nullptr;   // S
    double *eps = nullptr;      // S
    double *beta_tab = nullptr; // cycles * nmax * S
    int32_t *cyc = nullptr;     // device cycle counter
};
int batch_vox_per_wg(int S);
int64_t batch_num_parts(const GridDev &g, int S);
hipError_t launch_tvb_grad(const GridDev &g, const BatchBuffers &b, uint32_t active,
                           hipStream_t stream);
hipError_t launch_tvb_step(const BatchBuffers &b, uint32_t active, int n, int nmax,
                           hipStream_t stream);
hipError_t launch_set_counter(int32_t *cyc, int32_t v, hipStream_t stream);
hipError_t launch_tick(int32_t *cyc, hipStream_t stream);
hipError_t launch_replicate(const double *x0, const BatchBuffers &b, hipStream_t stream);
hipError_t launch_extract(const GridDev &g, const BatchBuffers &b, int s, float *out,
                          hipStream_t stream);
// The tile-wise DROP step for S settings at once (dot arrays hold B x S
// values, row-major by row; a.lambda is unused, the per-setting relaxations
// come from b.lambda).
hipError_t launch_drop_tiles_batch(const DropTileArgs &a, const BatchBuffers &b, int64_t ntiles,
                                   int threads, int group, hipStream_t stream);
// threads (128, 256) and settings per LDS pass (4, 8, 16) the batched step
// is built for.
bool batch_shape_ok(int threads, int group);

}  // namespace tvs
