// tvs_internal.hpp -- internal declarations of the MI355X TVS library: the
// context, device-side parameter blocks and the kernel launchers.  Nothing
// here is part of the public ABI (include/tvs.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tvs.h"

namespace tvs {

// Voxel grid as the kernels see it.  Every device image (and every voxel
// index a row holds) uses the brick layout below; images cross the ABI in
// plain x-fastest order and are converted on the way in and out.
struct GridDev {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double ox, oy, oz;
    int32_t nbx, nby;         // bricks per slice along x and y
};

// Brick layout: each slice is tiled by 4 x 2 (x, y) bricks of 8 float64
// words, one 64-byte line, bricks x-fastest, slices outermost.  A proton
// path crosses a brick in a few consecutive entries, so the entries a
// wavefront gathers or scatters at once touch about a third fewer lines
// than in x-fastest order (atomics are priced per line).  Voxels past nx / ny
// in the last brick column / row are padding: never indexed by a row, zero
// in every image and subgradient.
constexpr int kBrickX = 4, kBrickY = 2, kBrick = kBrickX * kBrickY;

__host__ __device__ inline int64_t vaddr(const GridDev &g, int64_t i, int64_t j, int64_t k)
{
    return (((k * g.nby + (j >> 1)) * g.nbx + (i >> 2)) << 3) + ((j & 1) << 2) + (i & 3);
}

// Inverse of vaddr: voxel coordinates of brick-layout word a.
__host__ __device__ inline void vcoord(const GridDev &g, int64_t a, int64_t &i, int64_t &j,
                                       int64_t &k)
{
    const int64_t b = a >> 3, w = a & 7;
    const int64_t t = b / g.nbx;
    i = (b - t * g.nbx) * kBrickX + (w & 3);
    k = t / g.nby;
    j = (t - k * g.nby) * kBrickY + (w >> 2);
}

// Words of a device image (padding included).
__host__ __device__ inline int64_t padded_voxels(const GridDev &g)
{
    return (int64_t)g.nbx * g.nby * kBrick * g.nz;
}

inline GridDev make_grid_dev(const tvs_grid &g)
{
    return GridDev{g.nx, g.ny, g.nz, g.vx, g.vy, g.vz, g.ox, g.oy, g.oz,
                   (g.nx + kBrickX - 1) / kBrickX, (g.ny + kBrickY - 1) / kBrickY};
}

// SoA history streams on the device (13 float32 arrays of length n_hist).
struct HistDev {
    const float *ex, *ey, *ez, *qx, *qy, *qz, *eth, *eps, *qth, *qps, *ux, *uy, *wepl;
};

struct MlpCfg {
    double step;
    int32_t log_term;
    int32_t const_power;
};

// Rows of a contiguous range of histories [first, first + n): CSR with
// offsets relative to the start of this row set.
struct RowSet {
    int64_t first = 0;        // global index of the first history
    int64_t n = 0;            // histories in the set
    int64_t nnz = 0;          // entries
    int64_t base = 0;         // entries of row q start at row_off[q] - base
    int64_t *row_off = nullptr;   // n + 1 offsets
    int32_t *idx = nullptr;       // voxel indices
    float *chord32 = nullptr;     // chords (float32) or
    __half *chord16 = nullptr;    // chords (float16)
    float *norm2 = nullptr;       // ||a_i||^2 per history (0: the history forms no row)
};

// ----------------------------------------------------------------- rows.hip
// Forms the rows of histories [first, first + n) in two passes.  Pass 1
// writes nnz[i] (int32); after an exclusive scan into row_off, pass 2 fills
// idx / chord / norm2.  All launches are asynchronous on `stream`.
hipError_t launch_rows_count(const GridDev &g, const HistDev &h, const MlpCfg &m, int64_t first,
                             int64_t n, int32_t *nnz, hipStream_t stream);
hipError_t launch_rows_fill(const GridDev &g, const HistDev &h, const MlpCfg &m, const RowSet &rs,
                            hipStream_t stream);
// Exclusive scan of n int32 counts into n+1 int64 offsets (off[n] = total).
// `tmp` needs scan_tmp_elems(n) int64 elements.
int64_t scan_tmp_elems(int64_t n);
// Counts histories with non-finite values, a degenerate beam axis,
// coordinates beyond 1e6 mm or more than 2^20 MLP vertices into *bad.
hipError_t launch_validate(const HistDev &h, int64_t n, double step, uint32_t *bad,
                           hipStream_t stream);
hipError_t launch_scan(const int32_t *cnt, int64_t n, int64_t *off, int64_t *tmp,
                       hipStream_t stream);

// ----------------------------------------------------------------- drop.hip
struct DropBuffers {
    double *x;           // image (float64: keeps the small DROP increments exact
                         // enough for the scale-free TV subgradient)
    double *c;           // correction sums (float64, like the image)
    uint32_t *s;         // hit counts
    int32_t *touched;    // voxels touched by the current block (capacity nvox)
    uint32_t *ntouched;  // two counters used alternately by consecutive blocks
    uint32_t *barrier;   // persistent sweep: grid barrier counter + error flag
    int64_t nvox;
    double *c64 = nullptr;   // non-null: packed per-block scatter (c holds the packed words,
                             // c64 the float64 part of large contributions)
    uint32_t *omask = nullptr;  // one bit per voxel: the float64 part is non-zero
    double big = 0.0;        // largest contribution taken in fixed point
};

// Start/stop events of the two kernels of one block (the rows kernel, then
// the apply kernel); null events are not recorded.
struct KTimer {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
};

// One DROP block [r0, r1) (global history indices inside rs) with the
// one-launch-per-phase kernels; `parity` selects the touched counter.
// `kt` (may be null) times the block's two kernels.
hipError_t launch_drop_block(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                             double lambda, const DropBuffers &b, int parity, int lanes_per_row,
                             hipStream_t stream, const KTimer *kt = nullptr);
// All blocks of rs in one persistent launch with grid barriers.
hipError_t launch_drop_persistent(const RowSet &rs, const float *wepl, int64_t block_size,
                                  double lambda, const DropBuffers &b, int lanes_per_row,
                                  int grid_wgs, hipStream_t stream);
int persistent_grid_size(int device, int lanes_per_row);
// Clears both touched-list counters.
hipError_t launch_zero_counters(uint32_t *cnt, hipStream_t stream);

// Voxel-major form of one DROP block (csc.hip): distinct voxels uvox[0..U),
// their column starts ucol (relative to the block's first entry), and the
// block's ne column entries (row within the block, chord).
struct CscBlock {
    const int32_t *uvox = nullptr;
    const uint32_t *ucol = nullptr;
    int64_t U = 0, ne = 0;
    const uint16_t *cq = nullptr;
    const float *cch32 = nullptr;
    const __half *cch16 = nullptr;
};
// Residual launch + voxel-major apply launch of one block (no atomics).
hipError_t launch_drop_block_csc(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                                 double lambda, const CscBlock &cb, double *x, double *rbuf,
                                 int lanes_per_row, hipStream_t stream, const KTimer *kt = nullptr);
// Build steps of the voxel-major form for a batch of nb blocks from b0.
hipError_t csc_count(const RowSet &rs, int64_t r0, int64_t r1, int64_t block_size, int64_t b0,
                     int64_t nvox, uint32_t *cnt, hipStream_t st);
hipError_t csc_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst, hipStream_t st);
hipError_t csc_flags(const uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t st);
hipError_t csc_as_int(const uint32_t *cnt, int64_t n, int32_t *out, hipStream_t st);
hipError_t csc_emit(uint32_t *cnt, const int64_t *urank, const int64_t *cstart, int64_t nb,
                    int64_t nvox, const int64_t *ubase, const int64_t *ebase, int32_t *uvox,
                    uint32_t *ucol, hipStream_t st);
hipError_t csc_place(const RowSet &rs, int64_t r0, int64_t r1, int64_t block_size, int64_t b0,
                     int64_t nvox, uint32_t *cursor, const int64_t *ebase, uint16_t *cq,
                     float *cch32, __half *cch16, hipStream_t st);
hipError_t csc_sort(const uint32_t *ucol, const int64_t *ubase, const int64_t *ucount,
                    const int64_t *ebase, const int64_t *ecount, int64_t nb, int64_t max_u,
                    uint16_t *cq, float *cch32, __half *cch16, hipStream_t st);

// ----------------------------------------------------------------- tv.hip
struct TvBuffers {
    double *g;           // subgradient
    double *part;        // per-workgroup partial sums
    uint32_t *ticket;    // last-workgroup counter
    double *scal;        // [0] = ||g||^2, [1] = phi value
    int64_t nparts;
};
int64_t tv_num_parts(const GridDev &g);
// g = grad TV(x); scal[0] = ||g||^2 (fixed-order reduction).
hipError_t launch_tv_grad(const GridDev &g, const double *x, double eps, const TvBuffers &t,
                          hipStream_t stream);
// x = x + s * g with s = -beta / sqrt(scal[0]) (0 when the norm is 0).
hipError_t launch_tv_step(const GridDev &g, double *x, double beta, const TvBuffers &t,
                          hipStream_t stream);
// scal[1] = TV(x + s g) with s = -beta / sqrt(scal[0]) rounded as in
// launch_tv_step, so an accepted trial image equals the stepped image
// (beta = 0: TV(x)).
hipError_t launch_tv_phi(const GridDev &g, const double *x, double beta, double eps,
                         const TvBuffers &t, hipStream_t stream);
// Image conversions between the float32 ABI and the float64 device image.
// Image conversion between the ABI's x-fastest float32 and the device's
// float64 brick layout (the padding of dst is left untouched by widen).
hipError_t launch_widen(const GridDev &g, const float *src, double *dst, hipStream_t stream);
hipError_t launch_narrow(const GridDev &g, const double *src, float *dst, hipStream_t stream);
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream);

// ----------------------------------------------------------------- batch.hip
// S images interleaved by voxel (x[p*S + s]); hit counts and the touched list
// are shared by all settings.
struct BatchBuffers {
    int S = 0;
    int64_t nvox = 0;
    double *x = nullptr;        // nvox * S
    double *g = nullptr;        // nvox * S
    double *c = nullptr;        // nvox * S
    uint32_t *s = nullptr;      // nvox (shared)
    int32_t *touched = nullptr; // nvox (shared)
    uint32_t *ntouched = nullptr, *barrier = nullptr;
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
int batch_grid_size(int device, int S);
hipError_t launch_tvb_grad(const GridDev &g, const BatchBuffers &b, uint32_t active,
                           hipStream_t stream);
hipError_t launch_tvb_step(const BatchBuffers &b, uint32_t active, int n, int nmax,
                           hipStream_t stream);
hipError_t launch_set_counter(int32_t *cyc, int32_t v, hipStream_t stream);
hipError_t launch_tick(int32_t *cyc, hipStream_t stream);
hipError_t launch_replicate(const double *x0, const BatchBuffers &b, hipStream_t stream);
hipError_t launch_extract(const GridDev &g, const BatchBuffers &b, int s, float *out,
                          hipStream_t stream);
hipError_t launch_drop_batch(const RowSet &rs, const float *wepl, int64_t block_size,
                             const BatchBuffers &b, int grid_wgs, hipStream_t stream);
// Voxel-major block of a batch: S residuals per row into rbuf (B*S), then S
// corrections per distinct voxel.
hipError_t launch_batch_block_csc(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                                  const CscBlock &cb, const BatchBuffers &b, double *rbuf,
                                  hipStream_t stream);

}  // namespace tvs
