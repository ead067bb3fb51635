// drop.hip -- the feasibility-seeking sweep P_T on gfx950: block-iterative
// DROP (diagonally relaxed orthogonal projections) over blocks of B
// consecutive histories (arXiv 1803.01112, Section III-D; P_T in Appendix A).
//
// For block t, from one image x:
//   r_i = (b_i - a_i . x) / ||a_i||^2          every row i of the block
//   c_j = sum_i r_i a_ij,  s_j = #entries at j  (scatter)
//   x_j += lambda c_j / s_j                     where s_j > 0 (apply)
// Blocks are applied one after another.
//
// Rows are read from a CSR row set (int32 voxel index + float32 or float16
// chord).  A group of LPR lanes (a wavefront for LPR = 64) reads one row
// coalesced, gathers x (float64), reduces the dot product in float64 with
// cross-lane shuffles,
// and scatters r a_ij / 1 with hardware float64 / integer atomics.  The first
// hit of a voxel in a block appends it to a touched list (one atomic per
// wavefront), so the apply phase visits only touched voxels and clears them.
//
// Two forms: one launch per phase (rows, apply), or one persistent launch
// per sweep with a device-wide barrier between phases.  The barrier spins a
// bounded number of times; on timeout it raises an error flag that makes
// every workgroup leave, and the host reports a device error.
#include <hip/hip_ext.h>

#include "device_common.hpp"
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int kThreads = 256;
using dev::append_touched;
using dev::chord_at;
using dev::grid_barrier;
using dev::group_sum;

// One row: dot, residual, scatter.  All LPR lanes of the group call it.
template <int LPR, typename CH>
__device__ inline void drop_row(const RowSet &rs, const CH *chord, const float *wepl, int64_t row,
                                const double *x, double *c, uint32_t *s, int32_t *touched,
                                uint32_t *cnt)
{
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    double acc = 0.0;
    if (n2 > 0.0f)
        for (int64_t e = off + lane; e < end; e += LPR)
            acc += (double)chord_at(chord, e) * x[rs.idx[e]];
    acc = group_sum<LPR>(acc);
    const double r = (n2 > 0.0f) ? ((double)wepl[row] - acc) / (double)n2 : 0.0;
    const int64_t trips = (n2 > 0.0f) ? (end - off + LPR - 1) / LPR : 0;
    // Uniform trip count inside the group so the wavefront-wide ballot sees
    // every lane of the group.
    for (int64_t q = 0; q < trips; q++) {
        int64_t e = off + q * LPR + lane;
        bool first = false;
        int32_t j = 0;
        if (e < end) {
            j = rs.idx[e];
            unsafeAtomicAdd(c + j, r * (double)chord_at(chord, e));
            first = (atomicAdd(s + j, 1u) == 0u);
        }
        append_touched(first, j, touched, cnt);
    }
}

__device__ inline void apply_voxel(int32_t j, double lambda, double *x, double *c, uint32_t *s)
{
    double cj = c[j];
    uint32_t sj = s[j];
    x[j] += lambda * cj / (double)sj;
    c[j] = 0.0;
    s[j] = 0u;
}

__global__ void k_zero_counters(uint32_t *cnt)
{
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0u;
}

template <int LPR, typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_persistent(RowSet rs, const CH *chord, const float *wepl, int64_t block_size, double lambda,
                  double *x, double *c, uint32_t *s, int32_t *touched, uint32_t *cnt, uint32_t *bar)
{
    const int64_t groups = (int64_t)gridDim.x * (kThreads / LPR);
    const int64_t gid = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / LPR;
    const int64_t gthreads = (int64_t)gridDim.x * kThreads;
    const int64_t gtid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nblocks = (rs.n + block_size - 1) / block_size;
    for (int64_t t = 0; t < nblocks; t++) {
        const int64_t r0 = rs.first + t * block_size;
        const int64_t r1 = (r0 + block_size < rs.first + rs.n) ? r0 + block_size : rs.first + rs.n;
        uint32_t *cur = cnt + (t & 1);
        for (int64_t row = r0 + gid; row < r1; row += groups)
            drop_row<LPR, CH>(rs, chord, wepl, row, x, c, s, touched, cur);
        if (!grid_barrier(bar)) return;
        const uint32_t n = *cur;
        for (int64_t i = gtid; i < (int64_t)n; i += gthreads) apply_voxel(touched[i], lambda, x, c, s);
        if (gtid == 0) cnt[(t + 1) & 1] = 0u;
        if (!grid_barrier(bar)) return;
    }
    if (gtid == 0) {
        cnt[0] = 0u;
        cnt[1] = 0u;
    }
}

template <int LPR>
hipError_t persistent_launch(const RowSet &rs, const float *wepl, int64_t block_size,
                             double lambda, const DropBuffers &b, int grid_wgs, hipStream_t stream)
{
    if (rs.n <= 0) return hipSuccess;
    if (rs.chord16)
        hipLaunchKernelGGL((k_drop_persistent<LPR, __half>), dim3(grid_wgs), dim3(kThreads), 0,
                           stream, rs, rs.chord16, wepl, block_size, lambda, b.x, b.c, b.s,
                           b.touched, b.ntouched, b.barrier);
    else
        hipLaunchKernelGGL((k_drop_persistent<LPR, float>), dim3(grid_wgs), dim3(kThreads), 0,
                           stream, rs, rs.chord32, wepl, block_size, lambda, b.x, b.c, b.s,
                           b.touched, b.ntouched, b.barrier);
    return hipGetLastError();
}

// Scatter-only row kernel of the per-block form: dot, residual, then
// fire-and-forget float64 / uint32 atomics (no touched list: the apply
// pass scans the hit counts densely).
template <int LPR, typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_rows_dense(RowSet rs, const CH *chord, const float *wepl, int64_t r0, int64_t r1,
                  const double *x, double *c, uint32_t *s)
{
    const int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / LPR;
    if (row >= r1) return;
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    if (!(n2 > 0.0f)) return;   // uniform over the group
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    double acc = 0.0;
    for (int64_t e = off + lane; e < end; e += LPR)
        acc += (double)chord_at(chord, e) * x[rs.idx[e]];
    acc = group_sum<LPR>(acc);
    const double r = ((double)wepl[row] - acc) / (double)n2;
    for (int64_t e = off + lane; e < end; e += LPR) {
        const int32_t j = rs.idx[e];
        unsafeAtomicAdd(c + j, r * (double)chord_at(chord, e));
        __hip_atomic_fetch_add(s + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Packed scatter: correction and hit count of an entry in one 64-bit integer
// atomic.  Bits 48..63 count hits; bits 0..47 hold the correction in two's-
// complement fixed point with kFrac fraction bits (exact, order-independent
// integer sums).  A contribution larger than `big` (chosen by the host so
// that no voxel's sum can leave the 48-bit field) goes to a float64 atomic
// instead, with a count-only packed increment, and sets the voxel's bit in
// the outlier mask so that the apply reads the float64 part only there.
constexpr int kFrac = 30;
constexpr double kScale = (double)(1ull << kFrac);
constexpr uint64_t kHit = 1ull << 48;

// The first kHeld chunks of LPR entries of a row are loaded once, all at
// once (their gathers then overlap instead of forming a chain), and kept in
// registers for the scatter; entries past them are streamed twice.  Every
// lane sums its entries in ascending order either way.
constexpr int kHeld = 4;

template <int LPR, typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_rows_packed(RowSet rs, const CH *chord, const float *wepl, int64_t r0, int64_t r1,
                   const double *x, unsigned long long *P, double *c64, uint32_t *omask,
                   double big)
{
    const int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / LPR;
    if (row >= r1) return;
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    if (!(n2 > 0.0f)) return;
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    int32_t jh[kHeld];
    float ch[kHeld];
#pragma unroll
    for (int u = 0; u < kHeld; u++) {
        const int64_t e = off + lane + (int64_t)u * LPR;
        jh[u] = (e < end) ? rs.idx[e] : -1;
        ch[u] = (e < end) ? chord_at(chord, e) : 0.0f;
    }
    double xh[kHeld];
#pragma unroll
    for (int u = 0; u < kHeld; u++) xh[u] = (jh[u] >= 0) ? x[jh[u]] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kHeld; u++)
        if (jh[u] >= 0) acc += (double)ch[u] * xh[u];
    for (int64_t e = off + lane + (int64_t)kHeld * LPR; e < end; e += LPR)
        acc += (double)chord_at(chord, e) * x[rs.idx[e]];
    acc = group_sum<LPR>(acc);
    const double r = ((double)wepl[row] - acc) / (double)n2;
    auto scatter = [&](int32_t j, float a) {
        const double v = r * (double)a;
        if (fabs(v) <= big) {
            const long long f = __double2ll_rn(v * kScale);
            atomicAdd(P + j, (unsigned long long)kHit + (unsigned long long)f);
        } else {
            unsafeAtomicAdd(c64 + j, v);
            atomicAdd(P + j, (unsigned long long)kHit);
            atomicOr(omask + (j >> 5), 1u << (j & 31));
        }
    };
#pragma unroll
    for (int u = 0; u < kHeld; u++)
        if (jh[u] >= 0) scatter(jh[u], ch[u]);
    for (int64_t e = off + lane + (int64_t)kHeld * LPR; e < end; e += LPR)
        scatter(rs.idx[e], chord_at(chord, e));
}

// Voxel j is handled by a lane of the same wavefront instruction as the 31
// other voxels of its mask word (the stride is a multiple of 32), so the
// word's first lane may clear it right after the wavefront has read it.
__global__ void __launch_bounds__(kThreads)
k_drop_apply_packed(double lambda, double *x, unsigned long long *P, double *c64,
                    uint32_t *omask, int64_t nvox)
{
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < nvox;
         j += (int64_t)gridDim.x * kThreads) {
        // x is read with P (not after testing P) so the two loads overlap
        const unsigned long long p = P[j];
        const uint32_t m = omask[j >> 5];
        const double xj = x[j];
        if (m != 0u && (j & 31) == 0) omask[j >> 5] = 0u;
        if (p == 0ull) continue;
        const unsigned long long hits = (p + (1ull << 47)) >> 48;
        const long long fixed = (long long)(p - (hits << 48));
        double c = (double)fixed * (1.0 / kScale);
        if ((m >> (j & 31)) & 1u) {
            c += c64[j];
            c64[j] = 0.0;
        }
        x[j] = xj + lambda * c / (double)hits;
        P[j] = 0ull;
    }
}

// Dense apply: every voxel with hits in the block takes its correction and
// clears its accumulators (a coalesced pass over the hit counts).
__global__ void __launch_bounds__(kThreads)
k_drop_apply_dense(double lambda, double *x, double *c, uint32_t *s, int64_t nvox)
{
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < nvox;
         j += (int64_t)gridDim.x * kThreads) {
        const uint32_t sj = s[j];
        if (sj == 0u) continue;
        x[j] += lambda * c[j] / (double)sj;
        c[j] = 0.0;
        s[j] = 0u;
    }
}

// Residuals of the rows [r0, r1) into rbuf[row - r0] (voxel-major apply).
template <int LPR, typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_resid(RowSet rs, const CH *chord, const float *wepl, int64_t r0, int64_t r1,
             const double *x, double *rbuf)
{
    const int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / LPR;
    if (row >= r1) return;
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    int32_t jh[kHeld];
    float ch[kHeld];
#pragma unroll
    for (int u = 0; u < kHeld; u++) {
        const int64_t e = off + lane + (int64_t)u * LPR;
        jh[u] = (e < end) ? rs.idx[e] : -1;
        ch[u] = (e < end) ? chord_at(chord, e) : 0.0f;
    }
    double xh[kHeld];
#pragma unroll
    for (int u = 0; u < kHeld; u++) xh[u] = (jh[u] >= 0) ? x[jh[u]] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kHeld; u++)
        if (jh[u] >= 0) acc += (double)ch[u] * xh[u];
    for (int64_t e = off + lane + (int64_t)kHeld * LPR; e < end; e += LPR)
        acc += (double)chord_at(chord, e) * x[rs.idx[e]];
    acc = group_sum<LPR>(acc);
    if (lane == 0) rbuf[row - r0] = (n2 > 0.0f) ? ((double)wepl[row] - acc) / (double)n2 : 0.0;
}

// x_j += lambda * (sum over column j of r_q a_qj) / (column length), one
// thread per distinct voxel of the block; columns are summed in row order.
template <typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_apply_csc(const int32_t *uvox, const uint32_t *ucol, int64_t U, int64_t ne,
                 const uint16_t *cq, const CH *cch, const double *rbuf, double lambda, double *x)
{
    for (int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x; u < U;
         u += (int64_t)gridDim.x * kThreads) {
        const int64_t s = ucol[u];
        const int64_t e = (u + 1 < U) ? (int64_t)ucol[u + 1] : ne;
        const int32_t vj = uvox[u];
        const double xj = x[vj];          // issued before the column's loads
        double c = 0.0;
        int64_t k = s;
        for (; k + 2 <= e; k += 2) {      // two entries' loads in flight at once
            const uint16_t q0 = cq[k], q1 = cq[k + 1];
            const float a0 = chord_at(cch, k), a1 = chord_at(cch, k + 1);
            const double b0 = rbuf[q0], b1 = rbuf[q1];
            c += b0 * (double)a0;
            c += b1 * (double)a1;
        }
        if (k < e) c += rbuf[cq[k]] * (double)chord_at(cch, k);
        x[vj] = xj + lambda * c / (double)(e - s);
    }
}

// Launches one kernel; with a timer pair the launch carries its own start and
// stop events, which take the dispatch's timestamps (no gap around it).
template <typename F, typename... Args>
void launch(F kernel, dim3 grid, hipStream_t stream, hipEvent_t t0, hipEvent_t t1,
            Args... args)
{
    hipExtLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, stream, t0, t1, 0u, args...);
}

template <int LPR>
hipError_t block_launch(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1, double lambda,
                        const DropBuffers &b, hipStream_t stream, const KTimer *kt)
{
    const int64_t rows = r1 - r0;
    if (rows <= 0) return hipSuccess;
    const KTimer none{};
    const KTimer &t = kt ? *kt : none;
    dim3 grid((unsigned)((rows * LPR + kThreads - 1) / kThreads));
    int64_t wgs = (b.nvox + kThreads - 1) / kThreads;
    if (wgs > 8192) wgs = 8192;
    if (b.c64) {
        unsigned long long *P = reinterpret_cast<unsigned long long *>(b.c);
        if (rs.chord16)
            launch(k_drop_rows_packed<LPR, __half>, grid, stream, t.e[0], t.e[1], rs, rs.chord16,
                   wepl, r0, r1, (const double *)b.x, P, b.c64, b.omask, b.big);
        else
            launch(k_drop_rows_packed<LPR, float>, grid, stream, t.e[0], t.e[1], rs, rs.chord32,
                   wepl, r0, r1, (const double *)b.x, P, b.c64, b.omask, b.big);
        launch(k_drop_apply_packed, dim3((unsigned)wgs), stream, t.e[2], t.e[3], lambda, b.x, P,
               b.c64, b.omask, b.nvox);
        return hipGetLastError();
    }
    if (rs.chord16)
        launch(k_drop_rows_dense<LPR, __half>, grid, stream, t.e[0], t.e[1], rs, rs.chord16, wepl,
               r0, r1, (const double *)b.x, b.c, b.s);
    else
        launch(k_drop_rows_dense<LPR, float>, grid, stream, t.e[0], t.e[1], rs, rs.chord32, wepl,
               r0, r1, (const double *)b.x, b.c, b.s);
    launch(k_drop_apply_dense, dim3((unsigned)wgs), stream, t.e[2], t.e[3], lambda, b.x, b.c, b.s,
           b.nvox);
    return hipGetLastError();
}

template <int LPR>
hipError_t csc_block_launch(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                            double lambda, const CscBlock &cb, double *x, double *rbuf,
                            hipStream_t stream, const KTimer *kt)
{
    const int64_t rows = r1 - r0;
    if (rows <= 0) return hipSuccess;
    const KTimer none{};
    const KTimer &t = kt ? *kt : none;
    dim3 grid((unsigned)((rows * LPR + kThreads - 1) / kThreads));
    if (rs.chord16)
        launch(k_drop_resid<LPR, __half>, grid, stream, t.e[0], t.e[1], rs, rs.chord16, wepl, r0,
               r1, (const double *)x, rbuf);
    else
        launch(k_drop_resid<LPR, float>, grid, stream, t.e[0], t.e[1], rs, rs.chord32, wepl, r0,
               r1, (const double *)x, rbuf);
    if (cb.U <= 0) return hipGetLastError();
    int64_t wgs = (cb.U + kThreads - 1) / kThreads;
    if (wgs > 4096) wgs = 4096;
    if (cb.cch16)
        launch(k_drop_apply_csc<__half>, dim3((unsigned)wgs), stream, t.e[2], t.e[3], cb.uvox,
               cb.ucol, cb.U, cb.ne, cb.cq, cb.cch16, (const double *)rbuf, lambda, x);
    else
        launch(k_drop_apply_csc<float>, dim3((unsigned)wgs), stream, t.e[2], t.e[3], cb.uvox,
               cb.ucol, cb.U, cb.ne, cb.cq, cb.cch32, (const double *)rbuf, lambda, x);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_drop_block_csc(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                                 double lambda, const CscBlock &cb, double *x, double *rbuf,
                                 int lanes_per_row, hipStream_t stream, const KTimer *kt)
{
    switch (lanes_per_row) {
    case 16: return csc_block_launch<16>(rs, wepl, r0, r1, lambda, cb, x, rbuf, stream, kt);
    case 32: return csc_block_launch<32>(rs, wepl, r0, r1, lambda, cb, x, rbuf, stream, kt);
    default: return csc_block_launch<64>(rs, wepl, r0, r1, lambda, cb, x, rbuf, stream, kt);
    }
}

hipError_t launch_drop_block(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                             double lambda, const DropBuffers &b, int parity, int lanes_per_row,
                             hipStream_t stream, const KTimer *kt)
{
    (void)parity;
    switch (lanes_per_row) {
    case 16: return block_launch<16>(rs, wepl, r0, r1, lambda, b, stream, kt);
    case 32: return block_launch<32>(rs, wepl, r0, r1, lambda, b, stream, kt);
    default: return block_launch<64>(rs, wepl, r0, r1, lambda, b, stream, kt);
    }
}

hipError_t launch_zero_counters(uint32_t *cnt, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, cnt);
    return hipGetLastError();
}

hipError_t launch_drop_persistent(const RowSet &rs, const float *wepl, int64_t block_size,
                                  double lambda, const DropBuffers &b, int lanes_per_row,
                                  int grid_wgs, hipStream_t stream)
{
    switch (lanes_per_row) {
    case 16: return persistent_launch<16>(rs, wepl, block_size, lambda, b, grid_wgs, stream);
    case 32: return persistent_launch<32>(rs, wepl, block_size, lambda, b, grid_wgs, stream);
    default: return persistent_launch<64>(rs, wepl, block_size, lambda, b, grid_wgs, stream);
    }
}

int persistent_grid_size(int device, int lanes_per_row)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    hipError_t e;
    switch (lanes_per_row) {
    case 16:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_drop_persistent<16, float>), kThreads, 0);
        break;
    case 32:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_drop_persistent<32, float>), kThreads, 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_drop_persistent<64, float>), kThreads, 0);
        break;
    }
    if (e != hipSuccess || per_cu <= 0) return 0;
    // Stay well inside co-residency: at most 2 workgroups per CU.
    if (per_cu > 2) per_cu = 2;
    return cus * per_cu;
}

}  // namespace tvs
