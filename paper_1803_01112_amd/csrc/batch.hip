// batch.hip -- S reconstructions of the same histories advanced together
// (a parameter study over (lambda, N, alpha) as in arXiv 1803.01112,
// Section III-E, run as one job instead of one reconstruction each).
//
// The S images are interleaved by voxel, x[p*S + s], so that the S values a
// row entry gathers (or scatters) are contiguous.  One persistent sweep reads
// each row once from HBM and applies it to all S images: per row, S float64
// dot products (cross-lane sums), S residuals, S float64 atomic scatters per
// entry; hit counts s_j and the touched list depend only on the rows and are
// shared.  The TV steps of every setting run in one kernel per step index n,
// with per-setting beta read from a device table indexed by a device cycle
// counter, so the launches of one cycle can be captured once in a hipGraph
// and replayed for every cycle.
#include "device_common.hpp"
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int kThreads = 256;
using dev::append_touched;
using dev::chord_at;
using dev::grid_barrier;
using dev::group_sum;

// ------------------------------------------------------------- TV, S images
// Thread t of a workgroup handles setting s = t % S of voxel w*V + t / S.
__global__ void __launch_bounds__(kThreads)
k_tvb_grad(GridDev G, const double *x, int S, int V, uint32_t active, const double *eps,
           double *g, double *part, uint32_t *ticket, double *norm2)
{
    __shared__ double red[kThreads];
    __shared__ uint32_t last;
    const int t = threadIdx.x;
    const int v = t / S, s = t - v * S;
    const int64_t nx = G.nx, ny = G.ny;
    const int64_t nvox = padded_voxels(G);
    const int64_t p = (int64_t)blockIdx.x * V + v;     // brick-layout word
    int64_t i = 0, j = 0, k = 0;
    if (p < nvox) vcoord(G, p, i, j, k);
    double sq = 0.0;
    if (v < V && p < nvox && i < nx && j < ny && ((active >> s) & 1u)) {
        const double e2 = eps[s] * eps[s];
        auto X = [&](int64_t di, int64_t dj) { return x[vaddr(G, i + di, j + dj, k) * S + s]; };
        auto dxf = [&](int64_t ii, int64_t jj) {
            return (i + ii + 1 < nx) ? X(ii + 1, jj) - X(ii, jj) : 0.0;
        };
        auto dyf = [&](int64_t ii, int64_t jj) {
            return (j + jj + 1 < ny) ? X(ii, jj + 1) - X(ii, jj) : 0.0;
        };
        auto mf = [&](int64_t ii, int64_t jj) {
            double a = dxf(ii, jj), b = dyf(ii, jj);
            return sqrt(a * a + b * b + e2);
        };
        double gv = 0.0;
        double m = mf(0, 0);
        if (m > 0.0) gv -= (dxf(0, 0) + dyf(0, 0)) / m;
        if (i > 0) {
            double mm = mf(-1, 0);
            if (mm > 0.0) gv += dxf(-1, 0) / mm;
        }
        if (j > 0) {
            double mm = mf(0, -1);
            if (mm > 0.0) gv += dyf(0, -1) / mm;
        }
        g[p * S + s] = gv;
        sq = gv * gv;
    }
    red[t] = sq;
    __syncthreads();
    if (t < S) {
        double a = 0.0;
        for (int vv = 0; vv < V; vv++) a += red[vv * S + t];
        part[(int64_t)blockIdx.x * S + t] = a;
    }
    __syncthreads();
    if (t == 0) {
        __threadfence();
        uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (old == gridDim.x - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double a = 0.0;
    if (v < V)
        for (uint32_t w = v; w < gridDim.x; w += V)
            a += __hip_atomic_load(part + (int64_t)w * S + s, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    red[t] = a;
    __syncthreads();
    if (t < S) {
        double b = 0.0;
        for (int vv = 0; vv < V; vv++) b += red[vv * S + t];
        norm2[t] = b;
    }
    if (t == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// x += (-beta_s / ||g_s||) g for the active settings; beta of step n of the
// current cycle is beta_tab[(cyc * nmax + n) * S + s].
__global__ void __launch_bounds__(kThreads)
k_tvb_step(double *x, const double *g, int S, int64_t n_elems, uint32_t active,
           const double *beta_tab, const int32_t *cyc, int n, int nmax, const double *norm2)
{
    const int64_t base = ((int64_t)(*cyc) * nmax + n) * S;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n_elems;
         q += (int64_t)gridDim.x * kThreads) {
        const int s = (int)(q % S);
        if (!((active >> s) & 1u)) continue;
        const double nn = norm2[s];
        const double sc = (nn > 0.0) ? -beta_tab[base + s] / sqrt(nn) : 0.0;
        if (sc != 0.0) x[q] = fma(sc, g[q], x[q]);
    }
}

__global__ void k_set_counter(int32_t *cyc, int32_t v)
{
    if (threadIdx.x == 0) *cyc = v;
}

__global__ void k_tick(int32_t *cyc)
{
    if (threadIdx.x == 0) *cyc += 1;
}

__global__ void __launch_bounds__(kThreads)
k_replicate(const double *x0, double *xb, int S, int64_t nvox)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < nvox * S;
         q += (int64_t)gridDim.x * kThreads)
        xb[q] = x0[q / S];
}

__global__ void __launch_bounds__(kThreads)
k_extract(GridDev G, const double *xb, int S, int s, float *out)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads) {
        const int64_t i = p % G.nx, t = p / G.nx, j = t % G.ny, k = t / G.ny;
        out[p] = (float)xb[vaddr(G, i, j, k) * S + s];
    }
}

__global__ void __launch_bounds__(kThreads) k_zero_d(double *p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads)
        p[q] = 0.0;
}

// ------------------------------------------------------------- DROP, S images
template <int SMAX, typename CH>
__device__ inline void drop_row_batch(const RowSet &rs, const CH *chord, const float *wepl,
                                      int64_t row, int S, const double *x, double *c,
                                      uint32_t *s, int32_t *touched, uint32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    if (!(n2 > 0.0f)) return;   // uniform over the wavefront
    double acc[SMAX];
#pragma unroll
    for (int k = 0; k < SMAX; k++) acc[k] = 0.0;
    for (int64_t e = off + lane; e < end; e += 64) {
        const double ch = (double)chord_at(chord, e);
        const double *xp = x + (int64_t)rs.idx[e] * S;
#pragma unroll
        for (int k = 0; k < SMAX; k++)
            if (k < S) acc[k] += ch * xp[k];
    }
    const double b = (double)wepl[row];
#pragma unroll
    for (int k = 0; k < SMAX; k++) {
        if (k < S) acc[k] = (b - group_sum<64>(acc[k])) / (double)n2;   // residual r_k
        else acc[k] = 0.0;
    }
    const int64_t trips = (end - off + 63) / 64;
    for (int64_t q = 0; q < trips; q++) {
        const int64_t e = off + q * 64 + lane;
        bool first = false;
        int32_t j = 0;
        if (e < end) {
            j = rs.idx[e];
            const double ch = (double)chord_at(chord, e);
            double *cp = c + (int64_t)j * S;
#pragma unroll
            for (int k = 0; k < SMAX; k++)
                if (k < S) unsafeAtomicAdd(cp + k, acc[k] * ch);
            first = (atomicAdd(s + j, 1u) == 0u);
        }
        append_touched(first, j, touched, cnt);
    }
}

template <int SMAX, typename CH>
__global__ void __launch_bounds__(kThreads)
k_drop_batch(RowSet rs, const CH *chord, const float *wepl, int64_t block_size, int S,
             const double *lambda, double *x, double *c, uint32_t *s, int32_t *touched,
             uint32_t *cnt, uint32_t *bar)
{
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    const int64_t wid = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 64;
    const int64_t gthreads = (int64_t)gridDim.x * kThreads;
    const int64_t gtid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nblocks = (rs.n + block_size - 1) / block_size;
    for (int64_t t = 0; t < nblocks; t++) {
        const int64_t r0 = rs.first + t * block_size;
        const int64_t r1 = (r0 + block_size < rs.first + rs.n) ? r0 + block_size : rs.first + rs.n;
        uint32_t *cur = cnt + (t & 1);
        for (int64_t row = r0 + wid; row < r1; row += waves)
            drop_row_batch<SMAX, CH>(rs, chord, wepl, row, S, x, c, s, touched, cur);
        if (!grid_barrier(bar)) return;
        const uint32_t n = *cur;
        for (int64_t i = gtid; i < (int64_t)n; i += gthreads) {
            const int64_t j = touched[i];
            const double inv = 1.0 / (double)s[j];
            double *xp = x + j * S;
            double *cp = c + j * S;
            for (int k = 0; k < S; k++) {
                xp[k] += lambda[k] * cp[k] * inv;
                cp[k] = 0.0;
            }
            s[j] = 0u;
        }
        if (gtid == 0) cnt[(t + 1) & 1] = 0u;
        if (!grid_barrier(bar)) return;
    }
    if (gtid == 0) {
        cnt[0] = 0u;
        cnt[1] = 0u;
    }
}

// ------------------------------------------------------------- voxel-major form
// Residuals r[q*S + s] of the rows [r0, r1) for every setting: one wavefront
// per row, S float64 dot products over the row's entries.
template <int SMAX, typename CH>
__global__ void __launch_bounds__(kThreads)
k_batch_resid(RowSet rs, const CH *chord, const float *wepl, int64_t r0, int64_t r1, int S,
              const double *x, double *rbuf)
{
    const int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 64;
    if (row >= r1) return;
    const int lane = threadIdx.x & 63;
    const int64_t lr = row - rs.first;
    const float n2 = rs.norm2[lr];
    const int64_t off = rs.row_off[lr] - rs.base, end = rs.row_off[lr + 1] - rs.base;
    double acc[SMAX];
#pragma unroll
    for (int k = 0; k < SMAX; k++) acc[k] = 0.0;
    for (int64_t e = off + lane; e < end; e += 64) {
        const double ch = (double)chord_at(chord, e);
        const double *xp = x + (int64_t)rs.idx[e] * S;
#pragma unroll
        for (int k = 0; k < SMAX; k++)
            if (k < S) acc[k] += ch * xp[k];
    }
    const double b = (double)wepl[row];
    double *rp = rbuf + (row - r0) * S;
#pragma unroll
    for (int k = 0; k < SMAX; k++) {
        if (k < S) {
            const double d = group_sum<64>(acc[k]);
            if (lane == k) rp[k] = (n2 > 0.0f) ? (b - d) / (double)n2 : 0.0;
        }
    }
}

// One thread per (distinct voxel, setting): the column sum in row order.
template <typename CH>
__global__ void __launch_bounds__(kThreads)
k_batch_apply_csc(const int32_t *uvox, const uint32_t *ucol, int64_t U, int64_t ne,
                  const uint16_t *cq, const CH *cch, const double *rbuf, int S,
                  const double *lambda, double *x)
{
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < U * S;
         t += (int64_t)gridDim.x * kThreads) {
        const int64_t u = t / S;
        const int k = (int)(t - u * S);
        const int64_t s0 = ucol[u];
        const int64_t e0 = (u + 1 < U) ? (int64_t)ucol[u + 1] : ne;
        double c = 0.0;
        for (int64_t q = s0; q < e0; q++) c += rbuf[(int64_t)cq[q] * S + k] * (double)chord_at(cch, q);
        x[(int64_t)uvox[u] * S + k] += lambda[k] * c / (double)(e0 - s0);
    }
}

unsigned elem_grid(int64_t n)
{
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 8192) wgs = 8192;
    if (wgs < 1) wgs = 1;
    return (unsigned)wgs;
}

template <int SMAX>
hipError_t drop_batch_launch(const RowSet &rs, const float *wepl, int64_t block_size,
                             const BatchBuffers &b, int grid_wgs, hipStream_t stream)
{
    if (rs.chord16)
        hipLaunchKernelGGL((k_drop_batch<SMAX, __half>), dim3(grid_wgs), dim3(kThreads), 0, stream,
                           rs, rs.chord16, wepl, block_size, b.S, b.lambda, b.x, b.c, b.s,
                           b.touched, b.ntouched, b.barrier);
    else
        hipLaunchKernelGGL((k_drop_batch<SMAX, float>), dim3(grid_wgs), dim3(kThreads), 0, stream,
                           rs, rs.chord32, wepl, block_size, b.S, b.lambda, b.x, b.c, b.s,
                           b.touched, b.ntouched, b.barrier);
    return hipGetLastError();
}

template <int SMAX>
int occupancy_of()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_drop_batch<SMAX, float>), kThreads, 0) !=
        hipSuccess)
        return 0;
    return per_cu;
}

template <int SMAX>
hipError_t batch_csc_launch(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                            const CscBlock &cb, const BatchBuffers &b, double *rbuf,
                            hipStream_t stream)
{
    const int64_t rows = r1 - r0;
    if (rows <= 0) return hipSuccess;
    dim3 grid((unsigned)((rows * 64 + kThreads - 1) / kThreads));
    if (rs.chord16)
        hipLaunchKernelGGL((k_batch_resid<SMAX, __half>), grid, dim3(kThreads), 0, stream, rs,
                           rs.chord16, wepl, r0, r1, b.S, b.x, rbuf);
    else
        hipLaunchKernelGGL((k_batch_resid<SMAX, float>), grid, dim3(kThreads), 0, stream, rs,
                           rs.chord32, wepl, r0, r1, b.S, b.x, rbuf);
    if (cb.U <= 0) return hipGetLastError();
    const unsigned wgs = elem_grid(cb.U * b.S);
    if (cb.cch16)
        hipLaunchKernelGGL((k_batch_apply_csc<__half>), dim3(wgs), dim3(kThreads), 0, stream,
                           cb.uvox, cb.ucol, cb.U, cb.ne, cb.cq, cb.cch16, rbuf, b.S, b.lambda, b.x);
    else
        hipLaunchKernelGGL((k_batch_apply_csc<float>), dim3(wgs), dim3(kThreads), 0, stream,
                           cb.uvox, cb.ucol, cb.U, cb.ne, cb.cq, cb.cch32, rbuf, b.S, b.lambda, b.x);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_block_csc(const RowSet &rs, const float *wepl, int64_t r0, int64_t r1,
                                  const CscBlock &cb, const BatchBuffers &b, double *rbuf,
                                  hipStream_t stream)
{
    if (b.S <= 8) return batch_csc_launch<8>(rs, wepl, r0, r1, cb, b, rbuf, stream);
    if (b.S <= 16) return batch_csc_launch<16>(rs, wepl, r0, r1, cb, b, rbuf, stream);
    return batch_csc_launch<32>(rs, wepl, r0, r1, cb, b, rbuf, stream);
}

int batch_vox_per_wg(int S) { return kThreads / S; }

int64_t batch_num_parts(const GridDev &g, int S)
{
    const int64_t nvox = padded_voxels(g);
    const int V = batch_vox_per_wg(S);
    return (nvox + V - 1) / V;
}

hipError_t launch_tvb_grad(const GridDev &g, const BatchBuffers &b, uint32_t active,
                           hipStream_t stream)
{
    const int V = batch_vox_per_wg(b.S);
    hipLaunchKernelGGL(k_tvb_grad, dim3((unsigned)batch_num_parts(g, b.S)), dim3(V * b.S), 0,
                       stream, g, b.x, b.S, V, active, b.eps, b.g, b.part, b.ticket, b.norm2);
    return hipGetLastError();
}

hipError_t launch_tvb_step(const BatchBuffers &b, uint32_t active, int n, int nmax,
                           hipStream_t stream)
{
    const int64_t ne = b.nvox * b.S;
    hipLaunchKernelGGL(k_tvb_step, dim3(elem_grid(ne)), dim3(kThreads), 0, stream, b.x, b.g, b.S,
                       ne, active, b.beta_tab, b.cyc, n, nmax, b.norm2);
    return hipGetLastError();
}

hipError_t launch_set_counter(int32_t *cyc, int32_t v, hipStream_t stream)
{
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, stream, cyc, v);
    return hipGetLastError();
}

hipError_t launch_tick(int32_t *cyc, hipStream_t stream)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, stream, cyc);
    return hipGetLastError();
}

hipError_t launch_replicate(const double *x0, const BatchBuffers &b, hipStream_t stream)
{
    hipLaunchKernelGGL(k_replicate, dim3(elem_grid(b.nvox * b.S)), dim3(kThreads), 0, stream, x0,
                       b.x, b.S, b.nvox);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_zero_d, dim3(elem_grid(b.nvox * b.S)), dim3(kThreads), 0, stream, b.c,
                       b.nvox * b.S);
    return hipGetLastError();
}

hipError_t launch_extract(const GridDev &g, const BatchBuffers &b, int s, float *out,
                          hipStream_t stream)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_extract, dim3(elem_grid(n)), dim3(kThreads), 0, stream, g, b.x, b.S, s,
                       out);
    return hipGetLastError();
}

hipError_t launch_drop_batch(const RowSet &rs, const float *wepl, int64_t block_size,
                             const BatchBuffers &b, int grid_wgs, hipStream_t stream)
{
    if (rs.n <= 0) return hipSuccess;
    if (b.S <= 8) return drop_batch_launch<8>(rs, wepl, block_size, b, grid_wgs, stream);
    if (b.S <= 16) return drop_batch_launch<16>(rs, wepl, block_size, b, grid_wgs, stream);
    return drop_batch_launch<32>(rs, wepl, block_size, b, grid_wgs, stream);
}

int batch_grid_size(int device, int S)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    int per_cu = (S <= 8) ? occupancy_of<8>() : (S <= 16) ? occupancy_of<16>() : occupancy_of<32>();
    if (per_cu <= 0) return 0;
    if (per_cu > 2) per_cu = 2;
    return cus * per_cu;
}

}  // namespace tvs
