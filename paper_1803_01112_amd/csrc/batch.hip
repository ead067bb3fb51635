// batch.hip -- S reconstructions of the same histories advanced together
// (a parameter study over (lambda, N, alpha) as in arXiv 1803.01112,
// Section III-E, run as one job instead of one reconstruction each).
//
// The S images are interleaved by voxel, x[p*S + s], so that the S values an
// entry reads are contiguous.  The DROP sweep is the tile-wise chain of
// drop.hip with S images at once: one workgroup per (tile, group of up to
// 16 settings) applies each entry of the tile's lists to the settings of its
// group through LDS; hit counts depend only on the rows.  The TV steps of every
// setting run in one kernel per step index n, with per-setting beta read
// from a device table indexed by a device cycle counter, so the launches of
// one cycle can be captured once in a hipGraph and replayed for every cycle.
#include "device_common.hpp"
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int kThreads = 256;
using dev::entry_chord;
using dev::row_of;
using dev::kNoRow;

constexpr double kDotUnit = 1.0 / kDotScale;
constexpr double kCorrUnit = 1.0 / kCorrScale;

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
    // a fixed grid strides over batches of V voxels (few partial sums)
    double sq = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * V + v; v < V && p < nvox;
         p += (int64_t)gridDim.x * V) {     // tiled-layout word
        int64_t i = 0, j = 0, k = 0;
        vcoord(G, p, i, j, k);
        if (!(i < nx && j < ny && ((active >> s) & 1u))) continue;
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
        sq += gv * gv;
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

unsigned elem_grid(int64_t n)
{
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 4096) wgs = 4096;
    if (wgs < 1) wgs = 1;
    return (unsigned)wgs;
}

// ------------------------------------------------------------- DROP, S images
// Settings per pass through LDS (GP: 2, 4, 8 or 16) and threads per workgroup
// (NT: 128 or 256) are template parameters, picked by the batch autotuner.

// LDS index of (voxel word w, setting s of the group): the settings of a
// voxel are XOR-swizzled by w so that lanes holding different voxels and the
// same setting fall into different banks (without it every voxel's setting s
// shares one bank pair).
template <int GP>
__device__ inline int sx(int w, int s) { return w * GP + (s ^ (w & (GP - 1))); }

template <int GP>
struct BatchLds {
    double x[kTileWords * GP];
    long long cf[kTileWords * GP];
    double cb[kTileWords * GP];
    uint32_t hits[kTileWords];
};

// One step of the tile-wise chain for S settings: finish block P and form
// the dot products of block C (dot arrays row-major: dot[q * S + s]).  The
// per-entry quotient a_ij / ||a_i||^2 and the per-voxel 1 / s_j are formed
// once and shared by the settings (a rounding apart from the single-image
// kernel, which divides per value).
template <int NT, int GP, typename CH>
__global__ void __launch_bounds__(NT)
k_drop_tile_batch(DropTileArgs A, int S, const double *lambda)
{
    __shared__ BatchLds<GP> L;
    const int t = threadIdx.x;
    if (A.zero)
        for (int64_t q = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * NT + t;
             q < A.B * S; q += (int64_t)gridDim.x * gridDim.y * NT)
            A.zero[q] = 0;
    // workgroup x takes dispatch slot x: its lists' bounds at [x], its tile act[x]
    const int64_t T = A.tiles[blockIdx.x];
    int64_t p0 = 0, p1 = 0, c0 = 0, c1 = 0;
    if (A.P.valid) {
        p0 = A.P.toff[blockIdx.x];
        p1 = A.P.toff[blockIdx.x + 1];
    }
    if (A.C.valid) {
        c0 = A.C.toff[blockIdx.x];
        c1 = A.C.toff[blockIdx.x + 1];
    }
    if (p0 == p1 && c0 == c1) return;
    double *xt = A.x + (T << kTileShift) * S;
    // the first round of both lists and the finished rows' data, loaded once
    // for all setting groups
    uint32_t pm = 0u, cm = 0u;
    double pa = 0.0, ca = 0.0, pw = 0.0, pn2 = 1.0;
    const bool pok = p0 + t < p1, cok = c0 + t < c1;
    if (pok) {
        pm = A.P.meta[p0 + t - A.P.base];
        pa = (double)entry_chord<CH>(A.P, p0 + t - A.P.base, pm);
    }
    if (cok) {
        cm = A.C.meta[c0 + t - A.C.base];
        ca = (double)entry_chord<CH>(A.C, c0 + t - A.C.base, cm);
    }
    if (pok && row_of(A.P, pm) < A.P.rows) {
        pw = (double)A.P.wepl[row_of(A.P, pm)];
        pn2 = (double)A.P.n2[row_of(A.P, pm)];
    }
    // one group of settings per workgroup (the grid's second dimension)
    {
        const int g0 = (int)blockIdx.y * GP;
        const int G = (S - g0 < GP) ? S - g0 : GP;
        for (int i = t; i < kTileWords * G; i += NT) {
            const int w = i / G, s = i - w * G;
            L.x[sx<GP>(w, s)] = xt[(int64_t)w * S + g0 + s];
        }
        if (p1 > p0) {
            for (int i = t; i < kTileWords * GP; i += NT) {
                L.cf[i] = 0;
                L.cb[i] = 0.0;
            }
            for (int w = t; w < kTileWords; w += NT) L.hits[w] = 0u;
            __syncthreads();
            for (int64_t e = p0 + t; e < p1; e += NT) {
                const bool first = e == p0 + t;
                const uint32_t m = first ? pm : A.P.meta[e - A.P.base];
                const int w = (int)(m & (kTileWords - 1));
                const uint32_t q = row_of(A.P, m);
                if (q >= A.P.rows) {
                    atomicOr(A.err, 2u);
                    continue;
                }
                const double a = first ? pa : (double)entry_chord<CH>(A.P, e - A.P.base, m);
                const double wp = first ? pw : (double)A.P.wepl[q];
                const double n2 = first ? pn2 : (double)A.P.n2[q];
                const double an2 = a / n2;   // one division for all settings
                atomicAdd(&L.hits[w], 1u);
                for (int s = 0; s < G; s++) {
                    const double res = wp - (double)A.P.dot[(int64_t)q * S + g0 + s] * kDotUnit;
                    const double v = res * an2;
                    if (fabs(v) <= A.big)
                        atomicAdd(reinterpret_cast<unsigned long long *>(&L.cf[sx<GP>(w, s)]),
                                  (unsigned long long)__double2ll_rn(v * kCorrScale));
                    else
                        atomicAdd(&L.cb[sx<GP>(w, s)], v);
                }
            }
            __syncthreads();
            for (int w = t; w < kTileWords; w += NT) {
                const uint32_t h = L.hits[w];
                if (!h) continue;
                const double inv_h = 1.0 / (double)h;   // one division for all settings
                for (int s = 0; s < G; s++) {
                    const int k = sx<GP>(w, s);
                    const double c = (double)L.cf[k] * kCorrUnit + L.cb[k];
                    const double nx = L.x[k] + lambda[g0 + s] * c * inv_h;
                    L.x[k] = nx;
                    xt[(int64_t)w * S + g0 + s] = nx;
                }
            }
        }
        __syncthreads();
        // every thread runs the same rounds and settings (the shuffles are
        // uniform).  The run sums of the group's settings are staged in LDS
        // (in the finish sums' space, free by now) and leave as atomics of GP
        // settings of one row each: one line per run instead of GP.
        const int wave = t >> 6, lane = t & 63;
        long long *stg_v = reinterpret_cast<long long *>(L.cb) + wave * 64 * GP;
        uint32_t *stg_q = L.hits + wave * 64;
        for (int64_t r0 = c0; r0 < c1; r0 += NT) {
            const int64_t e = r0 + t;
            uint32_t q = kNoRow;
            int w = 0;
            double a = 0.0;
            if (e < c1) {
                const bool first = r0 == c0;
                const uint32_t m = first ? cm : A.C.meta[e - A.C.base];
                q = row_of(A.C, m);
                w = (int)(m & (kTileWords - 1));
                a = first ? ca : (double)entry_chord<CH>(A.C, e - A.C.base, m);
                if (q >= A.C.rows) {
                    atomicOr(A.err, 2u);
                    q = kNoRow;
                }
            }
            const dev::Runs runs = dev::wave_runs(q);
            const bool emit = runs.tail && q != kNoRow;
            const unsigned long long tails = __ballot(emit);
            const int k = __popcll(tails & ((1ull << lane) - 1ull));
            for (int s = 0; s < G; s++) {
                long long f = 0;
                if (q != kNoRow) {
                    const double p = a * L.x[sx<GP>(w, s)];
                    if (fabs(p) <= A.dot_max) f = __double2ll_rn(p * kDotScale);
                    else atomicOr(A.err, 1u);
                }
                f = dev::run_sum(f, runs);
                if (emit) stg_v[k * GP + s] = f;
            }
            if (emit) stg_q[k] = q;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const int n = __popcll(tails);
            for (int b = 0; b < n; b += 64 / GP) {
                const int j = b + lane / GP, s = lane & (GP - 1);
                if (j < n && s < G)
                    atomicAdd(reinterpret_cast<unsigned long long *>(A.C.dot + (int64_t)stg_q[j] * S +
                                                                     g0 + s),
                              (unsigned long long)stg_v[j * GP + s]);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
    }
}

}  // namespace

int batch_vox_per_wg(int S) { return kThreads / S; }

int64_t batch_num_parts(const GridDev &g, int S)
{
    const int64_t nvox = padded_voxels(g);
    const int V = batch_vox_per_wg(S);
    const int64_t batches = (nvox + V - 1) / V;
    return batches < 1024 ? batches : 1024;    // the gradient kernel's grid
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

namespace {

template <int NT, int GP>
hipError_t drop_batch(const DropTileArgs &a, const BatchBuffers &b, hipStream_t stream)
{
    const TileBlock &v = a.P.valid ? a.P : a.C;
    const dim3 grid((unsigned)a.nact, (unsigned)((b.S + GP - 1) / GP));
    if (v.chq)
        hipLaunchKernelGGL((k_drop_tile_batch<NT, GP, uint16_t>), grid, dim3(NT), 0, stream, a,
                           b.S, (const double *)b.lambda);
    else if (v.ch16)
        hipLaunchKernelGGL((k_drop_tile_batch<NT, GP, __half>), grid, dim3(NT), 0, stream, a, b.S,
                           (const double *)b.lambda);
    else
        hipLaunchKernelGGL((k_drop_tile_batch<NT, GP, float>), grid, dim3(NT), 0, stream, a, b.S,
                           (const double *)b.lambda);
    return hipGetLastError();
}

}  // namespace

bool batch_shape_ok(int threads, int group)
{
    return (threads == 128 || threads == 256) &&
           (group == 2 || group == 4 || group == 8 || group == 16);
}

hipError_t launch_drop_tiles_batch(const DropTileArgs &a, const BatchBuffers &b, int64_t ntiles,
                                   int threads, int group, hipStream_t stream)
{
    if (ntiles <= 0 || (!a.P.valid && !a.C.valid) || !a.tiles || a.nact <= 0) return hipSuccess;
    if (threads == 128) {
        if (group == 2) return drop_batch<128, 2>(a, b, stream);
        if (group == 4) return drop_batch<128, 4>(a, b, stream);
        if (group == 16) return drop_batch<128, 16>(a, b, stream);
        return drop_batch<128, 8>(a, b, stream);
    }
    if (group == 2) return drop_batch<256, 2>(a, b, stream);
    if (group == 4) return drop_batch<256, 4>(a, b, stream);
    if (group == 16) return drop_batch<256, 16>(a, b, stream);
    return drop_batch<256, 8>(a, b, stream);
}

}  // namespace tvs
