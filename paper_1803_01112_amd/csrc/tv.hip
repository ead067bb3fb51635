// tv.hip -- total variation, its subgradient and the normalised perturbation
// step on gfx950 (arXiv 1803.01112: phi = TV, the local variations added over
// every voxel, Section IV; v = -grad phi / ||grad phi||, Appendix A).
//
// TV is taken per slice (2-D isotropic forward differences, zero difference
// past the last row/column): m_ij = sqrt(dx^2 + dy^2 + eps^2),
// phi = sum (m_ij - eps).  The subgradient at x_ij collects the terms of
// m_ij, m_(i-1)j and m_i(j-1); a term whose m is zero contributes zero.
//
// The image and the subgradient are float64 on the device: DROP increments
// with a small relaxation are tiny next to the RSP itself, and the
// subgradient only sees the direction of (dx, dy), so a float32 image would
// turn its rounding into order-one changes of v.  A workgroup stages 64x4
// tiles of one slice plus a one-voxel halo in LDS (a grid of at most 1024
// workgroups strides over the tiles), evaluates the stencil, and writes a
// float64 partial sum.  The last workgroup to finish (ticket counter) adds
// the partials in a fixed order, so every reduction is deterministic and no
// host round trip is needed between the gradient and the update.
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int TX = 64, TY = 4, kThreads = TX * TY;
constexpr int HX = TX + 2, HY = TY + 2;

// Loads the tile of slice z (origin i0, j0) with a one-voxel halo.
__device__ inline void load_tile(double (*t)[HX], const double *x, const GridDev &G, int z, int i0,
                                 int j0)
{
    for (int q = threadIdx.x; q < HX * HY; q += kThreads) {
        int ly = q / HX, lx = q - ly * HX;
        int i = i0 + lx - 1, j = j0 + ly - 1;
        double v = 0.0;
        if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) v = x[vaddr(G, i, j, z)];
        t[ly][lx] = v;
    }
    __syncthreads();
}

__device__ inline double step_scale(double beta, const double *n2)
{
    double nn = *n2;
    return (nn > 0.0) ? -beta / sqrt(nn) : 0.0;
}

struct Stencil {
    const double (*t)[HX];
    int nx, ny, i0, j0;
    double eps2;
    __device__ double X(int i, int j) const { return t[j - j0 + 1][i - i0 + 1]; }
    __device__ double dx(int i, int j) const { return (i + 1 < nx) ? X(i + 1, j) - X(i, j) : 0.0; }
    __device__ double dy(int i, int j) const { return (j + 1 < ny) ? X(i, j + 1) - X(i, j) : 0.0; }
    __device__ double m(int i, int j) const
    {
        double a = dx(i, j), b = dy(i, j);
        return sqrt(a * a + b * b + eps2);
    }
};

__device__ inline double block_sum(double v)
{
    __shared__ double red[kThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; q++) tot += red[q];
    __syncthreads();
    return tot;   // valid in thread 0
}

// Writes this workgroup's partial; the last workgroup reduces all partials
// in a fixed order into *out and re-arms the ticket.  The partials are read
// with plain loads after the acquire that observed the last ticket (every
// writer released its partial before taking a ticket), four in flight per
// lane.
__device__ inline void finish_reduction(double partial, double *part, uint32_t *ticket,
                                        double *out)
{
    __shared__ uint32_t last;
    const uint32_t nwg = gridDim.x;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = partial;
        __threadfence();
        uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
        last = (old == nwg - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double v = 0.0;
#pragma unroll 4
    for (uint32_t q = threadIdx.x; q < nwg; q += kThreads) v += part[q];
    double tot = block_sum(v);
    if (threadIdx.x == 0) {
        *out = tot;
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Tiles of TX x TY voxels of one slice; a capped grid of workgroups strides
// over them (tile T of workgroup w: T = w, w + gridDim.x, ...), so the
// reductions have few partial sums.
constexpr int kMaxWgs = 1024;

struct TileGrid {
    int tx, ty, nz;
    __device__ int64_t count() const { return (int64_t)tx * ty * nz; }
    __device__ void at(int64_t T, int &i0, int &j0, int &zz) const
    {
        i0 = (int)(T % tx) * TX;
        j0 = (int)((T / tx) % ty) * TY;
        zz = (int)(T / ((int64_t)tx * ty));
    }
};

__device__ inline TileGrid tile_grid(const GridDev &G)
{
    return TileGrid{(G.nx + TX - 1) / TX, (G.ny + TY - 1) / TY, G.nz};
}

__global__ void __launch_bounds__(kThreads)
k_tv_grad(GridDev G, const double *x, double eps, double *gout, double *part, uint32_t *ticket,
          double *out)
{
    __shared__ double tile[HY][HX];
    const TileGrid TG = tile_grid(G);
    double sq = 0.0;
    for (int64_t T = blockIdx.x; T < TG.count(); T += gridDim.x) {
        int i0, j0, zz;
        TG.at(T, i0, j0, zz);
        __syncthreads();
        load_tile(tile, x, G, zz, i0, j0);
        const int i = i0 + (threadIdx.x % TX), j = j0 + (threadIdx.x / TX);
        if (i < G.nx && j < G.ny) {
            Stencil S{tile, G.nx, G.ny, i0, j0, eps * eps};
            double gv = 0.0;
            double m = S.m(i, j);
            if (m > 0.0) gv -= (S.dx(i, j) + S.dy(i, j)) / m;
            if (i > 0) {
                double mm = S.m(i - 1, j);
                if (mm > 0.0) gv += S.dx(i - 1, j) / mm;
            }
            if (j > 0) {
                double mm = S.m(i, j - 1);
                if (mm > 0.0) gv += S.dy(i, j - 1) / mm;
            }
            gout[vaddr(G, i, j, zz)] = gv;
            sq += gv * gv;
        }
    }
    finish_reduction(block_sum(sq), part, ticket, out);
}

// ---------------------------------------------------------------- checked step
// The TV-reduction check of a perturbation step (Appendix C, with beta =
// alpha^ell recomputed after every ell += 1) decided on the device.  One
// launch evaluates TV(x) and TV(x + s_t g) for the first kTries tries t
// (s_t = -alpha^(ell + t) / ||g||) in one pass over the tiles; the last
// workgroup to finish adds every workgroup's partials in a fixed order,
// takes the first try with TV(z) <= TV(x), and, only when none of them
// passes, evaluates further rounds of kTries tries alone (rare: each round
// shrinks the step by alpha^kTries).  It records the decision (scale and
// flag, read by k_tv_apply), advances ell by the tries and writes the step's
// log record.  No workgroup waits for another, so the launch needs no
// co-residency.
constexpr int kTries = 16;

__device__ inline double trial_scale(double alpha, int64_t ell, double gn2)
{
    const double beta = pow(alpha, (double)ell);
    return (gn2 > 0.0) ? -beta / sqrt(gn2) : 0.0;
}

// Loads x and g of one tile (origin i0, j0 of slice zz) with a one-voxel halo.
__device__ inline void load_pair(double (*tx)[HX], double (*tg)[HX], const double *x,
                                 const double *g, const GridDev &G, int zz, int i0, int j0)
{
    for (int q = threadIdx.x; q < HX * HY; q += kThreads) {
        const int ly = q / HX, lx = q - ly * HX;
        const int i = i0 + lx - 1, j = j0 + ly - 1;
        double a = 0.0, b = 0.0;
        if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) {
            const int64_t p = vaddr(G, i, j, zz);
            a = x[p];
            b = g[p];
        }
        tx[ly][lx] = a;
        tg[ly][lx] = b;
    }
    __syncthreads();
}

// This thread's voxel of the staged tile: adds m - eps of x (when with_x)
// and of z_t = x + s_t g for the tries t < cnt (z computed as the accepting
// update computes it).
__device__ inline void trial_terms(const double (*tx)[HX], const double (*tg)[HX],
                                   const double *sc, int cnt, const GridDev &G, int i0, int j0,
                                   double eps, bool with_x, double *acc, double &ax)
{
    const int li = threadIdx.x % TX, lj = threadIdx.x / TX;
    const int i = i0 + li, j = j0 + lj;
    if (i >= G.nx || j >= G.ny) return;
    const bool hx = i + 1 < G.nx, hy = j + 1 < G.ny;
    const double x00 = tx[lj + 1][li + 1], x10 = tx[lj + 1][li + 2], x01 = tx[lj + 2][li + 1];
    const double g00 = tg[lj + 1][li + 1], g10 = tg[lj + 1][li + 2], g01 = tg[lj + 2][li + 1];
    const double e2 = eps * eps;
    if (with_x) {
        const double dx = hx ? x10 - x00 : 0.0, dy = hy ? x01 - x00 : 0.0;
        ax += sqrt(dx * dx + dy * dy + e2) - eps;
    }
#pragma unroll
    for (int t = 0; t < kTries; t++) {
        if (t < cnt) {
            const double s = sc[t];
            const double z00 = fma(s, g00, x00);
            const double dx = hx ? fma(s, g10, x10) - z00 : 0.0;
            const double dy = hy ? fma(s, g01, x01) - z00 : 0.0;
            acc[t] += sqrt(dx * dx + dy * dy + e2) - eps;
        }
    }
}

// Sums v over the workgroup for kTries + 1 values at once (thread 0 holds
// the totals in out); a fixed order of additions.
__device__ inline void block_sums(const double *v, double *out)
{
    __shared__ double red[kThreads / 64][kTries + 1];
#pragma unroll
    for (int t = 0; t <= kTries; t++) {
        double a = v[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][t] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 0; t <= kTries; t++) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; w++) s += red[w][t];
            out[t] = s;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kThreads)
k_tv_check(GridDev G, const double *x, const double *g, const double *n2, double eps,
           double alpha, int32_t max_tries, int32_t k, int32_t n, SchedDev *sd, tvs_step_log *rec,
           double *part, uint32_t *ticket, double *dec)
{
    __shared__ double tx[HY][HX], tg[HY][HX];
    __shared__ double sc[kTries];
    __shared__ double tot[kTries + 1];
    __shared__ uint32_t last;
    const TileGrid TG = tile_grid(G);
    const int64_t ell0 = sd->ell;
    const double gn2 = *n2;
    const int cnt0 = max_tries < kTries ? max_tries : kTries;
    if (threadIdx.x < kTries) sc[threadIdx.x] = trial_scale(alpha, ell0 + threadIdx.x, gn2);
    double acc[kTries + 1];
#pragma unroll
    for (int t = 0; t <= kTries; t++) acc[t] = 0.0;
    for (int64_t T = blockIdx.x; T < TG.count(); T += gridDim.x) {
        int i0, j0, zz;
        TG.at(T, i0, j0, zz);
        __syncthreads();
        load_pair(tx, tg, x, g, G, zz, i0, j0);
        trial_terms(tx, tg, sc, cnt0, G, i0, j0, eps, true, acc, acc[kTries]);
    }
    block_sums(acc, tot);
    // partials of this workgroup; the last one to finish decides
    const uint32_t nwg = gridDim.x;
    const uint32_t wg = blockIdx.x;
    if (threadIdx.x == 0) {
        for (int t = 0; t <= kTries; t++) part[(int64_t)t * nwg + wg] = tot[t];
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        last = (old == nwg - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    // plain loads after the acquire above (every writer released its
    // partials before taking a ticket), kTries + 1 in flight per lane
    double v[kTries + 1];
#pragma unroll
    for (int t = 0; t <= kTries; t++) v[t] = 0.0;
    for (uint32_t q = threadIdx.x; q < nwg; q += kThreads) {
#pragma unroll
        for (int t = 0; t <= kTries; t++) v[t] += part[(int64_t)t * nwg + q];
    }
    block_sums(v, tot);
    const double phx = tot[kTries];
    int found = -1;
    for (int t = 0; t < cnt0; t++)
        if (found < 0 && tot[t] <= phx) found = t;
    double phz = found >= 0 ? tot[found] : 0.0;
    double s_acc = found >= 0 ? sc[found] : 0.0;
    int32_t tries = found >= 0 ? found + 1 : cnt0;
    // further rounds, this workgroup alone, over every tile
    for (int base = kTries; found < 0 && base < max_tries; base += kTries) {
        const int cnt = (max_tries - base < kTries) ? max_tries - base : kTries;
        __syncthreads();
        if (threadIdx.x < kTries) sc[threadIdx.x] = trial_scale(alpha, ell0 + base + threadIdx.x, gn2);
        double a[kTries + 1];
#pragma unroll
        for (int t = 0; t <= kTries; t++) a[t] = 0.0;
        for (int64_t T = 0; T < TG.count(); T++) {
            int i0, j0, zz;
            TG.at(T, i0, j0, zz);
            __syncthreads();
            load_pair(tx, tg, x, g, G, zz, i0, j0);
            trial_terms(tx, tg, sc, cnt, G, i0, j0, eps, false, a, a[kTries]);
        }
        block_sums(a, tot);
        for (int t = 0; t < cnt; t++)
            if (found < 0 && tot[t] <= phx) {
                found = t;
                phz = tot[t];
                s_acc = sc[t];
                tries = base + t + 1;
            }
        if (found < 0) tries = base + cnt;
    }
    if (threadIdx.x == 0) {
        dec[0] = s_acc;
        dec[1] = found >= 0 ? 1.0 : 0.0;
        sd->ell = ell0 + tries;
        tvs_step_log r;
        r.k = k;
        r.n = n;
        r.tries = tries;
        r.accepted = found >= 0 ? 1 : 0;
        r.ell_start = ell0;
        r.phi_x = phx;
        r.phi_z = phz;
        r.gnorm = sqrt(gn2);
        *rec = r;
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// x += s g with the scale the check accepted (nothing when it gave up).
__global__ void __launch_bounds__(kThreads) k_tv_apply(double *x, const double *g, int64_t n,
                                                       const double *dec)
{
    const double s = dec[0];
    if (dec[1] == 0.0 || s == 0.0) return;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads)
        x[p] = fma(s, g[p], x[p]);
}

// ell_k = rand(k, ell) on the device (the schedule of checked cycles): one
// SplitMix64 draw (Steele, Lea, Flood 2014), uniform in [k, ell], k when
// ell < k.
__global__ void k_sched_draw(SchedDev *sd, int64_t k)
{
    if (threadIdx.x != 0) return;
    const uint64_t st = sd->rng + 0x9E3779B97F4A7C15ull;
    sd->rng = st;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    const uint64_t u = z ^ (z >> 31);
    const int64_t ell = sd->ell;
    sd->ell = (ell < k) ? k : k + (int64_t)__umul64hi(u, (uint64_t)(ell - k) + 1u);
}

__global__ void k_sched_set(SchedDev *sd, int64_t ell, uint64_t rng)
{
    if (threadIdx.x != 0) return;
    sd->ell = ell;
    sd->rng = rng;
}

__global__ void __launch_bounds__(kThreads)
k_tv_step(double *x, const double *g, int64_t n, double beta, const double *n2)
{
    const double s = step_scale(beta, n2);
    if (s == 0.0) return;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads)
        x[p] = fma(s, g[p], x[p]);
}

// Image in: x-fastest float32 (the ABI order) to the float64 brick layout.
__global__ void __launch_bounds__(kThreads) k_widen(GridDev G, const float *src, double *dst)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads) {
        const int64_t i = p % G.nx, t = p / G.nx, j = t % G.ny, k = t / G.ny;
        dst[vaddr(G, i, j, k)] = (double)src[p];
    }
}

// Image out: brick layout to x-fastest float32.
__global__ void __launch_bounds__(kThreads) k_narrow(GridDev G, const double *src, float *dst)
{
    const int64_t n = (int64_t)G.nx * G.ny * G.nz;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads) {
        const int64_t i = p % G.nx, t = p / G.nx, j = t % G.ny, k = t / G.ny;
        dst[p] = (float)src[vaddr(G, i, j, k)];
    }
}

unsigned elem_grid(int64_t n)
{
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 4096) wgs = 4096;
    if (wgs < 1) wgs = 1;
    return (unsigned)wgs;
}

// workgroups of the TV kernels: one per tile, at most kMaxWgs
dim3 tv_grid(const GridDev &g)
{
    const int64_t tiles = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * g.nz;
    return dim3((unsigned)(tiles < kMaxWgs ? tiles : kMaxWgs));
}

}  // namespace

int64_t tv_num_parts(const GridDev &g)
{
    dim3 d = tv_grid(g);
    return (int64_t)d.x * d.y * d.z;
}

hipError_t launch_tv_grad(const GridDev &g, const double *x, double eps, const TvBuffers &t,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(k_tv_grad, tv_grid(g), dim3(kThreads), 0, stream, g, x, eps, t.g, t.part,
                       t.ticket, t.scal);
    return hipGetLastError();
}

hipError_t launch_tv_step(const GridDev &g, double *x, double beta, const TvBuffers &t,
                          hipStream_t stream)
{
    const int64_t n = padded_voxels(g);   // the padding's subgradient is zero
    hipLaunchKernelGGL(k_tv_step, dim3(elem_grid(n)), dim3(kThreads), 0, stream, x, t.g, n, beta,
                       t.scal);
    return hipGetLastError();
}

hipError_t launch_widen(const GridDev &g, const float *src, double *dst, hipStream_t stream)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_widen, dim3(elem_grid(n)), dim3(kThreads), 0, stream, g, src, dst);
    return hipGetLastError();
}

hipError_t launch_narrow(const GridDev &g, const double *src, float *dst, hipStream_t stream)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_narrow, dim3(elem_grid(n)), dim3(kThreads), 0, stream, g, src, dst);
    return hipGetLastError();
}

int64_t tv_check_parts(const GridDev &g) { return tv_num_parts(g) * (kTries + 1); }

hipError_t launch_tv_check(const GridDev &g, const double *x, double eps, double alpha,
                           int32_t max_tries, int32_t k, int32_t n, SchedDev *sd,
                           tvs_step_log *rec, const CheckBuffers &c, const TvBuffers &t,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(k_tv_check, tv_grid(g), dim3(kThreads), 0, stream, g, x,
                       (const double *)t.g, (const double *)t.scal, eps, alpha, max_tries, k, n,
                       sd, rec, c.part, c.ticket, c.dec);
    return hipGetLastError();
}

hipError_t launch_tv_apply(const GridDev &g, double *x, const TvBuffers &t, const CheckBuffers &c,
                           hipStream_t stream)
{
    const int64_t n = padded_voxels(g);
    hipLaunchKernelGGL(k_tv_apply, dim3(elem_grid(n)), dim3(kThreads), 0, stream, x,
                       (const double *)t.g, n, (const double *)c.dec);
    return hipGetLastError();
}

hipError_t launch_sched_draw(SchedDev *sd, int64_t k, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sched_draw, dim3(1), dim3(64), 0, stream, sd, k);
    return hipGetLastError();
}

hipError_t launch_sched_set(SchedDev *sd, int64_t ell, uint64_t rng, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sched_set, dim3(1), dim3(64), 0, stream, sd, ell, rng);
    return hipGetLastError();
}

}  // namespace tvs
