// tv.hip -- total variation, its subgradient and the normalised perturbation
// step on gfx950 (arXiv 1803.01112: phi = TV, "the sum of local variations
// over all voxels", Section IV; v = -grad phi / ||grad phi||, Appendix A).
//
// TV is taken per slice (2-D isotropic forward differences, zero difference
// past the last row/column): m_ij = sqrt(dx^2 + dy^2 + eps^2),
// phi = sum (m_ij - eps).  The subgradient at x_ij collects the terms of
// m_ij, m_(i-1)j and m_i(j-1); a term whose m is zero contributes zero.
//
// The image and the subgradient are float64 on the device: DROP increments
// with a small relaxation are tiny next to the RSP itself, and the
// subgradient only sees the direction of (dx, dy), so a float32 image would
// turn its rounding into order-one changes of v.  Each workgroup stages a
// 64x4 tile of one slice plus a one-voxel halo in LDS, evaluates the
// stencil, and writes a float64 partial sum.  The last workgroup to finish (ticket counter) adds
// the partials in a fixed order, so every reduction is deterministic and no
// host round trip is needed between the gradient and the update.
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int TX = 64, TY = 4, kThreads = TX * TY;
constexpr int HX = TX + 2, HY = TY + 2;

// Loads the tile of slice z (origin i0, j0) with a one-voxel halo.  With
// g != nullptr the staged values are z = x + s*g (the trial image of a
// checked step), computed exactly as the accepting update computes them.
__device__ inline void load_tile(double (*t)[HX], const double *x, const double *g, double s,
                                 const GridDev &G, int z, int i0, int j0)
{
    for (int q = threadIdx.x; q < HX * HY; q += kThreads) {
        int ly = q / HX, lx = q - ly * HX;
        int i = i0 + lx - 1, j = j0 + ly - 1;
        double v = 0.0;
        if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) {
            int64_t p = vaddr(G, i, j, z);
            v = x[p];
            if (g) v = fma(s, g[p], v);
        }
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
// in a fixed order into *out and re-arms the ticket.
__device__ inline void finish_reduction(double partial, double *part, uint32_t *ticket,
                                        double *out)
{
    __shared__ uint32_t last;
    const uint32_t nwg = gridDim.x * gridDim.y * gridDim.z;
    const uint32_t wg = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (threadIdx.x == 0) {
        part[wg] = partial;
        __threadfence();
        uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
        last = (old == nwg - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double v = 0.0;
    for (uint32_t q = threadIdx.x; q < nwg; q += kThreads)
        v += __hip_atomic_load(part + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double tot = block_sum(v);
    if (threadIdx.x == 0) {
        *out = tot;
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void __launch_bounds__(kThreads)
k_tv_grad(GridDev G, const double *x, double eps, double *gout, double *part, uint32_t *ticket,
          double *out)
{
    __shared__ double tile[HY][HX];
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    load_tile(tile, x, nullptr, 0.0, G, (int)blockIdx.z, i0, j0);
    const int i = i0 + (threadIdx.x % TX), j = j0 + (threadIdx.x / TX);
    double sq = 0.0;
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
        gout[vaddr(G, i, j, blockIdx.z)] = gv;
        sq = gv * gv;
    }
    finish_reduction(block_sum(sq), part, ticket, out);
}

__global__ void __launch_bounds__(kThreads)
k_tv_phi(GridDev G, const double *x, const double *g, double beta, const double *n2, double eps,
         double *part, uint32_t *ticket, double *out)
{
    __shared__ double tile[HY][HX];
    const double s = g ? step_scale(beta, n2) : 0.0;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    load_tile(tile, x, (s != 0.0) ? g : nullptr, s, G, (int)blockIdx.z, i0, j0);
    const int i = i0 + (threadIdx.x % TX), j = j0 + (threadIdx.x / TX);
    double v = 0.0;
    if (i < G.nx && j < G.ny) {
        Stencil S{tile, G.nx, G.ny, i0, j0, eps * eps};
        v = S.m(i, j) - eps;
    }
    finish_reduction(block_sum(v), part, ticket, out);
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

__global__ void __launch_bounds__(kThreads) k_fill_zero(float *p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads)
        p[q] = 0.0f;
}

unsigned elem_grid(int64_t n)
{
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 4096) wgs = 4096;
    if (wgs < 1) wgs = 1;
    return (unsigned)wgs;
}

dim3 tv_grid(const GridDev &g)
{
    return dim3((unsigned)((g.nx + TX - 1) / TX), (unsigned)((g.ny + TY - 1) / TY), (unsigned)g.nz);
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

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill_zero, dim3(elem_grid(n)), dim3(kThreads), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_tv_phi(const GridDev &g, const double *x, double beta, double eps,
                         const TvBuffers &t, hipStream_t stream)
{
    hipLaunchKernelGGL(k_tv_phi, tv_grid(g), dim3(kThreads), 0, stream, g, x,
                       (beta != 0.0) ? t.g : nullptr, beta, t.scal, eps, t.part, t.ticket,
                       t.scal + 1);
    return hipGetLastError();
}

}  // namespace tvs
