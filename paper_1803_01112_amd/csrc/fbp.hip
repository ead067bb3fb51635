// fbp.hip -- initial iterate on gfx950: filtered backprojection (FBP) of the
// binned histories and an in-slice median filter.
//
// The paper starts every reconstruction from an initial iterate to which a
// median filter of radius 2 has been applied (arXiv 1803.01112, Section
// V-A); it cites, and does not spell out, how that iterate is formed.
// Reading: textbook parallel-beam FBP.
//   binning      each history's straight line from entry to exit, at its
//                crossing of the depth u = 0 (the rotation axis): angle bin
//                round(phi / (2 pi / A)) mod A of the beam direction, lateral
//                bin of t in width tau (nt bins centred on t = 0), slice of
//                the height; a bin's projection is the mean WEPL of its
//                histories (0 when empty), the sums taken as 64-bit integers
//                in units of 2^-32 mm so that they do not depend on order;
//   filter       discrete Ram-Lak kernel h(0) = 1/(4 tau^2),
//                h(n odd) = -1/(n^2 pi^2 tau^2), h(n even) = 0, times tau;
//   backproject  linear interpolation, weight pi / A (A angles over 360
//                degrees see each line twice);
//   median       lower median of the (2r+1)^2 window clipped to the slice.
// Every step is one lane per output with a fixed order of summation, so
// the float64 results follow the written operations exactly.
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int kThreads = 256;
constexpr double kPi = 3.14159265358979323846;
constexpr double kFixed = 4294967296.0;   // 2^32

__global__ void __launch_bounds__(kThreads)
k_fbp_bin(GridDev g, HistDev H, int64_t n, int32_t A, double tau, int32_t nt,
          unsigned long long *sum, uint32_t *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double ex = H.s(kEx)[i], ey = H.s(kEy)[i], ez = H.s(kEz)[i];
    const double qx = H.s(kQx)[i], qy = H.s(kQy)[i], qz = H.s(kQz)[i];
    double ux = H.s(kUx)[i], uy = H.s(kUy)[i];
    const double nrm = sqrt(ux * ux + uy * uy);
    ux = ux / nrm;
    uy = uy / nrm;
    const double u0 = ex * ux + ey * uy, t0 = -ex * uy + ey * ux;
    const double u2 = qx * ux + qy * uy, t2 = -qx * uy + qy * ux;
    const double L = u2 - u0;
    if (!(L > 0.0)) return;
    const double f = (0.0 - u0) / L;
    const double tc = t0 + (t2 - t0) * f;
    const double vc = ez + (qz - ez) * f;
    const double phi = atan2(uy, ux);
    const double da = 2.0 * kPi / (double)A;
    int64_t a = (int64_t)floor(phi / da + 0.5);
    a %= A;
    if (a < 0) a += A;
    const double mm = floor(tc / tau + 0.5 * (double)nt);
    if (!(mm >= 0.0 && mm < (double)nt)) return;
    const double kk = floor((vc - g.oz) / g.vz);
    if (!(kk >= 0.0 && kk < (double)g.nz)) return;
    const int64_t b = (a * g.nz + (int64_t)kk) * nt + (int64_t)mm;
    atomicAdd(sum + b, (unsigned long long)(long long)llrint((double)H.s(kWepl)[i] * kFixed));
    atomicAdd(cnt + b, 1u);
}

__global__ void __launch_bounds__(kThreads)
k_fbp_mean(const unsigned long long *sum, const uint32_t *cnt, int64_t nb, double *p)
{
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= nb) return;
    p[b] = cnt[b] ? ((double)(long long)sum[b] / kFixed) / (double)cnt[b] : 0.0;
}

// q[r * nt + m] = tau * sum over s (ascending) of p[r * nt + s] h(m - s)
__global__ void __launch_bounds__(kThreads)
k_fbp_filter(const double *p, int64_t rows, int32_t nt, double tau, double *q)
{
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= rows * nt) return;
    const int64_t r = o / nt;
    const int32_t m = (int32_t)(o - r * nt);
    const double *pr = p + r * nt;
    double acc = 0.0;
    for (int32_t s = 0; s < nt; s++) {
        const int32_t d = m - s;
        double hv;
        if (d == 0) hv = 1.0 / (4.0 * tau * tau);
        else if (d % 2 != 0) hv = -1.0 / ((double)d * (double)d * kPi * kPi * tau * tau);
        else continue;
        acc += pr[s] * hv;
    }
    q[o] = tau * acc;
}

// x (x-fastest, float64) = pi / A * sum over angles of the interpolated
// filtered projection; cs[2a], cs[2a+1] = cos, sin of angle a (host table).
__global__ void __launch_bounds__(kThreads)
k_fbp_backproject(GridDev g, const double *q, const double *cs, int32_t A, double tau, int32_t nt,
                  int clip, double *x)
{
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    if (o >= nvox) return;
    const int64_t i = o % g.nx, j = (o / g.nx) % g.ny, k = o / ((int64_t)g.nx * g.ny);
    const double X = g.ox + ((double)i + 0.5) * g.vx;
    const double Y = g.oy + ((double)j + 0.5) * g.vy;
    double acc = 0.0;
    for (int32_t a = 0; a < A; a++) {
        const double t = -X * cs[2 * a + 1] + Y * cs[2 * a];
        const double sp = t / tau + 0.5 * (double)nt - 0.5;
        const double m0 = floor(sp);
        const double w = sp - m0;
        const double *row = q + ((int64_t)a * g.nz + k) * nt;
        const double v0 = (m0 >= 0.0 && m0 < (double)nt) ? row[(int64_t)m0] : 0.0;
        const double v1 = (m0 + 1.0 >= 0.0 && m0 + 1.0 < (double)nt) ? row[(int64_t)m0 + 1] : 0.0;
        acc += (1.0 - w) * v0 + w * v1;
    }
    double v = acc * (kPi / (double)A);
    if (clip && v < 0.0) v = 0.0;
    x[o] = v;
}

// Lower median of the (2R+1)^2 window clipped to the slice, by rank: the
// window value with fewer than (n+1)/2 smaller values and at least (n+1)/2
// values not larger (unrolled, so the window stays in registers).
template <int R>
__global__ void __launch_bounds__(kThreads)
k_median(GridDev g, const double *x, float *out)
{
    constexpr int W = 2 * R + 1;
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    if (o >= nvox) return;
    const int64_t i = o % g.nx, j = (o / g.nx) % g.ny, k = o / ((int64_t)g.nx * g.ny);
    double v[W * W];
    bool in[W * W];
    int n = 0;
#pragma unroll
    for (int dj = 0; dj < W; dj++)
#pragma unroll
        for (int di = 0; di < W; di++) {
            const int64_t ii = i + di - R, jj = j + dj - R;
            const bool ok = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny;
            in[dj * W + di] = ok;
            v[dj * W + di] = ok ? x[ii + g.nx * (jj + g.ny * k)] : 0.0;
            n += ok;
        }
    const int want = (n - 1) / 2;      // rank of the lower median (0-based)
    double med = 0.0;
#pragma unroll
    for (int c = 0; c < W * W; c++) {
        int lt = 0, le = 0;
#pragma unroll
        for (int d = 0; d < W * W; d++) {
            lt += in[d] && v[d] < v[c];
            le += in[d] && v[d] <= v[c];
        }
        if (in[c] && lt <= want && want < le) med = v[c];
    }
    out[o] = (float)med;
}

// cs[2a], cs[2a+1] = cos, sin of angle a * 2 pi / A, formed on the device
// (the allocation-free entry point takes no host table)
__global__ void __launch_bounds__(kThreads) k_fbp_angles(int32_t A, double *cs)
{
    const int32_t a = (int32_t)(blockIdx.x * kThreads + threadIdx.x);
    if (a >= A) return;
    const double phi = (double)a * (2.0 * kPi / (double)A);
    cs[2 * a] = cos(phi);
    cs[2 * a + 1] = sin(phi);
}

__global__ void __launch_bounds__(kThreads) k_narrow_abi(const double *x, int64_t n, float *out)
{
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o < n) out[o] = (float)x[o];
}

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kThreads - 1) / kThreads)); }

}  // namespace

hipError_t launch_fbp_bin(const GridDev &g, const HistDev &h, int64_t n, int32_t A, double tau,
                          int32_t nt, unsigned long long *sum, uint32_t *cnt, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fbp_bin, grid_for(n), dim3(kThreads), 0, stream, g, h, n, A, tau, nt, sum,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_fbp_mean(const unsigned long long *sum, const uint32_t *cnt, int64_t nb, double *p,
                           hipStream_t stream)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fbp_mean, grid_for(nb), dim3(kThreads), 0, stream, sum, cnt, nb, p);
    return hipGetLastError();
}

hipError_t launch_fbp_filter(const double *p, int64_t rows, int32_t nt, double tau, double *q,
                             hipStream_t stream)
{
    if (rows * nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fbp_filter, grid_for(rows * nt), dim3(kThreads), 0, stream, p, rows, nt,
                       tau, q);
    return hipGetLastError();
}

hipError_t launch_fbp_backproject(const GridDev &g, const double *q, const double *cs, int32_t A,
                                  double tau, int32_t nt, int clip, double *x, hipStream_t stream)
{
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_fbp_backproject, grid_for(nvox), dim3(kThreads), 0, stream, g, q, cs, A,
                       tau, nt, clip, x);
    return hipGetLastError();
}

hipError_t launch_fbp_angles(int32_t A, double *cs, hipStream_t stream)
{
    if (A <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fbp_angles, grid_for(A), dim3(kThreads), 0, stream, A, cs);
    return hipGetLastError();
}

hipError_t launch_median(const GridDev &g, const double *x, int radius, float *out,
                         hipStream_t stream)
{
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    switch (radius) {
    case 0: hipLaunchKernelGGL(k_narrow_abi, grid_for(nvox), dim3(kThreads), 0, stream, x, nvox, out); break;
    case 1: hipLaunchKernelGGL(k_median<1>, grid_for(nvox), dim3(kThreads), 0, stream, g, x, out); break;
    case 2: hipLaunchKernelGGL(k_median<2>, grid_for(nvox), dim3(kThreads), 0, stream, g, x, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tvs
