// csc.hip -- voxel-major form of the DROP blocks of a path store.
//
// DROP (arXiv 1803.01112, Section III-D) applies, per block of B rows,
// x_j += lambda * (sum over the block's entries at voxel j of r_i a_ij) / s_j.
// With the block's entries grouped by voxel (a compressed-sparse-column
// transpose of the block) the correction of voxel j is a short gather over
// its column, so the apply needs no atomics, visits each touched voxel once
// and sums in a fixed order (ascending row within the column): the sweep is
// deterministic.  Per block the store keeps
//   uvox[u]  (int32)  the block's distinct voxels, ascending,
//   ucol[u]  (uint32) start of voxel u's column among the block's entries,
//   cq[e]    (uint16) row (within the block) of column entry e,
//   cch[e]   (float32 / float16) its chord,
// with the column entries of block t stored at the same offsets as its row
// entries.  s_j is the column length.
//
// The transpose is built once, a batch of blocks at a time: count entries
// per (block, voxel), exclusive scans give each distinct voxel its rank and
// column start, rows then place their entries with a per-(block, voxel)
// cursor, and finally every column is sorted by row.
#include "device_common.hpp"
#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr int kThreads = 256;

// entries of the rows [r0, r1) (block-major batch starting at block b0)
__global__ void __launch_bounds__(kThreads)
k_csc_count(const int64_t *row_off, int64_t first, const int32_t *idx, int64_t r0, int64_t r1,
            int64_t block_size, int64_t b0, int64_t nvox, uint32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    for (int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 64; row < r1;
         row += (int64_t)gridDim.x * (kThreads / 64)) {
        const int64_t b = row / block_size - b0;
        const int64_t a = row_off[row - first], e = row_off[row - first + 1];
        for (int64_t k = a + lane; k < e; k += 64) atomicAdd(cnt + b * nvox + idx[k], 1u);
    }
}

__global__ void __launch_bounds__(kThreads)
k_csc_flags(const uint32_t *cnt, int64_t n, int32_t *flag)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads)
        flag[q] = cnt[q] > 0u ? 1 : 0;
}

__global__ void __launch_bounds__(kThreads)
k_csc_as_int(const uint32_t *cnt, int64_t n, int32_t *out)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads)
        out[q] = (int32_t)cnt[q];
}

// For every (block b, voxel j) present: its distinct-voxel record and the
// cursor (block-relative column start) used by the placement pass.
__global__ void __launch_bounds__(kThreads)
k_csc_emit(uint32_t *cnt, const int64_t *urank, const int64_t *cstart, int64_t nb, int64_t nvox,
           const int64_t *ubase, const int64_t *ebase, int32_t *uvox, uint32_t *ucol)
{
    const int64_t n = nb * nvox;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads) {
        if (cnt[q] == 0u) continue;
        const int64_t b = q / nvox, j = q - b * nvox;
        const int64_t u = urank[q] - urank[b * nvox];
        const int64_t start = cstart[q] - cstart[b * nvox];
        uvox[ubase[b] + u] = (int32_t)j;
        ucol[ubase[b] + u] = (uint32_t)start;
        (void)ebase;
        cnt[q] = (uint32_t)start;   // becomes the placement cursor
    }
}

template <typename CH>
__global__ void __launch_bounds__(kThreads)
k_csc_place(const int64_t *row_off, int64_t first, const int32_t *idx, const CH *chord,
            int64_t r0, int64_t r1, int64_t block_size, int64_t b0, int64_t nvox, uint32_t *cursor,
            const int64_t *ebase, uint16_t *cq, CH *cch)
{
    const int lane = threadIdx.x & 63;
    for (int64_t row = r0 + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 64; row < r1;
         row += (int64_t)gridDim.x * (kThreads / 64)) {
        const int64_t blk = row / block_size;
        const int64_t b = blk - b0;
        const uint16_t q = (uint16_t)(row - blk * block_size);
        const int64_t a = row_off[row - first], e = row_off[row - first + 1];
        for (int64_t k = a + lane; k < e; k += 64) {
            const uint32_t slot = atomicAdd(cursor + b * nvox + idx[k], 1u);
            cq[ebase[b] + slot] = q;
            cch[ebase[b] + slot] = chord[k];
        }
    }
}

// Sorts every column of the batch by row (insertion sort; columns are short).
template <typename CH>
__global__ void __launch_bounds__(kThreads)
k_csc_sort(const uint32_t *ucol, const int64_t *ubase, const int64_t *ucount, const int64_t *ebase,
           const int64_t *ecount, int64_t nb, uint16_t *cq, CH *cch)
{
    const int64_t b = blockIdx.y;
    if (b >= nb) return;
    const int64_t U = ucount[b];
    for (int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x; u < U;
         u += (int64_t)gridDim.x * kThreads) {
        const int64_t s = ucol[ubase[b] + u];
        const int64_t e = (u + 1 < U) ? (int64_t)ucol[ubase[b] + u + 1] : ecount[b];
        uint16_t *qq = cq + ebase[b];
        CH *cc = cch + ebase[b];
        for (int64_t i = s + 1; i < e; i++) {
            uint16_t kq = qq[i];
            CH kc = cc[i];
            int64_t m = i - 1;
            while (m >= s && qq[m] > kq) {
                qq[m + 1] = qq[m];
                cc[m + 1] = cc[m];
                m--;
            }
            qq[m + 1] = kq;
            cc[m + 1] = kc;
        }
    }
}

__global__ void k_csc_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst)
{
    for (int64_t b = threadIdx.x; b <= n; b += blockDim.x) dst[b] = src[b * stride];
}

unsigned grid_for(int64_t n)
{
    int64_t w = (n + kThreads - 1) / kThreads;
    if (w > 16384) w = 16384;
    if (w < 1) w = 1;
    return (unsigned)w;
}

}  // namespace

hipError_t csc_count(const RowSet &rs, int64_t r0, int64_t r1, int64_t block_size, int64_t b0,
                     int64_t nvox, uint32_t *cnt, hipStream_t st)
{
    const int64_t rows = r1 - r0;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csc_count, dim3(grid_for(rows * 64)), dim3(kThreads), 0, st, rs.row_off,
                       rs.first, rs.idx, r0, r1, block_size, b0, nvox, cnt);
    return hipGetLastError();
}

hipError_t csc_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_csc_pick, dim3(1), dim3(256), 0, st, src, stride, n, dst);
    return hipGetLastError();
}

hipError_t csc_flags(const uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_csc_flags, dim3(grid_for(n)), dim3(kThreads), 0, st, cnt, n, flag);
    return hipGetLastError();
}

hipError_t csc_as_int(const uint32_t *cnt, int64_t n, int32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_csc_as_int, dim3(grid_for(n)), dim3(kThreads), 0, st, cnt, n, out);
    return hipGetLastError();
}

hipError_t csc_emit(uint32_t *cnt, const int64_t *urank, const int64_t *cstart, int64_t nb,
                    int64_t nvox, const int64_t *ubase, const int64_t *ebase, int32_t *uvox,
                    uint32_t *ucol, hipStream_t st)
{
    hipLaunchKernelGGL(k_csc_emit, dim3(grid_for(nb * nvox)), dim3(kThreads), 0, st, cnt, urank,
                       cstart, nb, nvox, ubase, ebase, uvox, ucol);
    return hipGetLastError();
}

hipError_t csc_place(const RowSet &rs, int64_t r0, int64_t r1, int64_t block_size, int64_t b0,
                     int64_t nvox, uint32_t *cursor, const int64_t *ebase, uint16_t *cq,
                     float *cch32, __half *cch16, hipStream_t st)
{
    const int64_t rows = r1 - r0;
    if (rows <= 0) return hipSuccess;
    if (rs.chord16)
        hipLaunchKernelGGL(k_csc_place<__half>, dim3(grid_for(rows * 64)), dim3(kThreads), 0, st,
                           rs.row_off, rs.first, rs.idx, rs.chord16, r0, r1, block_size, b0, nvox,
                           cursor, ebase, cq, cch16);
    else
        hipLaunchKernelGGL(k_csc_place<float>, dim3(grid_for(rows * 64)), dim3(kThreads), 0, st,
                           rs.row_off, rs.first, rs.idx, rs.chord32, r0, r1, block_size, b0, nvox,
                           cursor, ebase, cq, cch32);
    return hipGetLastError();
}

hipError_t csc_sort(const uint32_t *ucol, const int64_t *ubase, const int64_t *ucount,
                    const int64_t *ebase, const int64_t *ecount, int64_t nb, int64_t max_u,
                    uint16_t *cq, float *cch32, __half *cch16, hipStream_t st)
{
    if (nb <= 0 || max_u <= 0) return hipSuccess;
    dim3 grid(grid_for(max_u) > 1024 ? 1024 : grid_for(max_u), (unsigned)nb);
    if (cch16)
        hipLaunchKernelGGL(k_csc_sort<__half>, grid, dim3(kThreads), 0, st, ucol, ubase, ucount,
                           ebase, ecount, nb, cq, cch16);
    else
        hipLaunchKernelGGL(k_csc_sort<float>, grid, dim3(kThreads), 0, st, ucol, ubase, ucount,
                           ebase, ecount, nb, cq, cch32);
    return hipGetLastError();
}

}  // namespace tvs
