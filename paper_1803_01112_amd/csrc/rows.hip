// rows.hip -- formation of the rows of the pCT linear system on gfx950.
//
// Each proton history gives one equation: the chord lengths of its most
// likely path (MLP) through the voxels, times the voxel RSPs, sum to its
// WEPL (arXiv 1803.01112, Section I).  One lane forms one row:
//   1. the MLP vertices at depths j*step along the beam axis, from the
//      Fermi-Eyges / Highland scattering moments of the entry->vertex and
//      vertex->exit slabs and the 2x2 Gaussian conditioning of the lateral
//      (t, dt/du) and vertical (v, dv/du) states on the entry and exit
//      measurements, all in float64;
//   2. a Siddon parametric walk of every polyline segment (crossings of the
//      integer grid planes merged in order, voxel of a piece taken at its
//      midpoint), merging consecutive pieces in the same voxel.
// Decisions that pick voxel indices are taken in float64; chords are
// rounded to float32 (or float16) only when written.  This file must be
// compiled with -ffp-contract=off so that no multiply-add is fused.
#include <type_traits>

#include "tvs_internal.hpp"

namespace tvs {
namespace {

constexpr double kE0 = 13.6;     // MeV, Highland constant
constexpr double kX0 = 360.8;    // mm, radiation length of water
constexpr int kThreads = 256;
__device__ const double kZero3[3] = {0.0, 0.0, 0.0};
// Row kernels: at least 2 wavefronts per SIMD (the two vertices a lane
// evaluates side by side need many VGPRs).  The tile-list kernel takes few
// enough to fit 3; its kRoom instance holds 2, leaving room for DROP waves.
constexpr int kRowWaves = 2;
// List entries staged per lane before they are written (LDS: 8 bytes each,
// 32 KB per 256-lane workgroup with float32 chords).
constexpr int kStage = 16;

__device__ inline double ipow(double base, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= base;
    return r;
}

// n! for n <= 9 (every use has a compile-time n after unrolling)
__device__ inline double fact(int n)
{
    constexpr double f[10] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0, 362880.0};
    return f[n];
}

// a / b, correctly rounded (the IEEE quotient bit for bit), from y = 1/b
// rounded to nearest: a * y corrected twice by its residual a - b q (exact
// in an FMA).  After the first correction the estimate lies within one ulp
// of a / b; from there one correction with a correctly rounded reciprocal
// gives the correctly rounded quotient (Markstein's theorem; it needs no
// underflow or overflow on the way, which holds for every quotient it is
// used for here).  Five float64 operations against the eleven, one of them a
// quarter-rate reciprocal, of a general division.
__device__ inline double div_rn(double a, double b, double y)
{
    double q = a * y;
    double r = fma(-q, b, a);
    q = fma(r, y, q);
    r = fma(-q, b, a);
    return fma(r, y, q);
}

// a / n for a small integer n known at compile time (after unrolling).
__device__ inline double div_int(double a, int n)
{
    if ((n & (n - 1)) == 0) return a / (double)n;     // power of two: exact multiply
    return div_rn(a, (double)n, 1.0 / (double)n);
}

// Natural logarithm of a positive, finite, normal x: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^21/21),
// s = (m - 1) / (m + 1), |s| <= 0.1716 (first omitted term below 2e-19).
// A fixed sequence of float64 operations (no library logarithm, whose last
// bit differs between math libraries), so the Highland factor, and with it
// every vertex, is the same double wherever the rows are formed.
__device__ inline double series_log(double x)
{
    int e = 0;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    return (double)e * 0.69314718055994530942 + 2.0 * s * p;
}

__device__ inline double highland(double depth, int log_term)
{
    double f = 1.0;
    if (log_term) f = 1.0 + 0.038 * series_log(div_rn(depth, kX0, 1.0 / kX0));
    return div_rn(kE0 * kE0 * f * f, kX0, 1.0 / kX0);
}

// 1/(beta^2 p^2) of a 200 MeV proton in water, per mm^k.
__device__ inline void power_coefs(int const_power, double b[6])
{
    b[0] = 7.457e-6;
    b[1] = 4.548e-8;
    b[2] = -5.777e-10;
    b[3] = 1.301e-11;
    b[4] = -9.228e-14;
    b[5] = 2.687e-16;
    if (const_power) b[1] = b[2] = b[3] = b[4] = b[5] = 0.0;
}

struct M2 { double a, b, c, d; };   // [[a, b], [c, d]]

__device__ inline M2 mul(const M2 &A, const M2 &B)
{
    return {A.a * B.a + A.b * B.c, A.a * B.b + A.b * B.d,
            A.c * B.a + A.d * B.c, A.c * B.b + A.d * B.d};
}
// Inverse as the adjugate times the reciprocal of the determinant.
__device__ inline M2 inv(const M2 &A)
{
    const double det = A.a * A.d - A.b * A.c;
    const double r = 1.0 / det;
    return {A.d * r, -A.b * r, -A.c * r, A.a * r};
}
__device__ inline void mvec(const M2 &A, double x0, double x1, double &y0, double &y1)
{
    double r0 = A.a * x0 + A.b * x1;
    double r1 = A.c * x0 + A.d * x1;
    y0 = r0;
    y1 = r1;
}

// Row emission state: consecutive pieces in one voxel merge into one entry.
// Entries also group into segments: maximal runs of consecutive entries in
// one image tile.  Modes:
//   kCount    counts entries and segments;
//   kSeg      reserves each segment's place in its (block, tile) list;
//   kRowMajor writes the entries in walk order (tvs_debug_rows);
//   kTiled    writes every entry into its tile list at the reserved place.
//   kHull     counts each voxel of a straight line once in in_cnt / out_cnt.
enum EmitMode { kCount = 0, kSeg = 1, kRowMajor = 2, kTiled = 3, kHull = 4 };

// A chord as an unsigned multiple of the fixed-point store's unit (1 / qinv
// mm), rounded to nearest; the unit is the longest chord of the loaded rows
// / qmax, rounded up, so the clamp only catches rounding at the top.
__device__ inline uint32_t encode_fixed(double len, double qinv, uint32_t qmax)
{
    const double u = rint(len * qinv);
    return u > (double)qmax ? qmax : (uint32_t)u;
}

template <int MODE, typename CH>
struct Emit {
    int32_t cur = -1;
    double cur_len = 0.0;
    double norm2 = 0.0;
    int64_t n = 0;               // entries emitted
    int32_t nseg = 0;            // segments opened
    int32_t tile = -1;           // tile of the open segment
    uint32_t seg_len = 0;        // kSeg: entries of the open segment
    int32_t *idx = nullptr;      // kRowMajor
    CH *chord = nullptr;         // kRowMajor, kTiled
    double qinv = 0.0;           // kTiled, fixed-point chords: units per mm
    uint32_t qmax = 0;           // kTiled, fixed-point chords: largest code
    uint32_t qshift = 31;        // kTiled, fixed-point chords: tag bit of the code's bit 16
    double maxc = 0.0;           // kSeg: longest entry of the row
    uint32_t *in_cnt = nullptr;  // kHull: this line counts (space modelling) into in_cnt,
    uint32_t *out_cnt = nullptr; //        carves (space carving) into out_cnt,
    uint32_t in_sat = 0;         //        each count only up to the value past which no
    uint32_t out_sat = 0;        //        further line changes the voxel's decision
    uint32_t *btc = nullptr;     // kSeg: list lengths of this row's block
    uint64_t *segtab = nullptr;  // kSeg: (tile, place) of this row's segments
    const int64_t *segdst = nullptr;  // kTiled: first entry of this row's segments
    uint32_t *meta = nullptr;    // kTiled
    int64_t base = 0, dst = 0;   // kTiled
    uint32_t q = 0;              // kTiled: row within its block
    // kTiled: entries of the open segment are staged in this lane's LDS slots
    // and written out together when the segment closes or the slots fill
    // (list places dst - ns .. dst - 1), so that every list line is written
    // in one burst instead of one 4-byte store per walk step
    int ns = 0;
    // kSeg, kTiled: guards against a walk that disagrees with the load-time
    // count (segments of this row, entries of the buffer); a disagreement
    // writes nothing and raises *err
    int32_t seg_cap = 0;
    int64_t cap = 0;
    uint32_t *err = nullptr;
    bool ok = true;

    __device__ inline void close_seg()
    {
        if constexpr (MODE == kSeg) {
            if (seg_len && ok) {
                const uint32_t pos = atomicAdd(btc + tile, seg_len);
                segtab[nseg - 1] = ((uint64_t)(uint32_t)tile << 32) | pos;
            }
            seg_len = 0;
        }
    }

    __device__ inline void bad()
    {
        if (ok) atomicOr(err, 1u);
        ok = false;
    }

    __device__ inline void flush()
    {
        if (cur < 0) return;
        if constexpr (MODE == kHull) {
            // a count read below its true value (another line's add not yet
            // seen) only costs an add; one at or past the saturation value
            // has reached it for good (counts only grow)
            if (in_cnt && __hip_atomic_load(in_cnt + cur, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < in_sat)
                atomicAdd(in_cnt + cur, 1u);
            if (out_cnt && __hip_atomic_load(out_cnt + cur, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) < out_sat)
                atomicAdd(out_cnt + cur, 1u);
            cur = -1;
            cur_len = 0.0;
            n++;
            return;
        }
        const int32_t t = cur >> kTileShift;
        if (t != tile) {
            close_seg();
            if constexpr (MODE == kTiled) drain();
            tile = t;
            if constexpr (MODE == kSeg || MODE == kTiled) {
                if (nseg >= seg_cap) bad();
            }
            if constexpr (MODE == kTiled) {
                if (ok) dst = segdst[nseg] - base;
            }
            nseg++;
        }
        if constexpr (MODE == kRowMajor) {
            idx[n] = cur;
            if constexpr (sizeof(CH) == 4) chord[n] = (float)cur_len;
            else chord[n] = __float2half((float)cur_len);
        }
        if constexpr (MODE == kTiled) {
            if (ok && (dst < 0 || dst >= cap)) bad();
            if (ok) {
                const int slot = ns * kThreads + (int)threadIdx.x;
                uint32_t tag = (uint32_t)(cur & (kTileWords - 1)) | (q << kTileShift);
                if constexpr (sizeof(CH) == 4) {
                    stage_chord()[slot] = (float)cur_len;
                } else if constexpr (std::is_same<CH, uint16_t>::value) {
                    const uint32_t code = encode_fixed(cur_len, qinv, qmax);
                    tag |= (code >> 16) << qshift;
                    stage_chord()[slot] = (uint16_t)(code & 0xffffu);
                } else {
                    stage_chord()[slot] = __float2half((float)cur_len);
                }
                stage_meta()[slot] = tag;
                dst++;
                if (++ns == kStage) drain();
            }
        }
        if constexpr (MODE == kSeg) {
            seg_len++;
            maxc = fmax(maxc, cur_len);
        }
        norm2 += cur_len * cur_len;
        n++;
        cur = -1;
        cur_len = 0.0;
    }

    // kTiled staging slots: slot k of lane l at k * kThreads + l (LDS)
    static __device__ inline uint32_t *stage_meta()
    {
        __shared__ uint32_t sm[kStage * kThreads];
        return sm;
    }
    static __device__ inline CH *stage_chord()
    {
        __shared__ CH sc[kStage * kThreads];
        return sc;
    }

    // kTiled: writes the staged entries to their consecutive list places
    __device__ inline void drain()
    {
        const int64_t d0 = dst - ns;
        for (int k = 0; k < ns; k++) {
            const int slot = k * kThreads + (int)threadIdx.x;
            meta[d0 + k] = stage_meta()[slot];
            chord[d0 + k] = stage_chord()[slot];
        }
        ns = 0;
    }

    __device__ inline void finish()
    {
        flush();
        close_seg();
        if constexpr (MODE == kTiled) drain();
    }
};

// Grid coordinates (p - o) / v of a point (quotients correctly rounded).
__device__ inline void to_grid(const GridDev &g, const double p[3], double gp[3])
{
    gp[0] = div_rn(p[0] - g.ox, g.vx, g.rvx);
    gp[1] = div_rn(p[1] - g.oy, g.vy, g.rvy);
    gp[2] = div_rn(p[2] - g.oz, g.vz, g.rvz);
}

// Walks segment q0 -> q1 given both end points and their grid coordinates
// g0, g1 (each point's coordinates are computed once and shared by the two
// segments that meet there).
template <int MODE, typename CH>
__device__ void walk_segment(const GridDev &g, const double q0[3], const double q1[3],
                             const double g0[3], const double g1[3], Emit<MODE, CH> &e)
{
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    double dg[3];
    for (int a = 0; a < 3; a++) dg[a] = g1[a] - g0[a];
    double dx = q1[0] - q0[0], dy = q1[1] - q0[1], dz = q1[2] - q0[2];
    double len = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(len > 0.0)) return;

    // Per axis: next integer plane in the direction of travel, how many
    // planes inside [0, n] remain after it, and its crossing parameter
    // tau = (m - g0) / dg.  An axis with no plane left has tau = 2, past the
    // segment's end, so it is never the nearest crossing.
    double mnext[3], tnext[3];
    int rem[3];
    for (int a = 0; a < 3; a++) {
        mnext[a] = 0.0;
        tnext[a] = 2.0;
        rem[a] = 0;
        if (dg[a] == 0.0) continue;
        double lo = (g0[a] < g1[a]) ? g0[a] : g1[a];
        double hi = (g0[a] < g1[a]) ? g1[a] : g0[a];
        double mlo = floor(lo) + 1.0;
        double mhi = ceil(hi) - 1.0;
        if (mlo < 0.0) mlo = 0.0;
        if (mhi > (double)n[a]) mhi = (double)n[a];
        if (mlo > mhi) continue;
        mnext[a] = (dg[a] > 0.0) ? mlo : mhi;
        rem[a] = (int)(mhi - mlo);
        tnext[a] = (mnext[a] - g0[a]) / dg[a];
    }

    double prev = 0.0;
    for (;;) {
        double tb = 1.0;
        for (int a = 0; a < 3; a++)
            if (tnext[a] < tb) tb = tnext[a];
        if (tb > prev) {
            double ta = prev;
            prev = tb;
            double tm = (ta + tb) * 0.5;
            double c[3];
            bool inside = true;
            for (int a = 0; a < 3; a++) {
                c[a] = floor(g0[a] + tm * dg[a]);
                inside = inside && !(c[a] < 0.0 || c[a] >= (double)n[a]);
            }
            if (inside) {
                int32_t lin = vaddr32(g, (int32_t)c[0], (int32_t)c[1], (int32_t)c[2]);
                double clen = (tb - ta) * len;
                if (lin == e.cur) {
                    e.cur_len += clen;
                } else {
                    e.flush();
                    e.cur = lin;
                    e.cur_len = clen;
                }
            }
        }
        if (tb >= 1.0) break;
        for (int a = 0; a < 3; a++) {
            if (tnext[a] == tb) {
                if (rem[a] == 0) {
                    tnext[a] = 2.0;
                } else {
                    rem[a]--;
                    mnext[a] += (dg[a] > 0.0) ? 1.0 : -1.0;
                    tnext[a] = (mnext[a] - g0[a]) / dg[a];
                }
            }
        }
    }
}

// Inverse covariance of the entry-side slab at depth d1, (Sigma_1(d1))^-1,
// as {a, b, d} of the symmetric 2x2 matrix [[a, b], [b, d]].  It depends on
// the depth only, so a context computes it once per vertex depth j * step
// (k_mlp_table) and every row reads it from that table.
__device__ inline void entry_sigma_inv(double d1, const MlpCfg &m, double s[3])
{
    double b[6];
    power_coefs(m.const_power, b);
    double i1[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int mm = 0; mm < 3; mm++) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const double beta = fact(mm) * fact(k) / fact(mm + k + 1);
            i1[mm] += b[k] * ipow(d1, mm + k + 1) * beta;
        }
    }
    double A1 = highland(d1, m.log_term);
    M2 S1 = {A1 * i1[2], A1 * i1[1], A1 * i1[1], A1 * i1[0]};
    M2 S1i = inv(S1);
    s[0] = S1i.a;
    s[1] = S1i.b;   // equals S1i.c: S1 is symmetric
    s[2] = S1i.d;
}

// MLP of history i and the Siddon walk of its polyline.
template <int MODE, typename CH>
__device__ void form_row(const GridDev &g, const HistDev &H, const MlpCfg &m, int64_t i,
                         Emit<MODE, CH> &e)
{
    double ex = H.s(kEx)[i], ey = H.s(kEy)[i], ez = H.s(kEz)[i];
    double qx = H.s(kQx)[i], qy = H.s(kQy)[i], qz = H.s(kQz)[i];
    double eth = H.s(kEth)[i], eps = H.s(kEps)[i], qth = H.s(kQth)[i], qps = H.s(kQps)[i];
    double ux = H.s(kUx)[i], uy = H.s(kUy)[i];
    double nrm = sqrt(ux * ux + uy * uy);
    ux = ux / nrm;
    uy = uy / nrm;

    double u0 = ex * ux + ey * uy, t0 = -ex * uy + ey * ux, v0 = ez;
    double u2 = qx * ux + qy * uy, t2 = -qx * uy + qy * ux, v2 = qz;
    double L = u2 - u0;
    if (!(L > 0.0)) return;
    double Jd = ceil(L / m.step);
    int64_t J = (Jd < 1.0) ? 1 : (int64_t)Jd;

    double b[6];
    power_coefs(m.const_power, b);
    // Exit-side expansion P(L - s) = sum_k c_k s^k.
    double c[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double acc = 0.0;
#pragma unroll
        for (int q = k; q < 6; q++) {
            const double binom = fact(q) / (fact(k) * fact(q - k));
            acc += b[q] * binom * ipow(L, q - k);
        }
        c[k] = (k % 2) ? -acc : acc;
    }

    bool miss = false;
    // MLP vertex j (1 <= j < J); the table index is clamped and a depth past
    // the table only noted, so that the body has no branch and two vertices
    // can be evaluated side by side
    auto vertex = [&](int64_t j, double p[3]) {
        double d1 = (double)j * m.step;
        double d2 = L - d1;
        // (the table covers every depth of the loaded histories, their
        // vertex counts bound it; a depth past it raises the consistency
        // flag, and an empty table is never indexed)
        const bool in_tab = j < m.nj;
        miss |= !in_tab;
        const double *tab = m.nj > 0 ? m.s1i + 3 * (in_tab ? j : m.nj - 1) : kZero3;
        double s1[3] = {tab[0], tab[1], tab[2]};
        // integral_0^d2 s^(mm+k) ds = d2^n / n, n = mm + k + 1 (powers of
        // d2 as running products, which equal repeated multiplication)
        double pw = 1.0, q[9];
#pragma unroll
        for (int n = 1; n <= 8; n++) {
            pw = pw * d2;
            q[n] = div_int(pw, n);
        }
        double j2[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int mm = 0; mm < 3; mm++)
#pragma unroll
            for (int k = 0; k < 6; k++)
                j2[mm] += c[k] * q[mm + k + 1];
        double A2 = highland(d2, m.log_term);
        M2 S2 = {A2 * j2[2], A2 * j2[1], A2 * j2[1], A2 * j2[0]};
        M2 R0 = {1.0, d1, 0.0, 1.0};
        M2 R1 = {1.0, d2, 0.0, 1.0};
        M2 S1i = {s1[0], s1[1], s1[1], s1[2]};
        M2 S2i = inv(S2);
        M2 R1t = {R1.a, R1.c, R1.b, R1.d};
        M2 T = mul(R1t, S2i);
        M2 T2 = mul(T, R1);
        M2 M = {S1i.a + T2.a, S1i.b + T2.b, S1i.c + T2.c, S1i.d + T2.d};
        M2 Mi = inv(M);
        double y1t, y1v;
        {
            double a0, a1, p0, p1, q0, q1, r0, r1, y0_, y1_;
            mvec(R0, t0, eth, a0, a1);
            mvec(S1i, a0, a1, p0, p1);
            mvec(T, t2, qth, q0, q1);
            r0 = p0 + q0;
            r1 = p1 + q1;
            mvec(Mi, r0, r1, y0_, y1_);
            y1t = y0_;
        }
        {
            double a0, a1, p0, p1, q0, q1, r0, r1, y0_, y1_;
            mvec(R0, v0, eps, a0, a1);
            mvec(S1i, a0, a1, p0, p1);
            mvec(T, v2, qps, q0, q1);
            r0 = p0 + q0;
            r1 = p1 + q1;
            mvec(Mi, r0, r1, y0_, y1_);
            y1v = y0_;
        }
        double u = u0 + d1;
        p[0] = u * ux - y1t * uy;
        p[1] = u * uy + y1t * ux;
        p[2] = y1v;
    };

    double prevp[3] = {ex, ey, ez};
    double prevg[3];
    to_grid(g, prevp, prevg);
    int64_t j = 1;
    for (; j + 1 < J; j += 2) {
        double pa[3], pb[3], ga[3], gb[3];
        vertex(j, pa);
        vertex(j + 1, pb);
        to_grid(g, pa, ga);
        to_grid(g, pb, gb);
        walk_segment<MODE, CH>(g, prevp, pa, prevg, ga, e);
        walk_segment<MODE, CH>(g, pa, pb, ga, gb, e);
        for (int a = 0; a < 3; a++) {
            prevp[a] = pb[a];
            prevg[a] = gb[a];
        }
    }
    if (j < J) {
        double p[3], pg[3];
        vertex(j, p);
        to_grid(g, p, pg);
        walk_segment<MODE, CH>(g, prevp, p, prevg, pg, e);
        for (int a = 0; a < 3; a++) {
            prevp[a] = p[a];
            prevg[a] = pg[a];
        }
    }
    if (miss && m.err) atomicOr(m.err, 1u);
    double last[3] = {qx, qy, qz};
    double lastg[3];
    to_grid(g, last, lastg);
    walk_segment<MODE, CH>(g, prevp, last, prevg, lastg, e);
}

__global__ void __launch_bounds__(kThreads) k_mlp_table(MlpCfg m, int64_t nj, double *tab)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nj) return;
    double s[3] = {0.0, 0.0, 0.0};
    if (j > 0) entry_sigma_inv((double)j * m.step, m, s);
    tab[3 * j] = s[0];
    tab[3 * j + 1] = s[1];
    tab[3 * j + 2] = s[2];
}

__global__ void __launch_bounds__(kThreads, kRowWaves)
k_rows_count(GridDev g, HistDev H, MlpCfg m, int64_t first, int64_t n, int32_t *nnz, int32_t *nseg)
{
    int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= n) return;
    Emit<kCount, float> e;
    form_row<kCount, float>(g, H, m, first + q, e);
    e.finish();
    nnz[q] = (int32_t)e.n;
    if (nseg) nseg[q] = (int32_t)e.nseg;
}

__global__ void __launch_bounds__(kThreads, kRowWaves)
k_rows_seg(GridDev g, HistDev H, MlpCfg m, int64_t n, int64_t B, int64_t ntiles,
           const int64_t *seg_off, uint32_t *btc, uint64_t *segtab, uint32_t *err,
           uint32_t *chmax, const int32_t *order)
{
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t bits = 0u;
    if (i < n) {
        if (order) i = order[i];
        Emit<kSeg, float> e;
        e.btc = btc + (i / B) * ntiles;
        e.segtab = segtab + seg_off[i];
        e.seg_cap = (int32_t)(seg_off[i + 1] - seg_off[i]);
        e.err = err;
        form_row<kSeg, float>(g, H, m, i, e);
        e.finish();
        // longest chord as float32 bits, rounded up (non-negative floats
        // order as their bit patterns)
        float mf = (float)e.maxc;
        if ((double)mf < e.maxc) mf = nextafterf(mf, INFINITY);
        bits = __float_as_uint(mf);
    }
    // the wavefront's maximum (every lane takes part), one atomic per wavefront
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(bits, d, 64);
        bits = o > bits ? o : bits;
    }
    if ((threadIdx.x & 63) == 0 && chmax && bits) atomicMax(chmax, bits);
}

__global__ void __launch_bounds__(kThreads)
k_seg_dest(int64_t n, int64_t B, int64_t ntiles, const int64_t *seg_off, const int64_t *bt_off,
           const int32_t *slot_of, int64_t nslots, uint64_t *segtab, uint32_t *err)
{
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t *bto = bt_off + (i / B) * nslots;
    for (int64_t s = seg_off[i]; s < seg_off[i + 1]; s++) {
        const uint64_t v = segtab[s];
        const int64_t T = (int64_t)(v >> 32);
        const int32_t slot = T < ntiles ? slot_of[T] : -1;
        if (slot < 0) {
            atomicOr(err, 1u);
            segtab[s] = 0;
            continue;
        }
        segtab[s] = (uint64_t)(bto[slot] + (int64_t)(v & 0xffffffffull));
    }
}

// kRoom: the kernel takes at least 171 VGPRs (176 allocated: the empty asm
// below claims v170), so that a SIMD holds two of its waves and four 40-VGPR
// DROP waves beside them; otherwise it fits three waves per SIMD, and a DROP
// step finds no room on a SIMD that holds three.
template <typename CH, bool kRoom>
__global__ void __launch_bounds__(kThreads, kRowWaves)
k_rows_fill_tiled(GridDev g, HistDev H, MlpCfg m, TileFill f, CH *chord)
{
    if constexpr (kRoom) asm volatile("" ::: "v170");
    // grid-stride: the grid may be held below the device's capacity so that
    // the DROP launches running beside it always find free slots
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < f.n;
         q += (int64_t)gridDim.x * kThreads) {
        const int64_t i = f.order ? (int64_t)f.order[f.first + q] : f.first + q;
        Emit<kTiled, CH> e;
        e.segdst = f.segdst + f.seg_off[i];
        e.seg_cap = (int32_t)(f.seg_off[i + 1] - f.seg_off[i]);
        e.cap = f.cap;
        e.err = f.err;
        e.meta = f.meta;
        e.chord = chord;
        e.base = f.base;
        e.qinv = f.qinv;
        e.qmax = f.qmax;
        e.qshift = f.qshift;
        e.q = (uint32_t)(i % f.B);
        form_row<kTiled, CH>(g, H, m, i, e);
        e.finish();
        f.norm2[i] = (float)e.norm2;
    }
}

__global__ void __launch_bounds__(kThreads, kRowWaves)
k_rows_fill(GridDev g, HistDev H, MlpCfg m, int64_t first, int64_t n, const int64_t *row_off,
            int64_t base, int32_t *idx, float *chord, float *norm2)
{
    int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= n) return;
    Emit<kRowMajor, float> e;
    int64_t off = row_off[q] - base;
    e.idx = idx + off;
    e.chord = chord + off;
    form_row<kRowMajor, float>(g, H, m, first + q, e);
    e.finish();
    norm2[q] = (float)e.norm2;
}

__global__ void __launch_bounds__(kThreads)
k_validate(HistDev H, int64_t n, double step, uint32_t *bad, uint32_t *jmax)
{
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    bool ok = true;
    for (int q = 0; q < 13; q++) {
        float v = H.s(q)[i];
        if (!isfinite(v) || fabsf(v) > 1.0e6f) ok = false;
    }
    if (ok) {
        double ux = H.s(kUx)[i], uy = H.s(kUy)[i];
        double nn = ux * ux + uy * uy;
        if (!(nn >= 1.0e-12)) {
            ok = false;
        } else {
            double nrm = sqrt(nn);
            double L = ((double)H.s(kQx)[i] - (double)H.s(kEx)[i]) * (ux / nrm) +
                       ((double)H.s(kQy)[i] - (double)H.s(kEy)[i]) * (uy / nrm);
            if (L / step > 1048576.0) ok = false;
            else if (L > 0.0) atomicMax(jmax, (uint32_t)ceil(L / step) + 2u);
        }
    }
    if (!ok) atomicAdd(bad, 1u);
}

// Hull detection: every history's straight line from its entry to its exit
// point, walked like a row segment; a line whose WEPL reaches wepl_in counts
// its voxels (space modelling), one whose WEPL is below wepl_out carves them
// (space carving).  One lane per history; the counters are in the tiled
// layout and saturate at in_sat / out_sat (min_in and max_out + 1): past
// them no further line changes a decision, and most adds are skipped.
__global__ void __launch_bounds__(kThreads)
k_hull_counts(GridDev g, HistDev H, int64_t n, double wepl_in, double wepl_out, uint32_t *in_cnt,
              uint32_t *out_cnt, uint32_t in_sat, uint32_t out_sat)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double w = H.s(kWepl)[i];
    const bool in = w >= wepl_in, out = w < wepl_out;
    if (!in && !out) return;
    const double p0[3] = {H.s(kEx)[i], H.s(kEy)[i], H.s(kEz)[i]};
    const double p1[3] = {H.s(kQx)[i], H.s(kQy)[i], H.s(kQz)[i]};
    double g0[3], g1[3];
    to_grid(g, p0, g0);
    to_grid(g, p1, g1);
    Emit<kHull, float> e;
    e.in_cnt = in ? in_cnt : nullptr;
    e.out_cnt = out ? out_cnt : nullptr;
    e.in_sat = in_sat;
    e.out_sat = out_sat;
    walk_segment<kHull, float>(g, p0, p1, g0, g1, e);
    e.flush();
}

// hull[p] (x-fastest) = in_cnt >= min_in and out_cnt <= max_out; with mask,
// the image x (tiled layout) is multiplied by the hull.
__global__ void __launch_bounds__(kThreads)
k_hull_decide(GridDev g, const uint32_t *in_cnt, const uint32_t *out_cnt, uint32_t min_in,
              uint32_t max_out, uint8_t *hull, double *mask)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kThreads) {
        const int64_t ii = p % g.nx, t = p / g.nx, jj = t % g.ny, kk = t / g.ny;
        const int64_t a = vaddr(g, ii, jj, kk);
        const bool inside = in_cnt[a] >= min_in && out_cnt[a] <= max_out;
        hull[p] = inside ? 1u : 0u;
        if (mask && !inside) mask[a] = 0.0;
    }
}

// dst[b] = src[b * stride] for b = 0 .. n - 1
__global__ void __launch_bounds__(kThreads)
k_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst)
{
    for (int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x; b < n;
         b += (int64_t)gridDim.x * kThreads)
        dst[b] = src[b * stride];
}

// ---------------------------------------------------------------- scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t warp_sums[kThreads / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) warp_sums[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int q = 0; q < kThreads / 64; q++) {
        if (q < w) before += warp_sums[q];
        all += warp_sums[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void __launch_bounds__(kThreads)
k_scan_tiles(const int32_t *cnt, int64_t n, int64_t *tile_sum)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        if (i < n) s += cnt[i];
    }
    int64_t total;
    block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads)
k_scan_partials(int64_t *tile_sum, int64_t ntiles)
{
    // Single workgroup: exclusive scan of the tile sums in place, in chunks.
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kThreads) {
        int64_t i = base + threadIdx.x;
        int64_t v = (i < ntiles) ? tile_sum[i] : 0;
        int64_t total;
        int64_t ex = block_exclusive_scan(v, &total);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ void __launch_bounds__(kThreads)
k_scan_write(const int32_t *cnt, int64_t n, const int64_t *tile_off, int64_t ntiles, int64_t *off)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        v[q] = (i < n) ? (int64_t)cnt[i] : 0;
        s += v[q];
    }
    int64_t total;
    int64_t ex = block_exclusive_scan(s, &total) + tile_off[blockIdx.x];
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        if (i < n) off[i] = ex;
        ex += v[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = tile_off[ntiles];
}

}  // namespace

hipError_t launch_rows_count(const GridDev &g, const HistDev &h, const MlpCfg &m, int64_t first,
                             int64_t n, int32_t *nnz, int32_t *nseg, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_rows_count, grid, dim3(kThreads), 0, stream, g, h, m, first, n, nnz, nseg);
    return hipGetLastError();
}

hipError_t launch_rows_seg(const GridDev &g, const HistDev &h, const MlpCfg &m, int64_t n,
                           int64_t B, const int64_t *seg_off, uint32_t *btc, uint64_t *segtab,
                           uint32_t *err, uint32_t *chmax, const int32_t *order,
                           hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_rows_seg, grid, dim3(kThreads), 0, stream, g, h, m, n, B, num_tiles(g),
                       seg_off, btc, segtab, err, chmax, order);
    return hipGetLastError();
}

hipError_t launch_seg_dest(const GridDev &g, int64_t n, int64_t B, const int64_t *seg_off,
                           const int64_t *bt_off, const int32_t *slot_of, int64_t nslots,
                           uint64_t *segtab, uint32_t *err, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_seg_dest, grid, dim3(kThreads), 0, stream, n, B, num_tiles(g), seg_off,
                       bt_off, slot_of, nslots, segtab, err);
    return hipGetLastError();
}

hipError_t launch_rows_fill_tiled(const GridDev &g, const HistDev &h, const MlpCfg &m,
                                  const TileFill &f, hipStream_t stream)
{
    if (f.n <= 0) return hipSuccess;
    int64_t wgs = (f.n + kThreads - 1) / kThreads;
    if (f.max_wgs > 0 && wgs > f.max_wgs) wgs = f.max_wgs;
    dim3 grid((unsigned)wgs);
    if (f.chq)
        hipLaunchKernelGGL((k_rows_fill_tiled<uint16_t, false>), grid, dim3(kThreads), 0, stream,
                           g, h, m, f, f.chq);
    else if (f.ch16)
        hipLaunchKernelGGL((k_rows_fill_tiled<__half, false>), grid, dim3(kThreads), 0, stream, g,
                           h, m, f, f.ch16);
    else if (f.room)
        hipLaunchKernelGGL((k_rows_fill_tiled<float, true>), grid, dim3(kThreads), 0, stream, g, h,
                           m, f, f.ch32);
    else
        hipLaunchKernelGGL((k_rows_fill_tiled<float, false>), grid, dim3(kThreads), 0, stream, g,
                           h, m, f, f.ch32);
    return hipGetLastError();
}

hipError_t launch_rows_fill(const GridDev &g, const HistDev &h, const MlpCfg &m, const RowSet &rs,
                            hipStream_t stream)
{
    if (rs.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((rs.n + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_rows_fill, grid, dim3(kThreads), 0, stream, g, h, m, rs.first, rs.n,
                       rs.row_off, rs.base, rs.idx, rs.chord32, rs.norm2);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_validate(const HistDev &h, int64_t n, double step, uint32_t *bad,
                           uint32_t *jmax, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, stream, h, n, step, bad, jmax);
    return hipGetLastError();
}

hipError_t launch_hull_counts(const GridDev &g, const HistDev &h, int64_t n, double wepl_in,
                              double wepl_out, uint32_t *in_cnt, uint32_t *out_cnt,
                              uint32_t in_sat, uint32_t out_sat, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hull_counts, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, stream, g, h, n, wepl_in, wepl_out, in_cnt, out_cnt,
                       in_sat, out_sat);
    return hipGetLastError();
}

hipError_t launch_hull_decide(const GridDev &g, const uint32_t *in_cnt, const uint32_t *out_cnt,
                              uint32_t min_in, uint32_t max_out, uint8_t *hull, double *mask,
                              hipStream_t stream)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 4096) wgs = 4096;
    hipLaunchKernelGGL(k_hull_decide, dim3((unsigned)wgs), dim3(kThreads), 0, stream, g, in_cnt,
                       out_cnt, min_in, max_out, hull, mask);
    return hipGetLastError();
}

hipError_t launch_pick(const int64_t *src, int64_t stride, int64_t n, int64_t *dst,
                       hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    int64_t wgs = (n + kThreads - 1) / kThreads;
    if (wgs > 1024) wgs = 1024;
    hipLaunchKernelGGL(k_pick, dim3((unsigned)wgs), dim3(kThreads), 0, stream, src, stride, n, dst);
    return hipGetLastError();
}

hipError_t launch_mlp_table(const MlpCfg &m, int64_t nj, double *tab, hipStream_t stream)
{
    if (nj <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_table, dim3((unsigned)((nj + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, stream, m, nj, tab);
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t *cnt, int64_t n, int64_t *off, int64_t *tmp,
                       hipStream_t stream)
{
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles == 0) {
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, stream, tmp, (int64_t)0);
        hipLaunchKernelGGL(k_scan_write, dim3(1), dim3(kThreads), 0, stream, cnt, (int64_t)0, tmp,
                           (int64_t)0, off);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kThreads), 0, stream, cnt, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, stream, tmp, ntiles);
    hipLaunchKernelGGL(k_scan_write, dim3((unsigned)ntiles), dim3(kThreads), 0, stream, cnt, n, tmp,
                       ntiles, off);
    return hipGetLastError();
}

}  // namespace tvs
