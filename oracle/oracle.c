/*
 * oracle.c -- plain, slow, double-precision CPU reference of TV-superiorized
 * proton-CT reconstruction (Schultze, Censor, Karbasi, Schubert, Schulte,
 * "An Improved Method of Total Variation Superiorization Applied to
 * Reconstruction in Proton Computed Tomography", arXiv 1803.01112).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library: every formula below is written out here on its own.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 * Single precision inputs are promoted exactly to double.
 *
 * What is computed, and where the paper defines it:
 *   - the linear system, one equation per proton history: chord lengths of
 *     its most likely path (MLP) through the voxels times the unknown RSP
 *     equal its WEPL (Section I);
 *   - the MLP itself is only cited by the paper; this is the Fermi-Eyges /
 *     Highland form (Gaussian multiple-scattering model conditioned on the
 *     measured entry and exit positions and directions);
 *   - the voxel walk of each path segment uses Siddon's parametric method
 *     with the midpoint rule (the paper is silent on the walk);
 *   - P_T is one sweep of block-iterative DROP (Section III-D; Appendix A),
 *     with the block form U_t = diag(1/s_j), unit row weights;
 *   - phi = total variation, the local variations added over every voxel
 *     (Section IV), read as 2-D isotropic forward differences per slice;
 *   - the perturbation vector v = -grad(phi)/||grad(phi)|| (Appendix A);
 *   - the NTVS cycle with and without the TV-reduction check (Appendix C),
 *     the OTVS cycle (Appendix B) and the decoupled schedule proposed in
 *     Section VI (beta = alpha^n gamma^k);
 *   - the front end the paper cites: an initial iterate by parallel-beam
 *     filtered backprojection of the binned straight entry-exit lines with
 *     the in-slice median of radius 2 (Section V-A), and hull detection by
 *     space modelling and space carving on those lines (the preprocessing
 *     of Section III-D).
 *
 * Parity pins live in tests/ (closed forms, invariants, brute force).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the row formation (the only parallel loop); rows are
 * independent, so the results do not depend on it. */
void or_set_threads(int32_t n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

int32_t or_max_threads(void)
{
    return (int32_t)omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Grid.  Voxel (i,j,k) occupies [ox+i*vx, ox+(i+1)*vx) x ... ; x fastest.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double ox, oy, oz;
} or_grid;

/* ------------------------------------------------------------------------ */
/* MLP physics constants.                                                    */
/* Highland/Lynch-Dahl constant E0 = 13.6 MeV; radiation length of water     */
/* X0 = 36.08 cm = 360.8 mm.  1/(beta^2 p^2) of a 200 MeV proton in water as */
/* a 5th-order polynomial of depth (MeV^-2 cm^-k): 7.457e-6, 4.548e-7,       */
/* -5.777e-8, 1.301e-8, -9.228e-10, 2.687e-11.  Written here per mm          */
/* (coefficient k divided by 10^k) so that all lengths are in mm.            */
/* ------------------------------------------------------------------------ */
#define OR_E0_MEV 13.6
#define OR_X0_MM 360.8
static const double or_pcoef_mm[6] = {
    7.457e-6, 4.548e-8, -5.777e-10, 1.301e-11, -9.228e-14, 2.687e-16
};

typedef struct {
    double step_mm;     /* depth spacing of MLP vertices, > 0 */
    int32_t log_term;   /* 1: Highland log correction on; 0: off */
    int32_t const_power;/* 1: scattering power = its value at depth 0 */
} or_mlp_cfg;

static void or_power_coefs(const or_mlp_cfg *cfg, double b[6])
{
    for (int k = 0; k < 6; k++) b[k] = or_pcoef_mm[k];
    if (cfg->const_power)
        for (int k = 1; k < 6; k++) b[k] = 0.0;
}

static double or_factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= (double)i;
    return f;
}

static double or_ipow(double base, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= base;
    return r;
}

/*
 * Natural logarithm of a positive, finite, normal x, by the textbook
 * reduction x = m 2^e with m in [sqrt(1/2), sqrt(2)) and the series
 *   ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ... + s^21/21),
 *   s = (m - 1) / (m + 1), |s| <= 0.1716,
 * whose first omitted term is below 2e-19.  Written out here rather than
 * taken from the C library so that the MLP's Highland factor is the same
 * double on every platform (libraries round their logarithms differently).
 */
double or_log(double x)
{
    int e = 0;
    double m = frexp(x, &e);            /* x = m 2^e, m in [0.5, 1) */
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
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

static double or_highland_scale(double depth_mm, int log_term)
{
    double f = 1.0;
    if (log_term) f = 1.0 + 0.038 * or_log(depth_mm / OR_X0_MM);
    return OR_E0_MEV * OR_E0_MEV * f * f / OR_X0_MM;
}

/*
 * Scattering moments from the entry plane to depth d1 (Sigma1) and from
 * depth d1 to the exit plane at depth L (Sigma2), as {s_tt, s_tth, s_thth}.
 *
 * Sigma1: A(d1) * integral_0^d1 (d1-w)^m P(w) dw, m = 2,1,0, evaluated with
 *   integral_0^d (d-w)^m w^k dw = d^(m+k+1) m! k! / (m+k+1)!.
 * Sigma2: A(d2) * integral_d1^L (L-w)^m P(w) dw with d2 = L - d1, evaluated
 *   by substituting s = L - w and expanding P(L - s) in powers of s.
 */
void or_mlp_sigmas(double d1, double L, const or_mlp_cfg *cfg,
                   double S1[3], double S2[3])
{
    double b[6];
    or_power_coefs(cfg, b);
    double d2 = L - d1;

    double i[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < 3; m++) {
        for (int k = 0; k < 6; k++) {
            double beta = or_factorial(m) * or_factorial(k) / or_factorial(m + k + 1);
            i[m] += b[k] * or_ipow(d1, m + k + 1) * beta;
        }
    }
    double A1 = or_highland_scale(d1, cfg->log_term);
    S1[0] = A1 * i[2];
    S1[1] = A1 * i[1];
    S1[2] = A1 * i[0];

    /* P(L - s) = sum_k c_k s^k, c_k = (-1)^k sum_{q>=k} b_q C(q,k) L^(q-k). */
    double c[6];
    for (int k = 0; k < 6; k++) {
        double acc = 0.0;
        for (int q = k; q < 6; q++) {
            double binom = or_factorial(q) / (or_factorial(k) * or_factorial(q - k));
            acc += b[q] * binom * or_ipow(L, q - k);
        }
        c[k] = (k % 2) ? -acc : acc;
    }
    /* integral_0^d2 s^m s^k ds = d2^(m+k+1) / (m+k+1) */
    double q[9];
    for (int n = 1; n <= 8; n++) q[n] = or_ipow(d2, n) / (double)n;
    double j[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < 3; m++)
        for (int k = 0; k < 6; k++)
            j[m] += c[k] * q[m + k + 1];
    double A2 = or_highland_scale(d2, cfg->log_term);
    S2[0] = A2 * j[2];
    S2[1] = A2 * j[1];
    S2[2] = A2 * j[0];
}

/* 2x2 matrices, row major {a00, a01, a10, a11}. */
static void m2_mul(const double A[4], const double B[4], double C[4])
{
    double c0 = A[0] * B[0] + A[1] * B[2];
    double c1 = A[0] * B[1] + A[1] * B[3];
    double c2 = A[2] * B[0] + A[3] * B[2];
    double c3 = A[2] * B[1] + A[3] * B[3];
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}
/* Inverse as the adjugate times the reciprocal of the determinant. */
static void m2_inv(const double A[4], double R[4])
{
    double det = A[0] * A[3] - A[1] * A[2];
    double rd = 1.0 / det;
    double r0 = A[3] * rd, r1 = -A[1] * rd, r2 = -A[2] * rd, r3 = A[0] * rd;
    R[0] = r0; R[1] = r1; R[2] = r2; R[3] = r3;
}
static void m2_transpose(const double A[4], double R[4])
{
    double r1 = A[2], r2 = A[1];
    R[0] = A[0]; R[1] = r1; R[2] = r2; R[3] = A[3];
}
static void m2_vec(const double A[4], const double v[2], double r[2])
{
    double r0 = A[0] * v[0] + A[1] * v[1];
    double r1 = A[2] * v[0] + A[3] * v[1];
    r[0] = r0; r[1] = r1;
}

/*
 * Most likely (t, slope) at depth d1 given the entry state y0 = (t0, th0)
 * and the exit state y2 = (t2, th2):
 *   y1 = (S1^-1 + R1^T S2^-1 R1)^-1 (S1^-1 R0 y0 + R1^T S2^-1 y2),
 *   R0 = [[1, d1], [0, 1]], R1 = [[1, d2], [0, 1]].
 */
static void or_mlp_solve(const double S1[3], const double S2[3], double d1, double d2,
                         const double y0[2], const double y2[2], double y1[2])
{
    double Sig1[4] = {S1[0], S1[1], S1[1], S1[2]};
    double Sig2[4] = {S2[0], S2[1], S2[1], S2[2]};
    double R0[4] = {1.0, d1, 0.0, 1.0};
    double R1[4] = {1.0, d2, 0.0, 1.0};
    double S1i[4], S2i[4], R1t[4], T[4], M[4], Mi[4];
    m2_inv(Sig1, S1i);
    m2_inv(Sig2, S2i);
    m2_transpose(R1, R1t);
    m2_mul(R1t, S2i, T);          /* R1^T S2^-1 */
    double T2[4];
    m2_mul(T, R1, T2);            /* R1^T S2^-1 R1 */
    for (int q = 0; q < 4; q++) M[q] = S1i[q] + T2[q];
    double a[2], a2[2], bb[2], rhs[2];
    m2_vec(R0, y0, a);            /* R0 y0 */
    m2_vec(S1i, a, a2);           /* S1^-1 R0 y0 */
    m2_vec(T, y2, bb);            /* R1^T S2^-1 y2 */
    rhs[0] = a2[0] + bb[0];
    rhs[1] = a2[1] + bb[1];
    m2_inv(M, Mi);
    m2_vec(Mi, rhs, y1);
}

/*
 * MLP polyline of one history, in mm: [entry, vertices at depths j*step
 * (j = 1..J-1, J = max(1, ceil(L/step))), exit].  The depth axis u is the
 * beam axis (ux, uy, 0) normalised; t is the in-plane lateral axis
 * (-uy, ux, 0); v is z.  Slopes th = dt/du, ps = dv/du.
 * Returns the number of points written (J+1), -1 when L = u_exit - u_entry
 * is not positive (the history forms no row), or -2 when cap is too small.
 */
int64_t or_mlp_polyline(const double h[12], const or_mlp_cfg *cfg,
                        double *pts, int64_t cap)
{
    double ex = h[0], ey = h[1], ez = h[2], qx = h[3], qy = h[4], qz = h[5];
    double eth = h[6], eps = h[7], qth = h[8], qps = h[9];
    double ux = h[10], uy = h[11];
    double nrm = sqrt(ux * ux + uy * uy);
    ux = ux / nrm;
    uy = uy / nrm;

    double u0 = ex * ux + ey * uy, t0 = -ex * uy + ey * ux, v0 = ez;
    double u2 = qx * ux + qy * uy, t2 = -qx * uy + qy * ux, v2 = qz;
    double L = u2 - u0;
    if (!(L > 0.0)) return -1;
    double Jd = ceil(L / cfg->step_mm);
    int64_t J = (Jd < 1.0) ? 1 : (int64_t)Jd;
    if (J + 1 > cap) return -2;

    pts[0] = ex; pts[1] = ey; pts[2] = ez;
    for (int64_t j = 1; j < J; j++) {
        double d1 = (double)j * cfg->step_mm;
        double d2 = L - d1;
        double S1[3], S2[3];
        or_mlp_sigmas(d1, L, cfg, S1, S2);
        double yt0[2] = {t0, eth}, yt2[2] = {t2, qth}, yt1[2];
        double yv0[2] = {v0, eps}, yv2[2] = {v2, qps}, yv1[2];
        or_mlp_solve(S1, S2, d1, d2, yt0, yt2, yt1);
        or_mlp_solve(S1, S2, d1, d2, yv0, yv2, yv1);
        double u = u0 + d1;
        pts[3 * j + 0] = u * ux - yt1[0] * uy;
        pts[3 * j + 1] = u * uy + yt1[0] * ux;
        pts[3 * j + 2] = yv1[0];
    }
    pts[3 * J + 0] = qx; pts[3 * J + 1] = qy; pts[3 * J + 2] = qz;
    return J + 1;
}

/* ------------------------------------------------------------------------ */
/* Siddon walk of a polyline, midpoint rule.                                 */
/* ------------------------------------------------------------------------ */
static int or_cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

typedef struct {
    int32_t *idx;      /* NULL: count only */
    double *chord;
    int64_t cap;
    int64_t n;         /* entries emitted so far */
    int32_t cur;       /* voxel of the open entry, -1 if none */
    double cur_len;
    double norm2;
    int overflow;
} or_emit;

static void or_emit_flush(or_emit *e)
{
    if (e->cur < 0) return;
    if (e->idx) {
        if (e->n < e->cap) {
            e->idx[e->n] = e->cur;
            e->chord[e->n] = e->cur_len;
        } else {
            e->overflow = 1;
        }
    }
    e->norm2 += e->cur_len * e->cur_len;
    e->n++;
    e->cur = -1;
    e->cur_len = 0.0;
}

/*
 * Walk one segment q0 -> q1 (mm).  Grid coordinates g = (p - o)/v.  The
 * parameters tau in [0,1] where the segment crosses an integer plane
 * 0..n of any axis, together with 0 and 1, are sorted and exactly equal
 * values merged; each consecutive pair is a piece whose voxel is the floor
 * of the grid coordinate at the piece midpoint.  Pieces outside the grid
 * are dropped; a piece in the same voxel as the open entry extends it, so
 * no two consecutive entries of a row share a voxel.
 */
static void or_walk_segment(const or_grid *g, const double q0[3], const double q1[3],
                            or_emit *e, double *taus, int64_t taus_cap)
{
    const int32_t n[3] = {g->nx, g->ny, g->nz};
    const double vs[3] = {g->vx, g->vy, g->vz};
    const double o[3] = {g->ox, g->oy, g->oz};
    double g0[3], g1[3], dg[3];
    for (int a = 0; a < 3; a++) {
        g0[a] = (q0[a] - o[a]) / vs[a];
        g1[a] = (q1[a] - o[a]) / vs[a];
        dg[a] = g1[a] - g0[a];
    }
    double dx = q1[0] - q0[0], dy = q1[1] - q0[1], dz = q1[2] - q0[2];
    double len = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(len > 0.0)) return;

    int64_t nt = 0;
    taus[nt++] = 0.0;
    taus[nt++] = 1.0;
    for (int a = 0; a < 3; a++) {
        if (dg[a] == 0.0) continue;
        double lo = (g0[a] < g1[a]) ? g0[a] : g1[a];
        double hi = (g0[a] < g1[a]) ? g1[a] : g0[a];
        double mlo = floor(lo) + 1.0;   /* smallest integer > lo */
        double mhi = ceil(hi) - 1.0;    /* largest integer < hi */
        if (mlo < 0.0) mlo = 0.0;
        if (mhi > (double)n[a]) mhi = (double)n[a];
        for (double m = mlo; m <= mhi; m += 1.0) {
            if (nt < taus_cap) taus[nt++] = (m - g0[a]) / dg[a];
        }
    }
    qsort(taus, (size_t)nt, sizeof(double), or_cmp_double);

    double prev = taus[0];
    for (int64_t q = 1; q < nt; q++) {
        double tb = taus[q];
        if (!(tb > prev)) continue;     /* merge exactly equal parameters */
        double ta = prev;
        prev = tb;
        double tm = (ta + tb) * 0.5;
        int inside = 1;
        int64_t vi[3];
        for (int a = 0; a < 3; a++) {
            double c = floor(g0[a] + tm * dg[a]);
            if (c < 0.0 || c >= (double)n[a]) { inside = 0; break; }
            vi[a] = (int64_t)c;
        }
        if (!inside) continue;
        int32_t lin = (int32_t)(vi[0] + (int64_t)n[0] * (vi[1] + (int64_t)n[1] * vi[2]));
        double clen = (tb - ta) * len;
        if (lin == e->cur) {
            e->cur_len += clen;
        } else {
            or_emit_flush(e);
            e->cur = lin;
            e->cur_len = clen;
        }
    }
}

static int64_t or_taus_cap(const or_grid *g)
{
    return (int64_t)g->nx + g->ny + g->nz + 8;
}

/*
 * Row of the linear system for one polyline: voxel indices (ix + nx*(iy +
 * ny*iz)) and chord lengths in mm, in traversal order; *norm2 = sum of
 * squared chords.  Returns the entry count (which may exceed cap; then only
 * cap entries were written and the caller must retry with more room).
 */
int64_t or_walk_polyline(const or_grid *g, const double *pts, int64_t npts,
                         int32_t *idx, double *chord, int64_t cap, double *norm2)
{
    or_emit e = {idx, chord, cap, 0, -1, 0.0, 0.0, 0};
    int64_t tcap = or_taus_cap(g);
    double *taus = (double *)malloc(sizeof(double) * (size_t)tcap);
    for (int64_t s = 0; s + 1 < npts; s++)
        or_walk_segment(g, pts + 3 * s, pts + 3 * (s + 1), &e, taus, tcap);
    or_emit_flush(&e);
    free(taus);
    if (norm2) *norm2 = e.norm2;
    return e.n;
}

/* ------------------------------------------------------------------------ */
/* Rows of many histories (SoA, single precision inputs).                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *ex, *ey, *ez, *qx, *qy, *qz;
    const float *eth, *eps, *qth, *qps;
    const float *ux, *uy;
    const float *wepl;
} or_hist;

static void or_hist_get(const or_hist *H, int64_t i, double h[12])
{
    h[0] = H->ex[i]; h[1] = H->ey[i]; h[2] = H->ez[i];
    h[3] = H->qx[i]; h[4] = H->qy[i]; h[5] = H->qz[i];
    h[6] = H->eth[i]; h[7] = H->eps[i]; h[8] = H->qth[i]; h[9] = H->qps[i];
    h[10] = H->ux[i]; h[11] = H->uy[i];
}

static int64_t or_row_one(const or_grid *g, const or_hist *H, int64_t i, const or_mlp_cfg *cfg,
                          int32_t *idx, double *chord, int64_t cap, double *norm2)
{
    double h[12];
    or_hist_get(H, i, h);
    double nrm = sqrt(h[10] * h[10] + h[11] * h[11]);
    double L = (h[3] - h[0]) * (h[10] / nrm) + (h[4] - h[1]) * (h[11] / nrm);
    if (!(L > -1.0)) L = 0.0;
    int64_t pcap = (int64_t)ceil((fabs(L) + 1.0) / cfg->step_mm) + 4;
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)pcap);
    int64_t np = or_mlp_polyline(h, cfg, pts, pcap);
    int64_t n = 0;
    *norm2 = 0.0;
    if (np > 0) n = or_walk_polyline(g, pts, np, idx, chord, cap, norm2);
    free(pts);
    return n;
}

/*
 * Pass 1 (idx == NULL): nnz[i] for every history.  Pass 2: fills idx/chord
 * at row_off[i] and norm2[i].  OpenMP over histories; every row is
 * independent, so the result does not depend on the thread count.
 */
void or_build_rows(const or_grid *g, const or_hist *H, int64_t nh, const or_mlp_cfg *cfg,
                   int64_t *nnz, const int64_t *row_off, int32_t *idx, double *chord,
                   double *norm2)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nh; i++) {
        double n2 = 0.0;
        if (idx == NULL) {
            nnz[i] = or_row_one(g, H, i, cfg, NULL, NULL, 0, &n2);
        } else {
            int64_t off = row_off[i], cap = row_off[i + 1] - row_off[i];
            or_row_one(g, H, i, cfg, idx + off, chord + off, cap, &n2);
            if (norm2) norm2[i] = n2;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* DROP: one sweep P_T over all blocks.                                      */
/* ------------------------------------------------------------------------ */
/*
 * Block t = histories [t*B, min((t+1)*B, H)) in load order.  From the same
 * x, every row i of the block with ||a_i||^2 > 0 gives
 * r_i = (b_i - a_i.x)/||a_i||^2; c_j = sum_i r_i a_ij; s_j = number of row
 * entries at voxel j; then x_j += lambda c_j / s_j where s_j > 0.
 */
void or_drop_sweep(int64_t nvox, double *x, int64_t nh, const int64_t *row_off,
                   const int32_t *idx, const double *chord, const double *norm2,
                   const double *wepl, double lambda, int64_t B)
{
    double *c = (double *)calloc((size_t)nvox, sizeof(double));
    int64_t *s = (int64_t *)calloc((size_t)nvox, sizeof(int64_t));
    for (int64_t t0 = 0; t0 < nh; t0 += B) {
        int64_t t1 = t0 + B < nh ? t0 + B : nh;
        for (int64_t i = t0; i < t1; i++) {
            if (!(norm2[i] > 0.0)) continue;
            double dot = 0.0;
            for (int64_t e = row_off[i]; e < row_off[i + 1]; e++) dot += chord[e] * x[idx[e]];
            double r = (wepl[i] - dot) / norm2[i];
            for (int64_t e = row_off[i]; e < row_off[i + 1]; e++) {
                c[idx[e]] += r * chord[e];
                s[idx[e]] += 1;
            }
        }
        for (int64_t i = t0; i < t1; i++) {
            for (int64_t e = row_off[i]; e < row_off[i + 1]; e++) {
                int32_t j = idx[e];
                if (s[j] > 0) {
                    x[j] += lambda * c[j] / (double)s[j];
                    c[j] = 0.0;
                    s[j] = 0;
                }
            }
        }
    }
    free(c);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Total variation (Section IV) and its subgradient.                         */
/* ------------------------------------------------------------------------ */
/*
 * Per slice, forward differences with a zero difference at the far edge:
 * dx_ij = x(i+1,j) - x(i,j), dy_ij = x(i,j+1) - x(i,j); local variation
 * m_ij = sqrt(dx^2 + dy^2 + eps^2); phi = sum over all voxels of (m - eps).
 */
static double or_dx(const or_grid *g, const double *x, int64_t i, int64_t j, int64_t k)
{
    if (i + 1 >= g->nx) return 0.0;
    int64_t p = i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
    return x[p + 1] - x[p];
}
static double or_dy(const or_grid *g, const double *x, int64_t i, int64_t j, int64_t k)
{
    if (j + 1 >= g->ny) return 0.0;
    int64_t p = i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
    return x[p + g->nx] - x[p];
}
static double or_m(const or_grid *g, const double *x, int64_t i, int64_t j, int64_t k, double eps)
{
    double a = or_dx(g, x, i, j, k), b = or_dy(g, x, i, j, k);
    return sqrt(a * a + b * b + eps * eps);
}

double or_tv(const or_grid *g, const double *x, double eps)
{
    double phi = 0.0;
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++)
                phi += or_m(g, x, i, j, k, eps) - eps;
    return phi;
}

/*
 * g_ij = d phi / d x_ij: x_ij enters m_ij (through -dx_ij - dy_ij),
 * m_(i-1)j (through +dx_(i-1)j) and m_i(j-1) (through +dy_i(j-1)).
 * A term whose m is zero contributes zero (the subgradient chosen at the
 * non-smooth points).  Returns ||g||^2.
 */
double or_tv_grad(const or_grid *g, const double *x, double eps, double *gout)
{
    double n2 = 0.0;
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                double gv = 0.0;
                double m = or_m(g, x, i, j, k, eps);
                if (m > 0.0) gv -= (or_dx(g, x, i, j, k) + or_dy(g, x, i, j, k)) / m;
                if (i > 0) {
                    double mm = or_m(g, x, i - 1, j, k, eps);
                    if (mm > 0.0) gv += or_dx(g, x, i - 1, j, k) / mm;
                }
                if (j > 0) {
                    double mm = or_m(g, x, i, j - 1, k, eps);
                    if (mm > 0.0) gv += or_dy(g, x, i, j - 1, k) / mm;
                }
                gout[i + (int64_t)g->nx * (j + (int64_t)g->ny * k)] = gv;
                n2 += gv * gv;
            }
    return n2;
}

/* ------------------------------------------------------------------------ */
/* Schedule: SplitMix64 and ell_k = rand(k, ell_{k-1}).                      */
/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014): the state advances by the golden    */
/* gamma and the output is the state passed through the variant-13 mixer.    */
uint64_t or_splitmix64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ull;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform integer in [k, ell] (both ends included), one draw per call; k    */
/* itself when ell < k.                                                       */
int64_t or_rand_ell(int64_t k, int64_t ell, uint64_t *state)
{
    uint64_t u = or_splitmix64_next(state);
    if (ell < k) return k;
    unsigned __int128 span = (unsigned __int128)(uint64_t)(ell - k + 1);
    unsigned __int128 prod = (unsigned __int128)u * span;
    return k + (int64_t)(uint64_t)(prod >> 64);
}

/* ------------------------------------------------------------------------ */
/* Superiorization driver: NTVS (Appendix C, with and without the TV check), */
/* OTVS (Appendix B) and the decoupled schedule of Section VI.               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lambda;
    int32_t N;
    double alpha;
    int32_t tv_check;   /* NTVS only */
    int32_t variant;    /* 0 NTVS, 1 OTVS, 2 decoupled alpha^n gamma^k */
    double tv_eps;
    uint64_t seed;
    double gamma;       /* variant 2 */
    int32_t max_tries;  /* bound on the retry loop of a checked step */
} or_params;

typedef struct {
    int64_t k;          /* cycles done */
    int64_t ell;
    uint64_t rng;
    int32_t seeded;
} or_state;

/* One log record per perturbation step. */
typedef struct {
    int32_t k, n;
    int32_t tries;       /* tries until accept (or max_tries) */
    int32_t accepted;    /* 0 when the step gave up after max_tries */
    int64_t ell_start;   /* ell at the first try */
    double phi_x;        /* phi before the step (checked steps) */
    double phi_z;        /* phi of the accepted z */
    double gnorm;        /* ||grad phi|| */
    int32_t disagree;    /* replay: tries where the oracle would decide otherwise */
    int32_t pad;
    double worst_margin; /* replay: largest |phi(z)-phi(x)| among disagreeing tries */
} or_step_log;

typedef struct {
    int64_t nh;
    const int64_t *row_off;
    const int32_t *idx;
    const double *chord;
    const double *norm2;
    const double *wepl;
    int64_t B;
} or_system;

/*
 * K more cycles from state st on image x (nvox = nx*ny*nz doubles).
 * ell_log[k] receives ell_k after its draw (before the steps).  log may be
 * NULL; otherwise it receives one record per step (capacity log_cap).
 * replay_tries (checked steps only) may be NULL; otherwise entry s is the
 * number of tries step s must take, the last one accepted, which lets the
 * oracle follow another implementation's decisions while recording where
 * its own decision would differ.  Returns the number of step records.
 */
int64_t or_superiorize(const or_grid *g, const or_system *sys, double *x,
                       const or_params *p, int32_t K, or_state *st,
                       int64_t *ell_log, or_step_log *log, int64_t log_cap,
                       const int32_t *replay_tries, int64_t replay_n)
{
    int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    double *gr = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *z = (double *)malloc(sizeof(double) * (size_t)nvox);
    int64_t nlog = 0;
    if (!st->seeded) {
        st->rng = p->seed;
        st->seeded = 1;
    }
    int checked = (p->variant == 1) || (p->variant == 0 && p->tv_check);
    int32_t Nsteps = (p->variant == 1) ? 1 : p->N;

    for (int32_t kk = 0; kk < K; kk++) {
        int64_t k = st->k;
        if (p->variant == 0) st->ell = or_rand_ell(k, st->ell, &st->rng);
        if (ell_log) ell_log[kk] = st->ell;
        for (int32_t n = 0; n < Nsteps; n++) {
            double n2 = or_tv_grad(g, x, p->tv_eps, gr);
            double gn = sqrt(n2);
            /* v = -g/||g|| (v = 0 when g = 0) */
            double inv = (gn > 0.0) ? 1.0 / gn : 0.0;
            or_step_log rec;
            memset(&rec, 0, sizeof(rec));
            rec.k = (int32_t)k;
            rec.n = n;
            rec.ell_start = st->ell;
            rec.gnorm = gn;
            if (!checked) {
                double beta;
                if (p->variant == 2) beta = pow(p->alpha, (double)(n + 1)) * pow(p->gamma, (double)k);
                else beta = pow(p->alpha, (double)st->ell);
                for (int64_t j = 0; j < nvox; j++) x[j] += beta * (-gr[j] * inv);
                st->ell += 1;
                rec.tries = 1;
                rec.accepted = 1;
            } else {
                double phx = or_tv(g, x, p->tv_eps);
                rec.phi_x = phx;
                int32_t want = -1;
                if (replay_tries && nlog < replay_n) want = replay_tries[nlog];
                int32_t tries = 0;
                int accepted = 0;
                while (tries < p->max_tries) {
                    double beta = (p->variant == 1) ? pow(0.5, (double)st->ell)
                                                    : pow(p->alpha, (double)st->ell);
                    for (int64_t j = 0; j < nvox; j++) z[j] = x[j] + beta * (-gr[j] * inv);
                    double phz = or_tv(g, z, p->tv_eps);
                    tries++;
                    st->ell += 1;
                    int mine = (phz <= phx);
                    int take = mine;
                    if (want > 0) {
                        take = (tries == want);
                        if (take != mine) {
                            rec.disagree++;
                            double mg = fabs(phz - phx);
                            if (mg > rec.worst_margin) rec.worst_margin = mg;
                        }
                    }
                    if (take) {
                        memcpy(x, z, sizeof(double) * (size_t)nvox);
                        rec.phi_z = phz;
                        accepted = 1;
                        break;
                    }
                }
                rec.tries = tries;
                rec.accepted = accepted;
            }
            if (log && nlog < log_cap) log[nlog] = rec;
            nlog++;
        }
        or_drop_sweep(nvox, x, sys->nh, sys->row_off, sys->idx, sys->chord, sys->norm2,
                      sys->wepl, p->lambda, sys->B);
        st->k += 1;
    }
    free(gr);
    free(z);
    return nlog;
}

/* ------------------------------------------------------------------------ */
/* Initial iterate: filtered backprojection of binned histories and an       */
/* in-slice median filter.  The paper starts its reconstructions from an     */
/* initial iterate with a median filter of radius 2 applied (Section V-A,   */
/* citing earlier work); the backprojection itself is not given there.      */
/* Reading: textbook parallel-beam FBP.  Each history's straight line from    */
/* entry to exit is binned at its crossing of the depth u = 0 (the rotation  */
/* axis): angle bin a = round(phi / (2 pi / A)) mod A of the beam direction, */
/* lateral bin m of t in width tau (nt bins centred on t = 0), slice k of    */
/* the height v.  A bin's projection is the mean WEPL of its histories      */
/* (0 when empty).  Rows are filtered with the discrete Ram-Lak kernel       */
/* h(0) = 1/(4 tau^2), h(n odd) = -1/(n^2 pi^2 tau^2), h(n even) = 0, times */
/* tau, and backprojected with linear interpolation and weight pi / A (A    */
/* angles over 360 degrees see every line twice).  Median: lower median of  */
/* the (2r+1)^2 window clipped to the slice.                                */
/* ------------------------------------------------------------------------ */
#define OR_FBP_FIXED 4294967296.0   /* WEPL sums in units of 2^-32 mm */

static const double or_pi = 3.14159265358979323846;

/* Bin index (a, k, m) of one history, or -1 when it falls outside. */
static int64_t or_fbp_bin_index(const or_grid *g, const double h[12], int32_t A, double tau,
                                int32_t nt)
{
    double ex = h[0], ey = h[1], ez = h[2], qx = h[3], qy = h[4], qz = h[5];
    double ux = h[10], uy = h[11];
    double nrm = sqrt(ux * ux + uy * uy);
    ux = ux / nrm;
    uy = uy / nrm;
    double u0 = ex * ux + ey * uy, t0 = -ex * uy + ey * ux;
    double u2 = qx * ux + qy * uy, t2 = -qx * uy + qy * ux;
    double L = u2 - u0;
    if (!(L > 0.0)) return -1;
    double f = (0.0 - u0) / L;
    double tc = t0 + (t2 - t0) * f;
    double vc = ez + (qz - ez) * f;
    double phi = atan2(uy, ux);
    double da = 2.0 * or_pi / (double)A;
    int64_t a = (int64_t)floor(phi / da + 0.5);
    a %= A;
    if (a < 0) a += A;
    double mm = floor(tc / tau + 0.5 * (double)nt);
    if (!(mm >= 0.0 && mm < (double)nt)) return -1;
    double kk = floor((vc - g->oz) / g->vz);
    if (!(kk >= 0.0 && kk < (double)g->nz)) return -1;
    return (a * g->nz + (int64_t)kk) * nt + (int64_t)mm;
}

/* Projections p[(a * nz + k) * nt + m]: mean WEPL per bin; counts too. */
void or_fbp_bin(const or_grid *g, const or_hist *H, int64_t nh, int32_t A, double tau,
                int32_t nt, double *p, int64_t *count)
{
    int64_t nb = (int64_t)A * g->nz * nt;
    int64_t *sum = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    for (int64_t b = 0; b < nb; b++) count[b] = 0;
    for (int64_t i = 0; i < nh; i++) {
        double h[12];
        or_hist_get(H, i, h);
        int64_t b = or_fbp_bin_index(g, h, A, tau, nt);
        if (b < 0) continue;
        sum[b] += (int64_t)llrint((double)H->wepl[i] * OR_FBP_FIXED);
        count[b] += 1;
    }
    for (int64_t b = 0; b < nb; b++)
        p[b] = count[b] ? ((double)sum[b] / OR_FBP_FIXED) / (double)count[b] : 0.0;
    free(sum);
}

/* Ram-Lak filtered rows: q[r * nt + m] = tau * sum_s p[r * nt + s] h(m - s). */
void or_fbp_filter(const double *p, int64_t rows, int32_t nt, double tau, double *q)
{
    for (int64_t r = 0; r < rows; r++)
        for (int32_t m = 0; m < nt; m++) {
            double acc = 0.0;
            for (int32_t s = 0; s < nt; s++) {
                int32_t n = m - s;
                double hv;
                if (n == 0) hv = 1.0 / (4.0 * tau * tau);
                else if (n % 2 != 0) hv = -1.0 / ((double)n * (double)n * or_pi * or_pi * tau * tau);
                else continue;
                acc += p[r * nt + s] * hv;
            }
            q[r * nt + m] = tau * acc;
        }
}

/* Backprojection into the x-fastest image x (nx * ny * nz). */
void or_fbp_backproject(const or_grid *g, const double *q, int32_t A, double tau, int32_t nt,
                        double *x)
{
    double da = 2.0 * or_pi / (double)A;
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                double X = g->ox + ((double)i + 0.5) * g->vx;
                double Y = g->oy + ((double)j + 0.5) * g->vy;
                double acc = 0.0;
                for (int32_t a = 0; a < A; a++) {
                    double phi = (double)a * da;
                    double t = -X * sin(phi) + Y * cos(phi);
                    double sp = t / tau + 0.5 * (double)nt - 0.5;
                    double m0 = floor(sp);
                    double w = sp - m0;
                    const double *row = q + ((int64_t)a * g->nz + k) * nt;
                    double v0 = (m0 >= 0.0 && m0 < (double)nt) ? row[(int64_t)m0] : 0.0;
                    double v1 = (m0 + 1.0 >= 0.0 && m0 + 1.0 < (double)nt) ? row[(int64_t)m0 + 1] : 0.0;
                    acc += (1.0 - w) * v0 + w * v1;
                }
                x[i + g->nx * (j + g->ny * k)] = acc * (or_pi / (double)A);
            }
}

static int or_cmp_double_asc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* In-slice median of radius r (window clipped to the slice, lower median). */
void or_median_slices(const or_grid *g, const double *x, int32_t r, double *y)
{
    int32_t w = 2 * r + 1;
    double *buf = (double *)malloc(sizeof(double) * (size_t)(w * w));
    for (int64_t k = 0; k < g->nz; k++)
        for (int64_t j = 0; j < g->ny; j++)
            for (int64_t i = 0; i < g->nx; i++) {
                int n = 0;
                for (int64_t dj = -r; dj <= r; dj++)
                    for (int64_t di = -r; di <= r; di++) {
                        int64_t ii = i + di, jj = j + dj;
                        if (ii < 0 || ii >= g->nx || jj < 0 || jj >= g->ny) continue;
                        buf[n++] = x[ii + g->nx * (jj + g->ny * k)];
                    }
                qsort(buf, (size_t)n, sizeof(double), or_cmp_double_asc);
                y[i + g->nx * (j + g->ny * k)] = buf[(n - 1) / 2];
            }
    free(buf);
}

/* ------------------------------------------------------------------------ */
/* Hull detection.  The paper's preprocessing (Section III-D, citing earlier */
/* work) bounds the object before the MLP is formed; how is not given.       */
/* Reading: the textbook straight-line hull detectors, on each history's     */
/* straight line from its entry to its exit point, voxels taken by the same  */
/* midpoint walk as the rows:                                                */
/*   space modelling: in_count[j] = histories with WEPL >= wepl_in whose     */
/*     line crosses voxel j (the object is where protons lost energy);       */
/*   space carving: out_count[j] = histories with WEPL < wepl_out whose line */
/*     crosses j (a proton that lost no energy crossed no object);           */
/*   hull[j] = in_count[j] >= min_in and out_count[j] <= max_out.            */
/* ------------------------------------------------------------------------ */
void or_hull_counts(const or_grid *g, const or_hist *H, int64_t nh, double wepl_in,
                    double wepl_out, int32_t *in_count, int32_t *out_count)
{
    int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    memset(in_count, 0, sizeof(int32_t) * (size_t)nvox);
    memset(out_count, 0, sizeof(int32_t) * (size_t)nvox);
    int64_t cap = (int64_t)g->nx + g->ny + g->nz + 8;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    double *chord = (double *)malloc(sizeof(double) * (size_t)cap);
    for (int64_t i = 0; i < nh; i++) {
        double w = H->wepl[i];
        int in = (w >= wepl_in), out = (w < wepl_out);
        if (!in && !out) continue;
        double pts[6] = {H->ex[i], H->ey[i], H->ez[i], H->qx[i], H->qy[i], H->qz[i]};
        int64_t n = or_walk_polyline(g, pts, 2, idx, chord, cap, NULL);
        if (n > cap) n = cap;
        for (int64_t q = 0; q < n; q++) {
            if (in) in_count[idx[q]] += 1;
            if (out) out_count[idx[q]] += 1;
        }
    }
    free(idx);
    free(chord);
}

void or_hull_decide(int64_t nvox, const int32_t *in_count, const int32_t *out_count,
                    int32_t min_in, int32_t max_out, uint8_t *hull)
{
    for (int64_t j = 0; j < nvox; j++)
        hull[j] = (uint8_t)(in_count[j] >= min_in && out_count[j] <= max_out);
}
