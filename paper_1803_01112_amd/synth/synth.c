/*
 * synth.c -- seeded synthetic proton-CT histories through a cylinder phantom
 * with material inserts (stands in for the Catphan CTP404 scans of the
 * paper, Section III-C, whose data are not available).
 *
 * This is an input generator only: it holds none of the reconstruction's
 * arithmetic (no MLP, no voxel walk, no projection, no TV).  Its transport
 * model is deliberately separate from the MLP model the reconstruction
 * assumes: a Gaussian small-angle random walk with a Highland-type angular
 * variance per step whose momentum follows the Bragg-Kleeman range-energy
 * rule R = 0.022 mm * E^1.77 (E in MeV), scaled by the local RSP.
 *
 * Every history h draws from its own counter-based stream keyed by
 * (seed, h, attempt), so the output does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double R;            /* phantom radius, mm; axis = z through the origin */
    int32_t n_ins;
    double ins_x[8], ins_y[8], ins_r[8], ins_rsp[8];
    double rsp_bg;
    double zlo, zhi;     /* slab every history must stay in (3-D) */
} sy_phantom;

typedef struct {
    int64_t n_hist;
    int32_t n_angles;
    int32_t two_d;       /* 1: v = 0 and no out-of-plane scattering */
    double e0_mev;
    double step_mm;
    double lat_frac;     /* lateral t ~ U(-lat_frac R, lat_frac R) */
    double v_margin_mm;  /* v ~ U(zlo + margin, zhi - margin) */
    double noise_frac;   /* WEPL *= 1 + noise_frac N(0,1) */
    uint64_t seed;
    int64_t first;       /* generate histories [first, first + count) */
    int64_t count;
} sy_cfg;

typedef struct {
    float *ex, *ey, *ez, *qx, *qy, *qz, *eth, *eps, *qth, *qps, *ux, *uy, *wepl;
} sy_out;

/* rrmxmx finalizer (Evensen) over a Weyl counter. */
static inline uint64_t sy_rotr(uint64_t v, int r) { return (v >> r) | (v << (64 - r)); }
static inline uint64_t sy_mix(uint64_t v)
{
    v ^= sy_rotr(v, 49) ^ sy_rotr(v, 24);
    v *= 0x9FB21C651E98DF25ull;
    v ^= v >> 28;
    v *= 0x9FB21C651E98DF25ull;
    return v ^ (v >> 28);
}
typedef struct { uint64_t key, ctr; } sy_rng;
static inline double sy_uniform(sy_rng *r)   /* (0, 1] */
{
    uint64_t z = sy_mix(r->key + 0x9E3779B97F4A7C15ull * (++r->ctr));
    return ((double)(z >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}
static inline double sy_normal(sy_rng *r)
{
    double u1 = sy_uniform(r), u2 = sy_uniform(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static double sy_rsp(const sy_phantom *p, double x, double y)
{
    if (x * x + y * y > p->R * p->R) return 0.0;
    for (int i = 0; i < p->n_ins; i++) {
        double dx = x - p->ins_x[i], dy = y - p->ins_y[i];
        if (dx * dx + dy * dy <= p->ins_r[i] * p->ins_r[i]) return p->ins_rsp[i];
    }
    return p->rsp_bg;
}

/* One attempt at history h; returns 1 on success. */
static int sy_one(const sy_phantom *p, const sy_cfg *c, int64_t h, int attempt, int planar,
                  float o[13])
{
    sy_rng rng;
    rng.key = sy_mix(c->seed ^ sy_mix((uint64_t)h * 0x100000001B3ull + (uint64_t)attempt + 1));
    rng.ctr = 0;

    int32_t a = (int32_t)((h * (int64_t)c->n_angles) / c->n_hist);
    double phi = 6.283185307179586 * (double)a / (double)c->n_angles;
    double ux = cos(phi), uy = sin(phi);
    double R = p->R;
    double t = (2.0 * sy_uniform(&rng) - 1.0) * c->lat_frac * R;
    double v = 0.0;
    if (!c->two_d)
        v = p->zlo + c->v_margin_mm + sy_uniform(&rng) * (p->zhi - p->zlo - 2.0 * c->v_margin_mm);
    double u = -sqrt(R * R - t * t);

    const double mp = 938.272;
    double range0 = 0.022 * pow(c->e0_mev, 1.77);
    double th = 0.0, ps = 0.0, wet = 0.0;
    double u_in = u, t_in = t, v_in = v;
    const double h_mm = c->step_mm;
    int64_t max_steps = (int64_t)(4.0 * R / h_mm) + 16;
    int exited = 0;
    for (int64_t s = 0; s < max_steps; s++) {
        double rr = range0 - wet;
        if (rr <= 1.0) return 0;
        double E = pow(rr / 0.022, 1.0 / 1.77);
        double pv = (E * E + 2.0 * E * mp) / (E + mp);
        double dl = h_mm * sqrt(1.0 + th * th + ps * ps);
        double um = u + 0.5 * h_mm, tm = t + 0.5 * th * h_mm;
        double rsp = sy_rsp(p, um * ux - tm * uy, um * uy + tm * ux);
        double sig = 13.6 / pv * sqrt(dl * rsp / 360.8);
        double th2 = th + sig * sy_normal(&rng);
        double ps2 = (c->two_d || planar) ? 0.0 : ps + sig * sy_normal(&rng);
        double un = u + h_mm, tn = t + 0.5 * (th + th2) * h_mm, vn = v + 0.5 * (ps + ps2) * h_mm;
        if (un > 0.0 && un * un + tn * tn > R * R) {
            /* leaves the cylinder in this step: cut the step at the surface */
            double du = un - u, dt = tn - t;
            double A = du * du + dt * dt, Bq = 2.0 * (u * du + t * dt), Cq = u * u + t * t - R * R;
            double disc = Bq * Bq - 4.0 * A * Cq;
            double f = (-Bq + sqrt(disc > 0.0 ? disc : 0.0)) / (2.0 * A);
            if (f < 0.0) f = 0.0;
            if (f > 1.0) f = 1.0;
            u += f * du;
            t += f * dt;
            v += f * (vn - v);
            wet += f * rsp * dl;
            th = th2;
            ps = ps2;
            exited = 1;
            break;
        }
        u = un; t = tn; v = vn; th = th2; ps = ps2;
        wet += rsp * dl;
        if (!c->two_d && (v < p->zlo || v > p->zhi)) return 0;
    }
    if (!exited) return 0;
    if (!c->two_d && (v < p->zlo || v > p->zhi)) return 0;

    double meas = wet * (1.0 + c->noise_frac * sy_normal(&rng));
    o[0] = (float)(u_in * ux - t_in * uy);
    o[1] = (float)(u_in * uy + t_in * ux);
    o[2] = (float)v_in;
    o[3] = (float)(u * ux - t * uy);
    o[4] = (float)(u * uy + t * ux);
    o[5] = (float)v;
    o[6] = 0.0f;
    o[7] = 0.0f;
    o[8] = (float)th;
    o[9] = (float)ps;
    o[10] = (float)ux;
    o[11] = (float)uy;
    o[12] = (float)meas;
    return 1;
}

/* Returns the number of histories that needed more than one attempt. */
int64_t sy_generate(const sy_phantom *p, const sy_cfg *c, sy_out *out)
{
    int64_t retried = 0;
    #pragma omp parallel for schedule(dynamic, 1024) reduction(+:retried)
    for (int64_t q = 0; q < c->count; q++) {
        int64_t h = c->first + q;
        float o[13] = {0};
        int ok = 0;
        for (int attempt = 0; attempt < 64 && !ok; attempt++) {
            ok = sy_one(p, c, h, attempt, 0, o);
            if (!ok) retried += (attempt == 0);
        }
        /* last resort: the same history without out-of-plane scattering */
        for (int attempt = 64; attempt < 128 && !ok; attempt++) ok = sy_one(p, c, h, attempt, 1, o);
        out->ex[q] = o[0]; out->ey[q] = o[1]; out->ez[q] = o[2];
        out->qx[q] = o[3]; out->qy[q] = o[4]; out->qz[q] = o[5];
        out->eth[q] = o[6]; out->eps[q] = o[7]; out->qth[q] = o[8]; out->qps[q] = o[9];
        out->ux[q] = o[10]; out->uy[q] = o[11]; out->wepl[q] = o[12];
    }
    return retried;
}
