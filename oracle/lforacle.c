/*
 * lforacle.c -- plain FP64 CPU oracle for the LumiPath light-field path.
 *
 * TEST INFRASTRUCTURE ONLY (see lforacle.h).  Written for reading, not for
 * speed: every quantity is computed in double precision, straight from its
 * definition, in the order the method states it.  Citations name the
 * section, equation or paragraph of Fink et al. 2019 (arXiv 1903.03837).
 * The volumetric path tracer is the repository's reading of the paper's
 * conventional, PBRT-like path tracer (Sec. 2) applied to a density volume;
 * its conventions (random-number counters, majorant, jitter frame, lights)
 * are stated at each step below.
 */
#include "lforacle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
/* Golden ratio: Phi = (1 + sqrt 5) / 2; 1/Phi = Phi - 1.  The paper writes
 * phi_i = 2 pi [i / Phi] with [x] the fractional part (Sec. 2, SF point
 * equation); Phi is not defined there and is read as the golden ratio of
 * the cited spherical-Fibonacci papers. */
static double golden(void) { return (1.0 + sqrt(5.0)) / 2.0; }

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double a[3], const double b[3], double r[3]) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static void cross3(const double a[3], const double b[3], double r[3]) {
    double x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void normalize3(double a[3]) { double l = norm3(a); a[0] /= l; a[1] /= l; a[2] /= l; }

/* ------------------------------------------------------------------------ */
/* Spherical Fibonacci point set (Sec. 2, SF point equation)                  */
/*   p_i = C(phi_i, acos z_i), phi_i = 2 pi frac(i / Phi), z_i = 1-(2i+1)/n   */
/* C converts (polar angle theta = acos z_i, azimuth phi_i) to Cartesian;    */
/* the argument order printed in the equation is read as (azimuth, polar).   */
/* ------------------------------------------------------------------------ */
void orc_sf_point(int64_t n, int64_t i, double p[3]) {
    double x = (double)i / golden();
    double f = x - floor(x);
    double phi = 2.0 * PI * f;
    double z = 1.0 - (2.0 * (double)i + 1.0) / (double)n;
    double theta = acos(z);
    p[0] = cos(phi) * sin(theta);
    p[1] = sin(phi) * sin(theta);
    p[2] = cos(theta);
    /* cos(acos z) may differ from z in the last bit; the definition fixes
     * the height exactly, so use it. */
    p[2] = z;
}

void orc_sf_points(int64_t n, double* xyz) {
    for (int64_t i = 0; i < n; ++i) orc_sf_point(n, i, xyz + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Nearest point: plain definition, argmin over all n points                 */
/* ------------------------------------------------------------------------ */
int64_t orc_nearest(int64_t n, const double q[3], double* d2_best, double* d2_second) {
    int64_t best = -1;
    double b = INFINITY, s = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double p[3], d[3];
        orc_sf_point(n, i, p);
        sub3(q, p, d);
        double e = dot3(d, d);
        if (e < b) { s = b; b = e; best = i; }
        else if (e < s) { s = e; }
    }
    if (d2_best) *d2_best = b;
    if (d2_second) *d2_second = s;
    return best;
}

int64_t orc_fib(int32_t k) {
    int64_t a = 0, b = 1;
    for (int32_t t = 0; t < k; ++t) { int64_t c = a + b; a = b; b = c; }
    return a;
}

/* Zone of the Fibonacci lattice around height qz (inverse SF mapping of
 * Keinert et al. 2015, used in Sec. 2 for the nearest-neighbour query).  The
 * local lattice is spanned by the index steps F(k) and F(k+1). */
int32_t orc_zone(int64_t n, double qz, double* margin) {
    double PHI = golden();
    double arg = (double)n * PI * sqrt(5.0) * (1.0 - qz) * (1.0 + qz);
    if (!(arg > 0.0)) { if (margin) *margin = 1e300; return 2; }
    double lv = log(arg) / log(PHI * PHI);
    int32_t k = (int32_t)floor(lv);
    if (k < 2) k = 2;
    if (margin) {
        double m = 1e300;
        double r = floor(lv + 0.5);
        if (r >= 3.0) m = fabs(lv - r);
        else m = 3.0 - lv;
        *margin = m;
    }
    return k;
}

/* K-neighbour query (Sec. 2: at most nine neighbours, five of them used per
 * hit point, weighted by distance with a filter of size R sqrt(4 pi / N)).
 * The nine are the nearest point and its eight Fibonacci-lattice
 * neighbours i* +- {F(k-1), F(k), F(k+1), F(k+2)}. */
int32_t orc_neighbors(int64_t n, const double q[3], int32_t K,
                      int64_t* idx, double* w, double* d2out, double margins[3]) {
    double b2, s2;
    int64_t ist = orc_nearest(n, q, &b2, &s2);
    double zm;
    int32_t k = orc_zone(n, q[2], &zm);
    int64_t off[4] = {orc_fib(k - 1), orc_fib(k), orc_fib(k + 1), orc_fib(k + 2)};
    int64_t cand[9];
    double cd[9];
    int nc = 0;
    for (int t = 0; t < 9; ++t) {
        int64_t c = ist;
        if (t > 0) c = ist + ((t & 1) ? off[(t - 1) / 2] : -off[(t - 1) / 2]);
        if (c < 0 || c >= n) continue;
        int dup = 0;
        for (int u = 0; u < nc; ++u) dup |= cand[u] == c;
        if (dup) continue;
        double p[3], d[3];
        orc_sf_point(n, c, p);
        sub3(q, p, d);
        cand[nc] = c;
        cd[nc] = dot3(d, d);
        ++nc;
    }
    /* order by (distance^2, index): plain insertion sort */
    for (int a = 1; a < nc; ++a)
        for (int b = a; b > 0; --b) {
            int swap = cd[b] < cd[b - 1] || (cd[b] == cd[b - 1] && cand[b] < cand[b - 1]);
            if (!swap) break;
            double td = cd[b]; cd[b] = cd[b - 1]; cd[b - 1] = td;
            int64_t tc = cand[b]; cand[b] = cand[b - 1]; cand[b - 1] = tc;
        }
    int32_t m = nc < K ? nc : K;
    /* filter size R sqrt(4 pi / n) (the printed R 5^(1/4) sqrt(4 pi /
     * (sqrt5 n)) simplifies to it); tent of that radius, unit-sphere chord. */
    double r = sqrt(4.0 * PI / (double)n);
    for (int32_t a = 0; a < m; ++a) {
        idx[a] = cand[a];
        if (d2out) d2out[a] = cd[a];
        double wt = 1.0 - sqrt(cd[a]) / r;
        w[a] = wt > 0.0 ? wt : 0.0;
    }
    if (margins) {
        margins[0] = s2 - b2;
        margins[1] = zm;
        margins[2] = nc > K ? cd[K] - cd[K - 1] : 1e300;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the      */
/* 4x32 Philox S-box with multipliers 0xD2511F53, 0xCD9E8D57 and the Weyl     */
/* key schedule 0x9E3779B9, 0xBB67AE85.                                       */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_uniform(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Random-number streams.  The counter is (ray, sample, bounce << 8 |
 * purpose, block) and block b supplies stream positions 4b .. 4b+3, word by
 * word; positions are used in pairs (pair p = positions 2p, 2p+1).
 *   purpose 1, "flight" of segment b: at b = 0 pair 0 jitters the origin and
 *     tentative collision n uses pair n+1; at b > 0 collision n uses pair n.
 *     A collision pair is (free-flight distance, acceptance).
 *   purpose 2, "vertex" b: pair 0 samples the light, pair 1 the phase
 *     function (mu, azimuth); shadow step n uses the first word of pair n+2. */
enum { P_FLIGHT = 1, P_VERTEX = 2 };
/* At most 2^20 pairs per stream: a segment that would need pair 2^20 ends
 * absorbed (free flight) or blocked (shadow).  Valid scenes never come near
 * it. */
#define MAX_PAIRS ((int64_t)1 << 20)
typedef struct { uint32_t key[2]; uint32_t ctr[3]; int64_t block; uint32_t words[4]; } ustream;

static void us_init(ustream* u, uint64_t seed, uint32_t ray, uint32_t sample, uint32_t bounce, uint32_t purpose) {
    u->key[0] = (uint32_t)seed;
    u->key[1] = (uint32_t)(seed >> 32);
    u->ctr[0] = ray;
    u->ctr[1] = sample;
    u->ctr[2] = (bounce << 8) | purpose;
    u->block = -1;
}
static double us_get(ustream* u, int64_t pos) {
    int64_t b = pos / 4;
    if (b != u->block) {
        uint32_t c[4] = {u->ctr[0], u->ctr[1], u->ctr[2], (uint32_t)b};
        orc_philox(c, u->key, u->words);
        u->block = b;
    }
    return orc_uniform(u->words[pos % 4]);
}

/* ------------------------------------------------------------------------ */
/* Medium: trilinear volume sample, transfer-function classification         */
/* ------------------------------------------------------------------------ */
static double voxel(const orc_volume* v, int64_t x, int64_t y, int64_t z) {
    int64_t idx;
    if (v->brick == 8) {
        int64_t nbx = v->nx / 8, nby = v->ny / 8;
        int64_t brick = (x / 8) + nbx * ((y / 8) + nby * (z / 8));
        int64_t inner = (x % 8) + 8 * ((y % 8) + 8 * (z % 8));
        idx = brick * 512 + inner;
    } else {
        idx = x + (int64_t)v->nx * (y + (int64_t)v->ny * z);
    }
    switch (v->type) {
        case ORC_U8: return (double)((const uint8_t*)v->data)[idx];
        case ORC_U16: return (double)((const uint16_t*)v->data)[idx];
        default: return (double)((const float*)v->data)[idx];
    }
}

/* Raw value at world point y: voxel centres at box_min + (idx + 0.5) *
 * extent / n, trilinear weights, coordinates clamped to the edge voxels. */
static double sample_volume(const orc_volume* v, const double y[3]) {
    int64_t n[3] = {v->nx, v->ny, v->nz};
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double g = (y[a] - v->box_min[a]) / (v->box_max[a] - v->box_min[a]) * (double)n[a] - 0.5;
        if (g < 0.0) g = 0.0;
        if (g > (double)(n[a] - 1)) g = (double)(n[a] - 1);
        int64_t b = (int64_t)floor(g);
        if (b > n[a] - 2) b = n[a] - 2;
        i0[a] = b;
        f[a] = g - (double)b;
    }
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wgt = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                s += wgt * voxel(v, i0[0] + dx, i0[1] + dy, i0[2] + dz);
            }
    return s;
}

typedef struct {
    int32_t l0;      /* lower LUT entry */
    double w;        /* weight of entry l0+1 */
    double alpha;    /* interpolated alpha */
    double rgb[3];   /* interpolated colour, before clamping */
} tfsample;

/* Post-classification: normalise the raw value by the window [vmin, vmax],
 * clamp to [0,1], and interpolate the LUT linearly. */
static tfsample classify(const orc_volume* v, const orc_medium* m, double raw) {
    tfsample t;
    double s = (raw - v->vmin) / (v->vmax - v->vmin);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double u = s * (double)(m->lut_size - 1);
    int32_t l0 = (int32_t)floor(u);
    if (l0 > m->lut_size - 2) l0 = m->lut_size - 2;
    t.l0 = l0;
    t.w = u - (double)l0;
    const float* a = m->lut + 4 * l0;
    const float* b = a + 4;
    for (int c = 0; c < 3; ++c) t.rgb[c] = (1.0 - t.w) * (double)a[c] + t.w * (double)b[c];
    t.alpha = (1.0 - t.w) * (double)a[3] + t.w * (double)b[3];
    return t;
}
static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

double orc_majorant(const orc_medium* sample, const orc_params* prm) {
    if (prm->majorant > 0.0) return prm->majorant;
    double amax = 0.0;
    for (int32_t e = 0; e < sample->lut_size; ++e)
        if ((double)sample->lut[4 * e + 3] > amax) amax = (double)sample->lut[4 * e + 3];
    return 1.25 * sample->scale * amax;
}

/* Majorant grid: see lforacle.h for the definition restated here step by
 * step.  Integer floor division for the block bounds (exact on both signs). */
static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

void orc_majorant_grid(const orc_volume* vol, const orc_medium* sample, const orc_params* prm, double* out) {
    const int64_t G = prm->grid;
    const int64_t n[3] = {vol->nx, vol->ny, vol->nz};
    const int32_t L = sample->lut_size;
    const double floor_maj = orc_majorant(sample, prm) / 256.0;
    for (int64_t cz = 0; cz < G; ++cz)
        for (int64_t cy = 0; cy < G; ++cy)
            for (int64_t cx = 0; cx < G; ++cx) {
                const int64_t c[3] = {cx, cy, cz};
                int64_t lo[3], hi[3];
                for (int a = 0; a < 3; ++a) {
                    /* floor(c n / G - 1/2) = floor((2 c n - G) / (2 G)) */
                    lo[a] = floor_div(2 * c[a] * n[a] - G, 2 * G) - 1;
                    hi[a] = floor_div(2 * (c[a] + 1) * n[a] - G, 2 * G) + 2;
                    if (lo[a] < 0) lo[a] = 0;
                    if (hi[a] > n[a] - 1) hi[a] = n[a] - 1;
                }
                double vlo = INFINITY, vhi = -INFINITY;
                for (int64_t z = lo[2]; z <= hi[2]; ++z)
                    for (int64_t y = lo[1]; y <= hi[1]; ++y)
                        for (int64_t x = lo[0]; x <= hi[0]; ++x) {
                            double v = voxel(vol, x, y, z);
                            if (v < vlo) vlo = v;
                            if (v > vhi) vhi = v;
                        }
                double ulo = clamp01((vlo - vol->vmin) / (vol->vmax - vol->vmin)) * (double)(L - 1);
                double uhi = clamp01((vhi - vol->vmin) / (vol->vmax - vol->vmin)) * (double)(L - 1);
                int64_t e0 = (int64_t)floor(ulo), e1 = (int64_t)floor(uhi);
                if (e0 > L - 2) e0 = L - 2;
                if (e1 > L - 2) e1 = L - 2;
                e1 += 1;
                double amax = 0.0;
                for (int64_t e = e0; e <= e1; ++e)
                    if ((double)sample->lut[4 * e + 3] > amax) amax = (double)sample->lut[4 * e + 3];
                double m = 1.25 * sample->scale * amax;
                out[(cz * G + cy) * G + cx] = m > floor_maj ? m : floor_maj;
            }
}

void orc_sigma_at(const orc_volume* vol, const orc_medium* med, const double* pts, int64_t npts, double* out) {
    for (int64_t p = 0; p < npts; ++p) {
        tfsample t = classify(vol, med, sample_volume(vol, pts + 3 * p));
        out[p] = med->scale * t.alpha;
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                           */
/* ------------------------------------------------------------------------ */
/* Parametric interval [tn, tf) of the ray o + t d (t >= 0) inside the box
 * (slab method); returns 0 when the interval is empty. */
static int clip_box(const double o[3], const double d[3], const double bmin[3], const double bmax[3],
                    double* tn, double* tf) {
    double t0 = 0.0, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < bmin[a] || o[a] > bmax[a]) return 0;
            continue;
        }
        double ta = (bmin[a] - o[a]) / d[a];
        double tb = (bmax[a] - o[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t0 < t1)) return 0;
    *tn = t0;
    *tf = t1;
    return 1;
}

/* Orthonormal frame (t1, t2) completing the unit vector n, after Duff et
 * al. 2017, "Building an orthonormal basis, revisited". */
void orc_frame(const double n[3], double t1[3], double t2[3]) {
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + n[2]);
    double b = n[0] * n[1] * a;
    t1[0] = 1.0 + sg * n[0] * n[0] * a; t1[1] = sg * b; t1[2] = -sg * n[0];
    t2[0] = b; t2[1] = sg + n[1] * n[1] * a; t2[2] = -n[1];
}

/* Henyey-Greenstein phase function in terms of mu, the cosine between the
 * propagation direction before and after scattering. */
double orc_hg_phase(double g, double mu) {
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * PI * den * sqrt(den));
}
/* Inversion of the HG cumulative distribution in mu. */
double orc_hg_sample_mu(double g, double u) {
    double mu;
    if (fabs(g) < 1e-3) mu = 1.0 - 2.0 * u;
    else {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    if (mu < -1.0) mu = -1.0;
    if (mu > 1.0) mu = 1.0;
    return mu;
}

/* ------------------------------------------------------------------------ */
/* One path sample (Sec. 2, ray r_k used as camera ray of the path tracer)   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_volume* vol;
    const orc_medium* eval;
    const orc_medium* samp;
    const orc_light* light;
    const orc_params* prm;
    double sigbar;
    int32_t grid;     /* cells per axis of the majorant grid, 0: global sigbar */
    const double* maj;/* [grid^3] cell majorants (shared by the call's threads) */
    int frozen;       /* sample medium differs from eval medium */
    int light_on;     /* light radiance not all zero */
    /* gradient accumulation (NULL in plain forward mode) */
    double* s_alpha;  /* [lut] score: d log / d alpha */
    double* s_rgb;    /* [3][lut] score: d log / d rgb_c */
    double s_scale;
    double* sh_alpha; /* [lut] shadow-ray score */
    double sh_scale;
    double* g_lut;    /* [lut][4] gradient accumulator */
    double g_scale;
    const double* adj;/* [3] adjoint of the current ray's texel, already /spp */
    double stats[4];
} tracer;

/* d(sigma_t)/d(theta) at a classified point, scattered into a score vector
 * with factor c: sigma_t = scale * ((1-w) alpha[l0] + w alpha[l0+1]). */
static void score_sigma(const tracer* tr, double* s_alpha, double* s_scale, const tfsample* t, double c) {
    double scale = tr->eval->scale;
    s_alpha[t->l0] += c * scale * (1.0 - t->w);
    s_alpha[t->l0 + 1] += c * scale * t->w;
    *s_scale += c * t->alpha;
}

/* Add contribution C (RGB) to L, and in gradient mode its derivative
 * C * (sum of scores of the events before it). */
static void contribute(tracer* tr, double L[3], const double C[3], int with_shadow) {
    for (int c = 0; c < 3; ++c) L[c] += C[c];
    if (!tr->g_lut) return;
    int n = tr->eval->lut_size;
    double aC = 0.0;
    for (int c = 0; c < 3; ++c) aC += tr->adj[c] * C[c];
    for (int e = 0; e < n; ++e) {
        double sa = tr->s_alpha[e] + (with_shadow ? tr->sh_alpha[e] : 0.0);
        tr->g_lut[4 * e + 3] += aC * sa;
        for (int c = 0; c < 3; ++c) tr->g_lut[4 * e + c] += tr->adj[c] * C[c] * tr->s_rgb[c * n + e];
    }
    tr->g_scale += aC * (tr->s_scale + (with_shadow ? tr->sh_scale : 0.0));
}

/* Piecewise-constant majorant along a segment.  The segment [tn, tf) of
 * x + t d is cut where it crosses the grid's interior cell planes; each piece
 * carries the majorant of the cell that holds its midpoint.  Without a grid
 * the segment is one piece with the global majorant. */
typedef struct { double t0, t1, maj; } piece;
#define MAX_PIECES (3 * 64 + 2)

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int segment_pieces(const tracer* tr, const double x[3], const double d[3], double tn, double tf,
                          piece* pc) {
    if (tr->grid <= 0) {
        pc[0].t0 = tn; pc[0].t1 = tf; pc[0].maj = tr->sigbar;
        return 1;
    }
    const int64_t G = tr->grid;
    const double* bmin = tr->vol->box_min;
    const double* bmax = tr->vol->box_max;
    double cut[MAX_PIECES];
    int nc = 0;
    cut[nc++] = tn;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        for (int64_t m = 1; m < G; ++m) {
            double plane = bmin[a] + (bmax[a] - bmin[a]) * (double)m / (double)G;
            double t = (plane - x[a]) / d[a];
            if (t > tn && t < tf) cut[nc++] = t;
        }
    }
    qsort(cut + 1, (size_t)(nc - 1), sizeof(double), cmp_double);
    cut[nc++] = tf;
    int np = 0;
    for (int q = 0; q + 1 < nc; ++q) {
        if (!(cut[q + 1] > cut[q])) continue;
        double mid = 0.5 * (cut[q] + cut[q + 1]);
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            double u = (x[a] + mid * d[a] - bmin[a]) / (bmax[a] - bmin[a]) * (double)G;
            int64_t ci = (int64_t)floor(u);
            c[a] = ci < 0 ? 0 : (ci > G - 1 ? G - 1 : ci);
        }
        pc[np].t0 = cut[q];
        pc[np].t1 = cut[q + 1];
        pc[np].maj = tr->maj[(c[2] * G + c[1]) * G + c[0]];
        ++np;
    }
    return np;
}

/* Next tentative point after t for the unit-rate exponential variate tau:
 * tau is spent piece by piece at each piece's majorant (a zero-majorant
 * piece spends none).  Returns 0 when the segment ends first; otherwise sets
 * t and the majorant in force there. */
static int next_tentative(const piece* pc, int np, double* t, double tau, double* maj) {
    for (int p = 0; p < np; ++p) {
        if (pc[p].t1 <= *t) continue;
        double a = pc[p].t0 > *t ? pc[p].t0 : *t;
        if (pc[p].maj > 0.0) {
            double tc = a + tau / pc[p].maj;
            if (tc < pc[p].t1) {
                *t = tc;
                *maj = pc[p].maj;
                return 1;
            }
            tau -= pc[p].maj * (pc[p].t1 - a);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Isosurface variant                                                          */
/* ------------------------------------------------------------------------ */
static double iso_field(const orc_volume* vol, const orc_params* P, const double x[3], const double d[3], double t) {
    double y[3] = {x[0] + t * d[0], x[1] + t * d[1], x[2] + t * d[2]};
    return sample_volume(vol, y) - P->iso;
}

static double half_voxel(const orc_volume* vol) {
    double h = INFINITY;
    int64_t n[3] = {vol->nx, vol->ny, vol->nz};
    for (int a = 0; a < 3; ++a) {
        double e = (vol->box_max[a] - vol->box_min[a]) / (double)n[a];
        if (e < h) h = e;
    }
    return 0.5 * h;
}

int32_t orc_surface_hit(const orc_volume* vol, const orc_params* prm, const double x[3], const double d[3],
                        double t0, double t1, double* thit) {
    const double h = half_voxel(vol);
    double ta = t0, fa = iso_field(vol, prm, x, d, t0);
    for (int64_t m = 1;; ++m) {
        double tb = t0 + (double)m * h;
        if (tb > t1) tb = t1;
        double fb = iso_field(vol, prm, x, d, tb);
        if ((fa >= 0.0) != (fb >= 0.0)) {
            double lo = ta, hi = tb, flo = fa;
            for (int it = 0; it < 40; ++it) {
                double mid = 0.5 * (lo + hi), fm = iso_field(vol, prm, x, d, mid);
                if ((fm >= 0.0) == (flo >= 0.0)) { lo = mid; flo = fm; }
                else hi = mid;
            }
            *thit = lo;  /* the bracket end on the ray's starting side */
            return 1;
        }
        if (tb >= t1) return 0;
        ta = tb;
        fa = fb;
    }
}

/* Unit normal of the surface at y: central differences of f over a quarter
 * voxel, turned to face the incoming direction d (-d where f is flat). */
static void surface_normal(const orc_volume* vol, const double y[3], const double d[3], double n[3]) {
    const double e = 0.5 * half_voxel(vol);
    for (int a = 0; a < 3; ++a) {
        double yp[3] = {y[0], y[1], y[2]}, ym[3] = {y[0], y[1], y[2]};
        yp[a] += e;
        ym[a] -= e;
        n[a] = (sample_volume(vol, yp) - sample_volume(vol, ym)) / (2.0 * e);
    }
    double l = norm3(n);
    if (!(l > 0.0)) {
        for (int a = 0; a < 3; ++a) n[a] = -d[a];
        return;
    }
    for (int a = 0; a < 3; ++a) n[a] /= l;
    if (dot3(n, d) > 0.0)
        for (int a = 0; a < 3; ++a) n[a] = -n[a];
}

/* Surface path: at each vertex the Lambertian BRDF rho / pi with rho the
 * LUT colour at the isovalue (clamped to [0, 1]); next-event estimation
 * towards the light with a visibility ray; a cosine-weighted bounce
 * (weight rho).  Vertex stream b: pair 0 light sample, pair 1 bounce
 * direction.  The vertex is the bracket end on the incoming side, so new
 * rays start on the side the path came from, with no offset. */
static void trace_surface_path(tracer* tr, uint32_t k, uint32_t s, const double x0[3], const double d0[3],
                               double L[3]) {
    const orc_params* P = tr->prm;
    const orc_light* lt = tr->light;
    const orc_volume* vol = tr->vol;
    const double* bmin = vol->box_min;
    const double* bmax = vol->box_max;
    double x[3] = {x0[0], x0[1], x0[2]}, dir[3] = {d0[0], d0[1], d0[2]};
    double T[3] = {1.0, 1.0, 1.0};
    double rho[3];
    {
        tfsample ts = classify(vol, tr->eval, P->iso);
        for (int c = 0; c < 3; ++c) rho[c] = clamp01(ts.rgb[c]);
    }
    L[0] = L[1] = L[2] = 0.0;
    tr->stats[3] += 1.0;
    for (int32_t b = 0; b < P->max_bounces; ++b) {
        double tn, tf, th;
        if (!clip_box(x, dir, bmin, bmax, &tn, &tf) || !orc_surface_hit(vol, P, x, dir, tn, tf, &th)) {
            for (int c = 0; c < 3; ++c) L[c] += T[c] * lt->env[c];
            return;
        }
        tr->stats[2] += 1.0;
        double y[3], n[3];
        for (int a = 0; a < 3; ++a) y[a] = x[a] + th * dir[a];
        surface_normal(vol, y, dir, n);
        ustream uv;
        us_init(&uv, P->seed, k, s, (uint32_t)b, P_VERTEX);
        double ul0 = us_get(&uv, 0), ul1 = us_get(&uv, 1), up0 = us_get(&uv, 2), up1 = us_get(&uv, 3);
        const double* org = y;
        if (tr->light_on) {
            double om[3], Le[3], tend = 0.0;
            if (lt->kind == ORC_LIGHT_DIRECTIONAL) {
                om[0] = lt->dir[0]; om[1] = lt->dir[1]; om[2] = lt->dir[2];
                for (int c = 0; c < 3; ++c) Le[c] = lt->radiance[c];
                double a0, a1;
                if (clip_box(org, om, bmin, bmax, &a0, &a1)) tend = a1;
            } else {
                double yl[3], v[3], nl[3];
                for (int a = 0; a < 3; ++a) yl[a] = lt->corner[a] + ul0 * lt->e1[a] + ul1 * lt->e2[a];
                sub3(yl, org, v);
                double dist = norm3(v);
                for (int a = 0; a < 3; ++a) om[a] = v[a] / dist;
                cross3(lt->e1, lt->e2, nl);
                double area = norm3(nl);
                for (int a = 0; a < 3; ++a) nl[a] /= area;
                double cl = -dot3(nl, om);
                if (cl < 0.0) cl = 0.0;
                for (int c = 0; c < 3; ++c) Le[c] = lt->radiance[c] * cl * area / (dist * dist);
                double a0, a1;
                tend = dist;
                if (clip_box(org, om, bmin, bmax, &a0, &a1)) { if (a1 < tend) tend = a1; }
                else tend = 0.0;
            }
            double cosl = dot3(n, om);
            double tv;
            if (cosl > 0.0 && !(tend > 0.0 && orc_surface_hit(vol, P, org, om, 0.0, tend, &tv)))
                for (int c = 0; c < 3; ++c) L[c] += T[c] * rho[c] / PI * cosl * Le[c];
        }
        if (b == P->max_bounces - 1) return;
        /* cosine-weighted direction about n: weight rho */
        double r = sqrt(up0), ph = 2.0 * PI * up1;
        double t1[3], t2[3];
        orc_frame(n, t1, t2);
        double cz = sqrt(1.0 - up0 > 0.0 ? 1.0 - up0 : 0.0);
        for (int a = 0; a < 3; ++a) dir[a] = r * cos(ph) * t1[a] + r * sin(ph) * t2[a] + cz * n[a];
        normalize3(dir);
        for (int c = 0; c < 3; ++c) T[c] *= rho[c];
        if (T[0] == 0.0 && T[1] == 0.0 && T[2] == 0.0) return;
        for (int a = 0; a < 3; ++a) x[a] = y[a];
    }
}

/* One path sample of stream key k, sample s, from x0 along the unit d0: the
 * path tracer of Sec. 2 (volumetric reading) with the random-number layout
 * described above. */
static void trace_path(tracer* tr, uint32_t k, uint32_t s, const double x0[3], const double d0[3], double L[3]) {
    if (tr->prm->surface) {
        trace_surface_path(tr, k, s, x0, d0, L);
        return;
    }
    const orc_params* P = tr->prm;
    const orc_light* lt = tr->light;
    const double* bmin = tr->vol->box_min;
    const double* bmax = tr->vol->box_max;
    double sigbar = tr->sigbar;   /* majorant in force at the current tentative point */
    double dir[3] = {d0[0], d0[1], d0[2]}, x[3] = {x0[0], x0[1], x0[2]};
    double T[3] = {1.0, 1.0, 1.0};
    double W = 1.0;
    L[0] = L[1] = L[2] = 0.0;
    if (tr->g_lut) {
        int n = tr->eval->lut_size;
        memset(tr->s_alpha, 0, sizeof(double) * n);
        memset(tr->s_rgb, 0, sizeof(double) * 3 * n);
        tr->s_scale = 0.0;
    }
    tr->stats[3] += 1.0;
    for (int32_t b = 0; b < P->max_bounces; ++b) {
        double tn, tf;
        int hit = clip_box(x, dir, bmin, bmax, &tn, &tf);
        int real = 0;
        double y[3];
        tfsample te = {0, 0.0, 0.0, {0.0, 0.0, 0.0}};
        if (hit && tr->sigbar > 0.0) {
            /* delta tracking: tentative collisions at the local majorant
             * rate; the n-th uses pair n (n+1 on the first segment, after
             * the jitter pair): distance variate tau = -ln(1 - u), then
             * acceptance */
            ustream uf;
            us_init(&uf, P->seed, k, s, (uint32_t)b, P_FLIGHT);
            int64_t first = b == 0 ? 1 : 0;
            piece pc[MAX_PIECES];
            int np = segment_pieces(tr, x, dir, tn, tf, pc);
            double t = tn;
            for (int64_t pair = first;; ++pair) {
                if (pair == MAX_PAIRS) return; /* cap reached: absorbed */
                double ud = us_get(&uf, 2 * pair), ua = us_get(&uf, 2 * pair + 1);
                if (!next_tentative(pc, np, &t, -log(1.0 - ud), &sigbar)) break;
                tr->stats[0] += 1.0;
                for (int a = 0; a < 3; ++a) y[a] = x[a] + t * dir[a];
                double raw = sample_volume(tr->vol, y);
                te = classify(tr->vol, tr->eval, raw);
                double sig_e = tr->eval->scale * te.alpha;
                double sig_s = sig_e;
                if (tr->frozen) sig_s = tr->samp->scale * classify(tr->vol, tr->samp, raw).alpha;
                if (ua * sigbar < sig_s) {
                    real = 1;
                    if (tr->frozen) W *= sig_e / sig_s;
                    if (tr->g_lut) score_sigma(tr, tr->s_alpha, &tr->s_scale, &te, 1.0 / sig_e);
                    break;
                }
                if (tr->frozen) W *= (sigbar - sig_e) / (sigbar - sig_s);
                if (tr->g_lut) score_sigma(tr, tr->s_alpha, &tr->s_scale, &te, -1.0 / (sigbar - sig_e));
            }
        }
        if (!real) {
            /* the path leaves the volume: environment radiance */
            double C[3];
            for (int c = 0; c < 3; ++c) C[c] = W * T[c] * lt->env[c];
            contribute(tr, L, C, 0);
            return;
        }
        tr->stats[2] += 1.0;
        x[0] = y[0]; x[1] = y[1]; x[2] = y[2];
        /* real collision: throughput times the single-scattering albedo */
        for (int c = 0; c < 3; ++c) {
            double rho = clamp01(te.rgb[c]);
            T[c] *= rho;
            if (tr->g_lut && te.rgb[c] > 0.0 && te.rgb[c] < 1.0) {
                int n = tr->eval->lut_size;
                tr->s_rgb[c * n + te.l0] += (1.0 - te.w) / rho;
                tr->s_rgb[c * n + te.l0 + 1] += te.w / rho;
            }
        }
        if (T[0] == 0.0 && T[1] == 0.0 && T[2] == 0.0) return;
        ustream uv;
        us_init(&uv, P->seed, k, s, (uint32_t)b, P_VERTEX);
        double ul0 = us_get(&uv, 0), ul1 = us_get(&uv, 1), up0 = us_get(&uv, 2), up1 = us_get(&uv, 3);
        /* next-event estimation towards the light, ratio-tracking
         * transmittance (product of 1 - sigma_t / sigbar at tentative points) */
        if (tr->light_on) {
            double om[3], Le[3], tend = 0.0;
            if (lt->kind == ORC_LIGHT_DIRECTIONAL) {
                om[0] = lt->dir[0]; om[1] = lt->dir[1]; om[2] = lt->dir[2];
                for (int c = 0; c < 3; ++c) Le[c] = lt->radiance[c];
                double a0, a1;
                if (clip_box(x, om, bmin, bmax, &a0, &a1)) tend = a1;
            } else {
                double yl[3], v[3], nl[3];
                for (int a = 0; a < 3; ++a) yl[a] = lt->corner[a] + ul0 * lt->e1[a] + ul1 * lt->e2[a];
                sub3(yl, x, v);
                double dist = norm3(v);
                for (int a = 0; a < 3; ++a) om[a] = v[a] / dist;
                cross3(lt->e1, lt->e2, nl);
                double area = norm3(nl);
                for (int a = 0; a < 3; ++a) nl[a] /= area;
                double cl = -dot3(nl, om);
                if (cl < 0.0) cl = 0.0;
                for (int c = 0; c < 3; ++c) Le[c] = lt->radiance[c] * cl * area / (dist * dist);
                double a0, a1;
                tend = dist;
                if (clip_box(x, om, bmin, bmax, &a0, &a1)) { if (a1 < tend) tend = a1; }
                else tend = 0.0;
            }
            double Tr = 1.0;
            if (tr->g_lut) {
                memset(tr->sh_alpha, 0, sizeof(double) * tr->eval->lut_size);
                tr->sh_scale = 0.0;
            }
            if (tr->sigbar > 0.0) {
                double t = 0.0;
                piece pc[MAX_PIECES];
                int np = segment_pieces(tr, x, om, 0.0, tend, pc);
                for (int64_t pair = 2;; ++pair) {
                    if (pair == MAX_PAIRS) { Tr = 0.0; break; } /* cap reached: blocked */
                    if (!next_tentative(pc, np, &t, -log(1.0 - us_get(&uv, 2 * pair)), &sigbar)) break;
                    tr->stats[1] += 1.0;
                    double z[3];
                    for (int a = 0; a < 3; ++a) z[a] = x[a] + t * om[a];
                    tfsample ts = classify(tr->vol, tr->eval, sample_volume(tr->vol, z));
                    double sig = tr->eval->scale * ts.alpha;
                    Tr *= 1.0 - sig / sigbar;
                    if (tr->g_lut) score_sigma(tr, tr->sh_alpha, &tr->sh_scale, &ts, -1.0 / (sigbar - sig));
                }
            }
            double fp = orc_hg_phase(P->g, dot3(dir, om));
            double C[3];
            for (int c = 0; c < 3; ++c) C[c] = W * T[c] * fp * Le[c] * Tr;
            contribute(tr, L, C, 1);
        }
        if (b == P->max_bounces - 1) return;
        /* sample the next direction from the phase function */
        double mu = orc_hg_sample_mu(P->g, up0);
        double ph = 2.0 * PI * up1;
        double st = sqrt(1.0 - mu * mu > 0.0 ? 1.0 - mu * mu : 0.0);
        double t1[3], t2[3], nd[3];
        orc_frame(dir, t1, t2);
        for (int a = 0; a < 3; ++a) nd[a] = st * cos(ph) * t1[a] + st * sin(ph) * t2[a] + mu * dir[a];
        dir[0] = nd[0]; dir[1] = nd[1]; dir[2] = nd[2];
    }
}

/* Ray r_k of the SF ray set (Sec. 2, ray equation), sample s. */
static void trace_sample(tracer* tr, uint32_t k, int64_t i, int64_t j, uint32_t s, double L[3]) {
    const orc_params* P = tr->prm;
    double po[3], pd[3], dir[3], x[3];
    orc_sf_point(P->M, i, po);
    orc_sf_point(P->N, j, pd);
    /* d_ij = p^d_j - p^o_i, normalised (Sec. 2, ray equation) */
    sub3(pd, po, dir);
    normalize3(dir);
    /* ray origin O + R p^o_i, jittered on a disk of area A_S / M = 4 pi R^2 / M
     * (radius 2R / sqrt M) in the tangent plane of S at p^o_i */
    for (int a = 0; a < 3; ++a) x[a] = P->center[a] + P->radius * po[a];
    if (P->jitter) {
        ustream uj;
        us_init(&uj, P->seed, k, s, 0, P_FLIGHT);
        double u0 = us_get(&uj, 0), u1 = us_get(&uj, 1);
        double rho = 2.0 * P->radius / sqrt((double)P->M) * sqrt(u0);
        double ang = 2.0 * PI * u1;
        double t1[3], t2[3];
        orc_frame(po, t1, t2);
        for (int a = 0; a < 3; ++a) x[a] += rho * (cos(ang) * t1[a] + sin(ang) * t2[a]);
    }
    trace_path(tr, k, s, x, dir, L);
}

/* ------------------------------------------------------------------------ */
/* Thread pool over ray chunks                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    tracer tr;
    const int64_t* rays;
    int64_t r0, r1;
    double* out;             /* generate */
    const double* adj;       /* gradient */
    double* g_lut;           /* per-thread gradient */
} job;

/* The majorant grid of a call is built once and shared by its threads. */
static double* build_grid(const orc_volume* vol, const orc_medium* eval, const orc_medium* sample,
                          const orc_params* prm) {
    if (prm->majorant > 0.0 || prm->grid <= 0) return NULL;
    size_t G = (size_t)prm->grid;
    double* maj = (double*)malloc(sizeof(double) * G * G * G);
    orc_majorant_grid(vol, sample ? sample : eval, prm, maj);
    return maj;
}

static void tracer_setup(tracer* tr, const orc_volume* vol, const orc_medium* eval,
                         const orc_medium* sample, const orc_light* light, const orc_params* prm,
                         double* maj) {
    memset(tr, 0, sizeof(*tr));
    tr->vol = vol;
    tr->eval = eval;
    tr->samp = sample ? sample : eval;
    tr->light = light;
    tr->prm = prm;
    tr->sigbar = orc_majorant(tr->samp, prm);
    tr->grid = maj ? prm->grid : 0;
    tr->maj = maj;
    tr->frozen = sample != NULL && sample != eval;
    tr->light_on = light->radiance[0] != 0.0 || light->radiance[1] != 0.0 || light->radiance[2] != 0.0;
}

static void* gen_worker(void* arg) {
    job* jb = (job*)arg;
    const orc_params* P = jb->tr.prm;
    for (int64_t r = jb->r0; r < jb->r1; ++r) {
        int64_t kk = jb->rays[r];
        int64_t i = kk / P->N, j = kk % P->N;
        double acc[3] = {0.0, 0.0, 0.0};
        /* a ray whose adjoint is zero adds nothing to the gradient */
        if (jb->g_lut && jb->adj[3 * r] == 0.0 && jb->adj[3 * r + 1] == 0.0 && jb->adj[3 * r + 2] == 0.0)
            continue;
        /* with P_o = P_d (M == N) the ray from p_i to p_i has no direction:
         * its texel is defined as 0 */
        if (!(P->M == P->N && i == j)) {
            for (int32_t s = 0; s < P->spp; ++s) {
                double L[3];
                if (jb->g_lut) {
                    double a[3];
                    for (int c = 0; c < 3; ++c) a[c] = jb->adj[3 * r + c] / (double)P->spp;
                    jb->tr.adj = a;
                    trace_sample(&jb->tr, (uint32_t)kk, i, j, (uint32_t)s, L);
                } else {
                    trace_sample(&jb->tr, (uint32_t)kk, i, j, (uint32_t)s, L);
                }
                for (int c = 0; c < 3; ++c) acc[c] += L[c];
            }
        }
        if (jb->out)
            for (int c = 0; c < 3; ++c) jb->out[3 * r + c] = acc[c] / (double)P->spp;
    }
    return NULL;
}

static void run_jobs(job* jobs, int32_t nthreads) {
    if (nthreads <= 1) { gen_worker(&jobs[0]); return; }
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, gen_worker, &jobs[t]);
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
}

void orc_generate(const orc_volume* vol, const orc_medium* eval, const orc_medium* sample,
                  const orc_light* light, const orc_params* prm, const int64_t* rays, int64_t nrays,
                  double* out, int32_t nthreads, double* stats) {
    if (nthreads < 1) nthreads = 1;
    double* maj = build_grid(vol, eval, sample, prm);
    job* jobs = (job*)calloc((size_t)nthreads, sizeof(job));
    for (int32_t t = 0; t < nthreads; ++t) {
        tracer_setup(&jobs[t].tr, vol, eval, sample, light, prm, maj);
        jobs[t].rays = rays;
        jobs[t].r0 = nrays * t / nthreads;
        jobs[t].r1 = nrays * (t + 1) / nthreads;
        jobs[t].out = out;
    }
    run_jobs(jobs, nthreads);
    free(maj);
    if (stats) {
        for (int a = 0; a < 4; ++a) stats[a] = 0.0;
        for (int32_t t = 0; t < nthreads; ++t)
            for (int a = 0; a < 4; ++a) stats[a] += jobs[t].tr.stats[a];
    }
    free(jobs);
}

void orc_gradient(const orc_volume* vol, const orc_medium* med, const orc_light* light,
                  const orc_params* prm, const int64_t* rays, int64_t nrays, const double* adj,
                  double* d_lut, double* d_scale, int32_t nthreads) {
    if (nthreads < 1) nthreads = 1;
    int n = med->lut_size;
    double* maj = build_grid(vol, med, NULL, prm);
    job* jobs = (job*)calloc((size_t)nthreads, sizeof(job));
    for (int32_t t = 0; t < nthreads; ++t) {
        tracer_setup(&jobs[t].tr, vol, med, NULL, light, prm, maj);
        jobs[t].tr.s_alpha = (double*)calloc((size_t)n, sizeof(double));
        jobs[t].tr.s_rgb = (double*)calloc((size_t)3 * n, sizeof(double));
        jobs[t].tr.sh_alpha = (double*)calloc((size_t)n, sizeof(double));
        jobs[t].tr.g_lut = (double*)calloc((size_t)4 * n, sizeof(double));
        jobs[t].g_lut = jobs[t].tr.g_lut;
        jobs[t].rays = rays;
        jobs[t].adj = adj;
        jobs[t].r0 = nrays * t / nthreads;
        jobs[t].r1 = nrays * (t + 1) / nthreads;
        jobs[t].out = NULL;
    }
    run_jobs(jobs, nthreads);
    for (int e = 0; e < 4 * n; ++e) d_lut[e] = 0.0;
    *d_scale = 0.0;
    for (int32_t t = 0; t < nthreads; ++t) {
        for (int e = 0; e < 4 * n; ++e) d_lut[e] += jobs[t].tr.g_lut[e];
        *d_scale += jobs[t].tr.g_scale;
        free(jobs[t].tr.s_alpha);
        free(jobs[t].tr.s_rgb);
        free(jobs[t].tr.sh_alpha);
        free(jobs[t].tr.g_lut);
    }
    free(maj);
    free(jobs);
}

/* ------------------------------------------------------------------------ */
/* Lookup (Sec. 2, image synthesis by sampling Lhat(i,j))                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int ok;
    int64_t ia[9], jb[9];
    double wa[9], wb[9];
    int na, nb;
    double margin[4];
} pixel_query;

/* Pinhole camera ray through the centre of pixel (x, y), row 0 at the top;
 * front and back hit points on S (tangential rays, with b^2 - c <= 1e-6 R^2,
 * are discarded); nearest and K neighbours of each hit point in its set. */
/* Unit direction of the pinhole ray through the centre of pixel (px, py). */
static void camera_dir(const orc_camera* cam, int32_t W, int32_t H, int32_t px, int32_t py, double d[3]) {
    double fwd[3], right[3], up[3];
    sub3(cam->target, cam->eye, fwd);
    normalize3(fwd);
    cross3(fwd, cam->up, right);
    normalize3(right);
    cross3(right, fwd, up);
    double th = tan(0.5 * cam->vfov);
    double aspect = (double)W / (double)H;
    double sx = (2.0 * ((double)px + 0.5) / (double)W - 1.0) * th * aspect;
    double sy = (1.0 - 2.0 * ((double)py + 0.5) / (double)H) * th;
    for (int a = 0; a < 3; ++a) d[a] = fwd[a] + sx * right[a] + sy * up[a];
    normalize3(d);
}

static void query_pixel(const orc_params* P, const orc_camera* cam, int32_t W, int32_t H, int32_t K,
                        int32_t px, int32_t py, pixel_query* q) {
    double d[3];
    camera_dir(cam, W, H, px, py, d);
    double oc[3];
    sub3(cam->eye, P->center, oc);
    double b = dot3(d, oc);
    double c = dot3(oc, oc) - P->radius * P->radius;
    double disc = b * b - c;
    double thr = 1e-6 * P->radius * P->radius;
    for (int a = 0; a < 4; ++a) q->margin[a] = 1e300;
    q->margin[0] = fabs(disc - thr) / (P->radius * P->radius);
    q->ok = disc > thr;
    if (!q->ok) return;
    double sq = sqrt(disc);
    double ho[3], hd[3], qo[3], qd[3];
    for (int a = 0; a < 3; ++a) {
        ho[a] = cam->eye[a] + (-b - sq) * d[a];
        hd[a] = cam->eye[a] + (-b + sq) * d[a];
    }
    sub3(ho, P->center, qo);
    normalize3(qo);
    sub3(hd, P->center, qd);
    normalize3(qd);
    double mo[3], md[3], d2[9];
    q->na = orc_neighbors(P->M, qo, K, q->ia, q->wa, d2, mo);
    q->nb = orc_neighbors(P->N, qd, K, q->jb, q->wb, d2, md);
    /* the gaps are in squared unit-sphere distance; express them relative to
     * each set's area per point so one tolerance fits every n */
    double ao = 4.0 * PI / (double)P->M, ad = 4.0 * PI / (double)P->N;
    q->margin[1] = fmin(mo[0] / ao, md[0] / ad);
    q->margin[2] = fmin(mo[1], md[1]);
    q->margin[3] = fmin(mo[2] / ao, md[2] / ad);
}

static int64_t stored_rows(const orc_params* P) { return P->origin_rows > 0 ? P->origin_rows : P->M; }

/* Normalised pair weights w_o(a) w_d(b) / sum; pairs with a == b are the
 * undefined texels of P_o = P_d and get weight 0, and so do origins that are
 * not stored.  K = 1 is nearest sampling: the single texel, unweighted, if
 * its origin is stored. */
static int pair_weights(const orc_params* P, int32_t K, const pixel_query* q, double* wab) {
    const int64_t rows = stored_rows(P);
    if (K == 1) { wab[0] = 1.0; return q->ia[0] < rows; }
    double sum = 0.0;
    for (int a = 0; a < q->na; ++a)
        for (int b = 0; b < q->nb; ++b) {
            double w = q->wa[a] * q->wb[b];
            if (P->M == P->N && q->ia[a] == q->jb[b]) w = 0.0;
            if (q->ia[a] >= rows) w = 0.0;
            wab[a * 9 + b] = w;
            sum += w;
        }
    if (!(sum > 0.0)) return 0;
    for (int a = 0; a < q->na; ++a)
        for (int b = 0; b < q->nb; ++b) wab[a * 9 + b] /= sum;
    return 1;
}

typedef struct {
    const float* lf; const orc_params* P; const orc_camera* cams; int32_t W, H, K;
    const int32_t* pix; int64_t p0, p1; double* rgb; int64_t* nn; double* margin;
} lookup_job;

static void* lookup_worker(void* arg) {
    lookup_job* jb = (lookup_job*)arg;
    const orc_params* P = jb->P;
    for (int64_t p = jb->p0; p < jb->p1; ++p) {
        const int32_t* px = jb->pix + 3 * p;
        pixel_query q;
        query_pixel(P, &jb->cams[px[0]], jb->W, jb->H, jb->K, px[1], px[2], &q);
        double out[3] = {0.0, 0.0, 0.0};
        double wab[81];
        if (jb->margin)
            for (int a = 0; a < 4; ++a) jb->margin[4 * p + a] = q.margin[a];
        if (!q.ok) {
            if (jb->nn) { jb->nn[2 * p] = -1; jb->nn[2 * p + 1] = -1; }
        } else {
            if (jb->nn) { jb->nn[2 * p] = q.ia[0]; jb->nn[2 * p + 1] = q.jb[0]; }
            if (pair_weights(P, jb->K, &q, wab)) {
                for (int a = 0; a < q.na; ++a)
                    for (int b = 0; b < q.nb; ++b) {
                        if (wab[a * 9 + b] == 0.0) continue;
                        const float* t = jb->lf + 3 * (q.ia[a] * P->N + q.jb[b]);
                        for (int c = 0; c < 3; ++c) out[c] += wab[a * 9 + b] * (double)t[c];
                    }
            }
        }
        for (int c = 0; c < 3; ++c) jb->rgb[3 * p + c] = out[c];
    }
    return NULL;
}

void orc_lookup(const float* lf, const orc_params* prm, const orc_camera* cams, int32_t W, int32_t H,
                int32_t K, const int32_t* pix, int64_t npx, double* rgb, int64_t* nn, double* margin,
                int32_t nthreads) {
    if (nthreads < 1) nthreads = 1;
    lookup_job* jobs = (lookup_job*)calloc((size_t)nthreads, sizeof(lookup_job));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        lookup_job j = {lf, prm, cams, W, H, K, pix, npx * t / nthreads, npx * (t + 1) / nthreads, rgb, nn, margin};
        jobs[t] = j;
        pthread_create(&th[t], NULL, lookup_worker, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}

void orc_lookup_adjoint(const orc_params* prm, const orc_camera* cams, int32_t W, int32_t H, int32_t K,
                        const int32_t* pix, int64_t npx, const double* dimg, double* d_lf) {
    for (int64_t p = 0; p < npx; ++p) {
        const int32_t* px = pix + 3 * p;
        pixel_query q;
        query_pixel(prm, &cams[px[0]], W, H, K, px[1], px[2], &q);
        if (!q.ok) continue;
        double wab[81];
        if (!pair_weights(prm, K, &q, wab)) continue;
        for (int a = 0; a < q.na; ++a)
            for (int b = 0; b < q.nb; ++b) {
                if (wab[a * 9 + b] == 0.0) continue;
                double* t = d_lf + 3 * (q.ia[a] * prm->N + q.jb[b]);
                for (int c = 0; c < 3; ++c) t[c] += wab[a * 9 + b] * dimg[3 * p + c];
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Ground-truth views: the same path tracer along pinhole camera rays         */
/* ------------------------------------------------------------------------ */
typedef struct {
    tracer tr;
    const orc_camera* cams; int32_t W, H; const int32_t* pix; int64_t p0, p1; double* rgb;
} render_job;

static void* render_worker(void* arg) {
    render_job* jb = (render_job*)arg;
    const orc_params* P = jb->tr.prm;
    for (int64_t p = jb->p0; p < jb->p1; ++p) {
        const int32_t* px = jb->pix + 3 * p;
        const orc_camera* cam = &jb->cams[px[0]];
        double d[3], acc[3] = {0.0, 0.0, 0.0};
        camera_dir(cam, jb->W, jb->H, px[1], px[2], d);
        /* stream key: the pixel's index in the [view][row][column] image */
        uint32_t k = (uint32_t)(((int64_t)px[0] * jb->H + px[2]) * jb->W + px[1]);
        for (int32_t s = 0; s < P->spp; ++s) {
            double L[3];
            trace_path(&jb->tr, k, (uint32_t)s, cam->eye, d, L);
            for (int c = 0; c < 3; ++c) acc[c] += L[c];
        }
        for (int c = 0; c < 3; ++c) jb->rgb[3 * p + c] = acc[c] / (double)P->spp;
    }
    return NULL;
}

void orc_render(const orc_volume* vol, const orc_medium* med, const orc_light* light, const orc_params* prm,
                const orc_camera* cams, int32_t W, int32_t H, const int32_t* pix, int64_t npx, double* rgb,
                int32_t nthreads) {
    if (nthreads < 1) nthreads = 1;
    double* maj = build_grid(vol, med, NULL, prm);
    render_job* jobs = (render_job*)calloc((size_t)nthreads, sizeof(render_job));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        tracer_setup(&jobs[t].tr, vol, med, NULL, light, prm, maj);
        jobs[t].cams = cams;
        jobs[t].W = W;
        jobs[t].H = H;
        jobs[t].pix = pix;
        jobs[t].p0 = npx * t / nthreads;
        jobs[t].p1 = npx * (t + 1) / nthreads;
        jobs[t].rgb = rgb;
        pthread_create(&th[t], NULL, render_worker, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    free(maj);
}

/* ------------------------------------------------------------------------ */
/* Mean SSIM (Wang, Bovik, Sheikh, Simoncelli 2004) as defined: windowed     */
/* means, variances and covariance with the 11 x 11 Gaussian window of sigma  */
/* 1.5 (sum 1), at every window position inside the image, per channel.      */
/* ------------------------------------------------------------------------ */
void orc_ssim(const float* a, const float* b, int32_t n, int32_t W, int32_t H, double data_range, double* out) {
    double g[11], gs = 0.0;
    for (int t = 0; t < 11; ++t) {
        g[t] = exp(-(double)((t - 5) * (t - 5)) / (2.0 * 1.5 * 1.5));
        gs += g[t];
    }
    for (int t = 0; t < 11; ++t) g[t] /= gs;
    const double c1 = (0.01 * data_range) * (0.01 * data_range);
    const double c2 = (0.03 * data_range) * (0.03 * data_range);
    for (int32_t m = 0; m < n; ++m) {
        const float* A = a + (size_t)m * H * W * 3;
        const float* B = b + (size_t)m * H * W * 3;
        double total = 0.0;
        for (int c = 0; c < 3; ++c)
            for (int32_t y = 0; y + 10 < H; ++y)
                for (int32_t x = 0; x + 10 < W; ++x) {
                    double ma = 0.0, mb = 0.0, aa = 0.0, bb = 0.0, ab = 0.0;
                    for (int v = 0; v < 11; ++v)
                        for (int u = 0; u < 11; ++u) {
                            double w = g[v] * g[u];
                            size_t o = ((size_t)(y + v) * W + (x + u)) * 3 + c;
                            double va = A[o], vb = B[o];
                            ma += w * va;
                            mb += w * vb;
                            aa += w * va * va;
                            bb += w * vb * vb;
                            ab += w * va * vb;
                        }
                    double sa = aa - ma * ma, sb = bb - mb * mb, sab = ab - ma * mb;
                    total += ((2.0 * ma * mb + c1) * (2.0 * sab + c2)) /
                             ((ma * ma + mb * mb + c1) * (sa + sb + c2));
                }
        out[m] = total / (3.0 * (double)(W - 10) * (double)(H - 10));
    }
}

/* ------------------------------------------------------------------------ */
/* Batched neighbour queries (threads over queries; each one is the plain     */
/* brute-force query above).                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n; const double* q; int64_t q0, q1; int32_t K;
    int64_t* idx; double* w; double* d2; double* margins; int32_t* count;
} nb_job;

static void* nb_worker(void* arg) {
    nb_job* jb = (nb_job*)arg;
    for (int64_t t = jb->q0; t < jb->q1; ++t) {
        int64_t idx[9];
        double w[9], d2[9], m[3];
        int32_t c = orc_neighbors(jb->n, jb->q + 3 * t, jb->K, idx, w, d2, m);
        for (int32_t a = 0; a < jb->K; ++a) {
            jb->idx[t * jb->K + a] = a < c ? idx[a] : -1;
            jb->w[t * jb->K + a] = a < c ? w[a] : 0.0;
            jb->d2[t * jb->K + a] = a < c ? d2[a] : 0.0;
        }
        for (int a = 0; a < 3; ++a) jb->margins[3 * t + a] = m[a];
        jb->count[t] = c;
    }
    return NULL;
}

void orc_neighbors_batch(int64_t n, const double* q, int64_t nq, int32_t K, int64_t* idx, double* w,
                         double* d2, double* margins, int32_t* count, int32_t nthreads) {
    if (nthreads < 1) nthreads = 1;
    nb_job* jobs = (nb_job*)calloc((size_t)nthreads, sizeof(nb_job));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int32_t t = 0; t < nthreads; ++t) {
        nb_job j = {n, q, nq * t / nthreads, nq * (t + 1) / nthreads, K, idx, w, d2, margins, count};
        jobs[t] = j;
        pthread_create(&th[t], NULL, nb_worker, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}
