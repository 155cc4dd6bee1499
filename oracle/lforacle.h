/*
 * lforacle.h -- plain FP64 CPU oracle for the LumiPath light-field path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU product path never calls it and shares no code, header or table with
 * it.  Everything is computed in double precision from the definitions in
 * Fink et al., "LumiPath -- Towards Real-time Physically-based Rendering on
 * Embedded Devices" (arXiv 1903.03837); where the paper is silent, the
 * reading taken is stated beside the function that takes it.
 *
 * Parity status of each function (what pins it) is stated beside it.
 */
#ifndef LFORACLE_H
#define LFORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Voxel storage types and layouts (inputs, not part of the paper). */
enum { ORC_U8 = 0, ORC_U16 = 1, ORC_F32 = 2 };
enum { ORC_LIGHT_DIRECTIONAL = 0, ORC_LIGHT_AREA = 1 };

typedef struct {
    const void* data;       /* host voxel array */
    int32_t type;           /* ORC_U8 / ORC_U16 / ORC_F32 */
    int32_t nx, ny, nz;     /* each >= 2 */
    int32_t brick;          /* 0: x-fastest linear; 8: 8^3 bricks, brick-major */
    double vmin, vmax;      /* raw-value window mapped onto the LUT */
    double box_min[3], box_max[3];
} orc_volume;

typedef struct {
    const float* lut;       /* [lut_size][4] RGBA, host */
    int32_t lut_size;       /* >= 2 */
    double scale;           /* density scale: sigma_t = scale * alpha */
} orc_medium;

typedef struct {
    int32_t kind;           /* ORC_LIGHT_DIRECTIONAL or ORC_LIGHT_AREA */
    double dir[3];          /* directional: unit vector towards the light */
    double corner[3], e1[3], e2[3]; /* area: parallelogram corner + edges;
                                       emits on the side of cross(e1,e2) */
    double radiance[3];     /* directional: irradiance; area: radiance */
    double env[3];          /* constant environment radiance for escapes */
} orc_light;

typedef struct {
    int64_t M, N;           /* origin / direction point-set sizes */
    double center[3];       /* O */
    double radius;          /* R */
    int32_t spp, max_bounces;
    double g;               /* Henyey-Greenstein asymmetry, |g| < 1 */
    double majorant;        /* <= 0: 1.25 * scale * max alpha of the sampling medium */
    uint64_t seed;
    int32_t jitter;         /* 1: jitter ray origins on the disk of area 4 pi R^2 / M */
    int32_t grid;           /* majorant grid: G cells per axis (0: one global
                               majorant); ignored when majorant > 0 */
    int32_t surface;        /* 1: isosurface variant (the volume's trilinear
                               field at raw value iso is an opaque Lambertian
                               surface); 0: participating medium */
    double iso;             /* isovalue of the surface variant (raw units) */
    int64_t origin_rows;    /* origins i < origin_rows are stored (0: all M); the
                               light field is [origin_rows][N][3] (Sec. 3 keeps the
                               upper hemisphere, origin_rows = M / 2) */
} orc_params;

typedef struct {
    double eye[3], target[3], up[3];
    double vfov;            /* vertical field of view, radians */
} orc_camera;

/* ---- Spherical Fibonacci point set (Sec. 2, SF point equation) ----------
 * Pinned by: z-coordinate identity, sum of z = 0, unit norm, hemisphere
 * split, and a golden-ratio-free recomputation of frac(i / Phi). */
void orc_sf_point(int64_t n, int64_t i, double p[3]);
void orc_sf_points(int64_t n, double* xyz /* [n][3] */);

/* ---- Nearest SF point: argmin_i |q - p_i|^2, ties to the lower index ----
 * (Sec. 2, image synthesis: nearest-neighbour query of a hit point).
 * Brute force over all n points.  Returns i*, the best and second-best
 * squared distances.  Pinned by: every p_i maps to itself, jittered points
 * map back, poles, seam. */
int64_t orc_nearest(int64_t n, const double q[3], double* d2_best, double* d2_second);

/* Zone number of the Fibonacci lattice at height qz (inverse SF mapping of
 * Keinert et al. 2015, cited in Sec. 2): k = max(2, floor(log_{Phi^2}(n pi
 * sqrt5 (1 - qz^2)))).  *margin receives the distance of the log value to
 * the nearest integer >= 3 (how close the floor is to flipping). */
int32_t orc_zone(int64_t n, double qz, double* margin);
int64_t orc_fib(int32_t k);

/* ---- K-neighbour query with filter weights (Sec. 2, "up to nine
 * neighbors", filter kernel of size R sqrt(4 pi / N)) ----------------------
 * Candidates: i* + {0, +-F(k-1), +-F(k), +-F(k+1), +-F(k+2)} inside [0,n),
 * duplicates dropped; keep the K nearest by (distance^2, index).
 * w = max(0, 1 - d / sqrt(4 pi / n)) with d the unit-sphere chord.
 * Returns the number of neighbours written (<= K).  margins[0] = nearest gap
 * (second - best squared distance), margins[1] = zone margin, margins[2] =
 * squared-distance gap between the K-th and (K+1)-th candidate (1e300 when
 * there is none). */
int32_t orc_neighbors(int64_t n, const double q[3], int32_t K,
                      int64_t* idx, double* w, double* d2, double margins[3]);

/* The same query for nq points q[3*t..] (threads over queries): idx, w, d2
 * are [nq][K] (-1 / 0 past the count), margins [nq][3], count [nq]. */
void orc_neighbors_batch(int64_t n, const double* q, int64_t nq, int32_t K, int64_t* idx, double* w,
                         double* d2, double* margins, int32_t* count, int32_t nthreads);

/* ---- Philox4x32-10 counter-based generator (Salmon et al., SC'11) ------
 * Pinned against rocRAND's independent implementation. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 24-bit uniform on [0,1): (x >> 8) * 2^-24, exact in binary32 and binary64 */
double orc_uniform(uint32_t x);

/* ---- Scattering helpers (exposed for their pins) -----------------------
 * orc_hg_phase: Henyey-Greenstein phase function of mu = cos(angle between
 * propagation directions); pinned by unit normalisation and isotropy at g=0.
 * orc_hg_sample_mu: inversion of its cumulative distribution; pinned by the
 * mean cosine g and the histogram of the phase function.
 * orc_frame: orthonormal completion (t1, t2) of a unit n (Duff et al. 2017);
 * pinned by orthonormality and handedness. */
double orc_hg_phase(double g, double mu);
double orc_hg_sample_mu(double g, double u);
void orc_frame(const double n[3], double t1[3], double t2[3]);

/* ---- Isosurface variant (the paper renders segmented surfaces) ----------
 * Surface: where the trilinear raw field f crosses prm->iso.  The first
 * crossing along x + t d in [t0, t1): f - iso is sampled at t0 + m h
 * (m = 0, 1, ...; the last sample at t1), h = half the smallest voxel
 * extent; the first pair of consecutive samples whose signs differ (a zero
 * counts as positive) is bisected 40 times, and the end of the final
 * bracket on the starting side is returned (so a path continues on the side
 * it came from).
 * Returns 0 when no pair changes sign.  Pinned by a sphere of a radial
 * field (analytic hit distance) and by exact white-furnace energy. */
int32_t orc_surface_hit(const orc_volume* vol, const orc_params* prm, const double x[3], const double d[3],
                        double t0, double t1, double* thit);

/* ---- Majorant: params majorant if > 0 else 1.25 * scale * max alpha ---- */
double orc_majorant(const orc_medium* sample, const orc_params* prm);

/* ---- Majorant grid (piecewise-constant majorant of delta and ratio
 * tracking, as in PBRT's grid media) -------------------------------------
 * G = prm->grid (1..64) splits the volume box into G^3 equal cells, x
 * fastest.  Cell c must bound sigma_t of the sampling medium wherever the
 * trilinear footprint of a point in it can reach, with one voxel to spare
 * on each side: per axis, voxels floor(c n / G - 1/2) - 1 ..
 * floor((c + 1) n / G - 1/2) + 2, clamped to the grid.  [lo, hi] is the raw
 * range of that block, u(v) = clamp((v - vmin) / (vmax - vmin), 0, 1) (L-1),
 * and the LUT entries min(floor u(lo), L-2) .. min(floor u(hi), L-2) + 1
 * hold every alpha a point of the cell can take; the majorant is
 * max(1.25 scale max alpha over them, orc_majorant / 256).  The floor keeps
 * null collisions, and so the score of every LUT entry, possible in empty
 * cells.  Pinned by brute-force sampling of sigma_t, a constant volume
 * (closed form) and the floor in empty space. */
void orc_majorant_grid(const orc_volume* vol, const orc_medium* sample, const orc_params* prm, double* out);

/* sigma_t = scale * alpha of `med` at npts world points pts[3p..] (trilinear
 * raw value, classification); exposed for the pins above. */
void orc_sigma_at(const orc_volume* vol, const orc_medium* med, const double* pts, int64_t npts, double* out);

/* ---- Light-field generation (Sec. 2, ray set R^K, origin jitter, path
 * tracer; volumetric reading) ---------------------------------------------
 * For each ray index k = i*N + j in rays[0..nrays) writes the mean radiance
 * over spp samples to out[3*r .. 3*r+2].  `sample` may equal `eval`; when it
 * differs, collisions are decided with `sample` and importance-weighted to
 * `eval` (frozen sampling).  With prm->grid > 0 (and no fixed majorant)
 * both trackings use the majorant grid above.  With prm->surface the path
 * runs on the isosurface instead (see orc_surface_hit; frozen sampling and
 * gradients do not apply).  Pinned by Beer-Lambert,
 * white furnace, vacuum, linearity and symmetry checks, and, for the grid,
 * by quadrature of heterogeneous transmittance and agreement in expectation
 * with the global majorant.  stats (may be NULL) receives
 * [tentative collisions of primary tracking, shadow steps, real collisions,
 * samples]. */
void orc_generate(const orc_volume* vol, const orc_medium* eval,
                  const orc_medium* sample, const orc_light* light,
                  const orc_params* prm, const int64_t* rays, int64_t nrays,
                  double* out, int32_t nthreads, double* stats);

/* ---- Gradient of sum_r adj[r] . Lhat(rays[r]) with respect to the LUT and
 * the density scale, for the fixed random stream (score terms of the
 * estimator, forward mode).  d_lut: [lut_size][4], d_scale: [1]; both
 * overwritten.  Pinned by central differences of orc_generate in frozen
 * sampling and by the closed-form Beer-Lambert derivative. */
void orc_gradient(const orc_volume* vol, const orc_medium* med,
                  const orc_light* light, const orc_params* prm,
                  const int64_t* rays, int64_t nrays, const double* adj,
                  double* d_lut, double* d_scale, int32_t nthreads);

/* ---- Lookup of view rays (Sec. 2, image synthesis) ----------------------
 * For npx pixels (view v, x, y) = (pix[3p], pix[3p+1], pix[3p+2]) of views
 * cams[] at W x H: RGB into rgb[3p..], nearest (i*, j*) into nn[2p..] (-1 on
 * miss), and the smallest decision margin into margin[4p..]: [tangent
 * test, nearest gap, zone, K-th gap] (min over both hit points).
 * lf is the light field as FP32 [rows][N][3], rows = origin_rows or M;
 * neighbours i >= rows are not stored and carry weight 0 (a pixel left with
 * none is 0, as is a K = 1 pixel whose nearest origin is not stored). */
void orc_lookup(const float* lf, const orc_params* prm, const orc_camera* cams,
                int32_t W, int32_t H, int32_t K, const int32_t* pix, int64_t npx,
                double* rgb, int64_t* nn, double* margin, int32_t nthreads);

/* Transpose of orc_lookup: d_lf[a][b][c] += weight(a,b) * dimg[p][c] for the
 * listed pixels; d_lf is FP64 [rows][N][3], accumulated (not cleared). */
void orc_lookup_adjoint(const orc_params* prm, const orc_camera* cams,
                        int32_t W, int32_t H, int32_t K, const int32_t* pix,
                        int64_t npx, const double* dimg, double* d_lf);

/* ---- Ground-truth views (the paper's reference images: the path tracer
 * itself along camera rays) -----------------------------------------------
 * For npx pixels (view v, x, y) = pix[3p..] of the pinhole views cams[] at
 * W x H (pixel centres, row 0 at the top), rgb[3p..] = mean over spp path
 * samples from the eye along the pixel's ray, traced as orc_generate traces
 * a light-field ray (no origin jitter).  Random-number stream key: the
 * pixel's index (v H + y) W + x.  Uses spp, max_bounces, g, majorant, grid
 * and seed of prm.  Pinned by vacuum, Beer-Lambert along camera rays, and
 * agreement in expectation with light-field rays on the same lines. */
void orc_render(const orc_volume* vol, const orc_medium* med, const orc_light* light, const orc_params* prm,
                const orc_camera* cams, int32_t W, int32_t H, const int32_t* pix, int64_t npx, double* rgb,
                int32_t nthreads);

/* ---- Mean SSIM (Wang et al. 2004), the image index the paper reports ----
 * out[m] for image pairs a, b ([n][H][W][3] float32): 11 x 11 Gaussian
 * window of sigma 1.5 normalised to sum 1, C1 = (0.01 range)^2,
 * C2 = (0.03 range)^2, every window position inside the image, averaged
 * over positions and channels.  Pinned by SSIM(x, x) = 1, the closed form
 * for constant images, symmetry, and a separable scipy filter. */
void orc_ssim(const float* a, const float* b, int32_t n, int32_t W, int32_t H, double data_range, double* out);

#ifdef __cplusplus
}
#endif
#endif
