/*
 * lumipath.h -- C ABI of the MI355X light-field library (liblumipath.so).
 *
 * Implements the data-parallel path of Fink et al., "LumiPath -- Towards
 * Real-time Physically-based Rendering on Embedded Devices" (arXiv
 * 1903.03837): the precomputed light field Lhat(i,j) over two spherical-
 * Fibonacci point sets on a sphere S bounding the scene (Sec. 2, Fig. 1), and
 * image synthesis by looking up and blending its texels (Sec. 2, Fig. 2).
 * The scene is a scalar density volume under a transfer function and a light,
 * path traced volumetrically (the paper renders surfaces; Sec. 4 names
 * volumes as the goal).
 *
 * Conventions shared by every entry point
 *  - Every array argument is device memory owned by the caller unless marked
 *    "host".  Structs passed by pointer are host memory, read during the call
 *    only.  The library allocates nothing and keeps no state between calls
 *    apart from the thread-local error message (and the fixed device scratch
 *    of lf_lookup_static, whose contents no call relies on).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    asynchronous and stream-ordered; the caller keeps buffers alive until
 *    the stream has passed the call.
 *  - Return value: LF_OK (0) or a negative lf_status.  Arguments are checked
 *    on the host before any GPU work; on error nothing is launched and
 *    lf_last_error() describes the problem.  HIP launch failures return
 *    LF_E_HIP with the HIP message.
 *  - Light fields are row-major [M][N][3] RGB: texel (i, j) for origin i of
 *    P_o (M points) and direction j of P_d (N points), stored as binary32,
 *    binary16 or bfloat16 (round to nearest even from the FP32 mean).
 */
#ifndef LUMIPATH_H
#define LUMIPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LUMIPATH_VERSION 1

typedef enum {
    LF_OK = 0,
    LF_E_ARG = -1,          /* bad pointer, size, enum or geometry */
    LF_E_RANGE = -2,        /* sizes beyond the supported range */
    LF_E_UNSUPPORTED = -3,  /* valid but not implemented combination */
    LF_E_WORKSPACE = -4,    /* workspace missing or too small */
    LF_E_HIP = -5           /* HIP runtime error */
} lf_status;

enum { LF_F32 = 0, LF_F16 = 1, LF_BF16 = 2 };           /* light-field storage */
enum { LF_VOX_U8 = 0, LF_VOX_U16 = 1, LF_VOX_F32 = 2 };   /* voxel types */
enum { LF_LIGHT_DIRECTIONAL = 0, LF_LIGHT_AREA = 1 };
enum { LF_LOOKUP_FORWARD = 0, LF_LOOKUP_ADJOINT = 1 };

/* Scalar volume filling the box [box_min, box_max] (inside S).  Voxel centres
 * sit at box_min + (idx + 0.5) * extent / n; values are interpolated
 * trilinearly (edge-clamped) and mapped through the window [vmin, vmax] onto
 * the transfer function.  brick = 0: x-fastest linear array; brick = 8: 8^3
 * bricks, bricks ordered x-fastest, voxels x-fastest inside a brick (each of
 * nx, ny, nz divisible by 8).  nx, ny, nz >= 2.  The tracing entry points
 * copy the volume into their workspace as 4^3-voxel bricks placed every 3
 * voxels (64 * prod((n - 2) / 3 + 1) voxels); a volume whose copy would exceed
 * 2^32 voxels, or with a dimension above 65535, is rejected with LF_E_RANGE. */
typedef struct {
    const void* data;       /* device [nx*ny*nz] of the voxel type, aligned to it */
    int32_t type;           /* LF_VOX_* */
    int32_t nx, ny, nz;
    int32_t brick;          /* 0 or 8 */
    float vmin, vmax;       /* vmax > vmin */
    float box_min[3], box_max[3];
} lf_volume;

/* Transfer function: lut_size RGBA entries (device, float32 [lut_size][4],
 * 16-byte aligned), interpolated linearly; sigma_t = density_scale * alpha, single-scattering
 * albedo = rgb clamped to [0,1].  2 <= lut_size <= 1024. */
typedef struct {
    const float* lut;
    int32_t lut_size;
    float density_scale;    /* >= 0 */
} lf_medium;

/* One light plus a constant environment radiance `env` seen by paths that
 * leave the volume.  Directional: unit `dir` towards the light, `radiance`
 * is its irradiance.  Area: parallelogram corner + s e1 + t e2 (s,t in
 * [0,1]), emitting `radiance` on the side cross(e1, e2) points to; it must
 * lie outside the volume box. */
typedef struct {
    int32_t kind;           /* LF_LIGHT_* */
    float dir[3];
    float corner[3], e1[3], e2[3];
    float radiance[3];
    float env[3];
} lf_light;

/* Ray set and path-tracer settings (Sec. 2: S with centre O = center and
 * radius R = radius; P_o of M points, P_d of N points; ray k = i*N + j runs
 * from O + R p_i towards O + R p_j with its origin jittered on the disk of
 * area 4 pi R^2 / M when jitter != 0).  M, N in [1, 65535], M*N < 2^32.
 * origin_rows (0 = M) keeps only the origins i < origin_rows: the light field
 * is stored as [origin_rows][N][3].  Heights of the SF set fall with i, so
 * origin_rows = M/2 keeps the upper hemisphere (Sec. 3 stores P_o that way,
 * halving the texture); lookups whose front hit has no stored origin are
 * uncovered (pixel 0).
 * spp >= 1 samples, 1 <= max_bounces <= 65535 scatter vertices, |hg_g| < 1.
 * majorant > 0 fixes one global majorant; otherwise it is 1.25 *
 * density_scale * max alpha of the sampling medium, and majorant_grid = G in
 * [1, 16] replaces it by a grid of G^3 cell majorants over the volume box
 * (piecewise-constant majorant, as in PBRT's grid media): each cell bounds
 * 1.25 sigma_t of the sampling medium over the voxels its points can reach
 * (one voxel to spare), floored at 1/256 of the global majorant so that null
 * collisions stay possible everywhere.  Tentative collisions then spend the
 * exponential variate cell by cell; the random-number layout is unchanged.
 * G = 0 keeps the global majorant.  Rows [row_begin, row_end) of i are
 * generated (row_end <= 0: origin_rows); results do not depend on this
 * split.  stats: NULL or device uint64[5] incremented by [tentative
 * collisions, shadow-ray steps, real collisions, path samples, majorant-cell
 * steps].
 * surface = 1 selects the isosurface variant (the paper renders segmented
 * surfaces): the surface is where the trilinear raw field crosses iso.  Its
 * first crossing along a segment is found by sampling the field every half
 * voxel from the segment start and bisecting the first pair of samples of
 * different sign; the vertex is the bracket end on the incoming side.  The
 * surface is a Lambertian reflector of albedo = the LUT colour at iso
 * (clamped to [0, 1]; the density scale and alpha are unused) with
 * next-event estimation (vertex stream pair 0, visibility by the same march)
 * and cosine-weighted bounces (pair 1); normals are central differences over
 * a quarter voxel.  The majorant grid size (8 when 0) sets the cells whose
 * raw ranges let the march skip fetches.  Frozen sampling and
 * lf_generate_backward are not available in this variant (LF_E_UNSUPPORTED).
 * sample_radiance (light-field calls only; NULL in the isosurface variant):
 * lf_generate writes the radiance of every sample of every generated ray
 * at ((i*N + j)*spp + s)*3 (texels i == j are not written, and of a ray
 * that misses the volume box in every sample only the last sample is);
 * lf_generate_backward reads it instead of tracing each sample a first
 * time.  It must come from lf_generate with the same parameters and medium
 * and sample == NULL.
 * waves_per_simd: the resident waves per SIMD the forward light-field and
 * view kernels' registers are budgeted for (0 = 4; otherwise 3 or 4, else
 * LF_E_ARG).  Results do not depend on it: the same code draws the same
 * random numbers in the same order.  Four waves hide more latency and suit
 * workloads whose volume traffic HBM absorbs; when the tracer already runs
 * HBM near its peak, three are faster (fewer concurrent misses).
 * lf_generate_backward always budgets for three. */
typedef struct {
    int32_t M, N;
    float center[3];
    float radius;
    int32_t spp, max_bounces;
    float hg_g;
    float majorant;
    int32_t majorant_grid;  /* cells per axis of the majorant grid, 0 = global */
    uint64_t seed;
    int32_t jitter;
    int32_t origin_rows;    /* stored origin rows: 0 = M; M/2 keeps the upper hemisphere */
    int64_t row_begin, row_end;
    uint64_t* stats;
    int32_t surface;        /* 1: isosurface variant at raw value iso */
    float iso;
    float* sample_radiance; /* NULL or device float32 [origin_rows][N][spp][3] */
    int32_t waves_per_simd; /* forward path tracer's register budget: 0 = the library's choice (4), 3 or 4 */
} lf_gen_params;

/* Pinhole view (host array): pixel (x, y) looks through its centre, row 0 at
 * the top, vertical field of view vfov radians, aspect W/H. */
typedef struct {
    float eye[3], target[3], up[3];
    float vfov;
} lf_camera;

/* Message of the last failing call on this thread ("" if none). */
const char* lf_last_error(void);
int lf_version(void);

/* Spherical-Fibonacci point set and its inverse query (Sec. 2, SF point
 * equation; nearest-neighbour query over at most nine neighbours and the
 * filter kernel of size R sqrt(4 pi / N)).
 *   xyz_out: NULL or float [n][3], p_i for i < n (frac(i/Phi) in FP64).
 *   query:   NULL or float [nq][3] unit vectors; then idx_out int32 [nq][K]
 *            receives the K nearest of the candidate set i* + {0, +-F(k-1),
 *            +-F(k), +-F(k+1), +-F(k+2)} in order of distance (on the
 *            first candidate set, squared distances compared to 20
 *            significant bits, ties by candidate slot; after a descent, by
 *            (distance, index)), -1 where fewer exist, and w_out (may be NULL) float
 *            [nq][K] the tent weights max(0, 1 - d / sqrt(4 pi / n)) (d:
 *            unit chord).
 *            idx_out[q][0] is the nearest point.  1 <= K <= 9.
 * n in [1, 65535]. */
int lf_points(int32_t n, float* xyz_out, const float* query, int64_t nq, int32_t K,
              int32_t* idx_out, float* w_out, void* stream);

/* Light-field generation (Sec. 2, Fig. 1): writes Lhat(i, j) = mean over spp
 * path samples of the radiance along ray k = i*N + j, for rows
 * [row_begin, row_end), into lf_out ([origin_rows][N][3] of `dtype`).  Texels with
 * M == N and i == j (no direction) are 0.  Random numbers: Philox4x32-10
 * keyed by `seed`, counter (k, sample, bounce << 8 | purpose, block), so the
 * result is independent of launch shape and row split.  The mean is summed in
 * FP32 over R equal ranges of consecutive samples, each in sample order, then
 * the R range sums in order, then divided by spp.  R = min(R_spp, R_rays):
 * R_spp = 4 when spp >= 32, 2 when spp >= 16, else 1; R_rays = 4 when
 * M*N < 1572864, 2 when M*N < 12582912, else 1; and R = 1 whenever
 * M*N*spp > 2^31 (the ranges are work items of their own, for load balance;
 * the workspace then holds their sums).
 *   eval:   medium evaluated.   sample: NULL, or the medium that decides
 *   collisions (frozen sampling: the path is importance-weighted from sample
 *   to eval; used for finite-difference checks of the adjoint).
 *   ws / ws_bytes: when ws == NULL only *ws_bytes is set (the workspace
 *   size); otherwise *ws_bytes must be at least that size. */
int lf_generate(const lf_volume* vol, const lf_medium* eval, const lf_medium* sample,
                const lf_light* light, const lf_gen_params* params, int32_t dtype, void* lf_out,
                void* ws, size_t* ws_bytes, void* stream);

/* Image synthesis from the light field (Sec. 2, Fig. 2).  For every pixel
 * of n_views W x H views: the view ray's front and back hits on S (tangential
 * rays discarded) are mapped to their K nearest points of P_o and P_d and the
 * K x K texels blended with normalised tent weights (pairs i == j excluded
 * when M == N); K = 1 is nearest sampling.  Uses M, N, origin_rows, center,
 * radius of params; neighbours i >= origin_rows are not stored and get weight
 * 0 (a pixel with none left is 0).
 *   mode LF_LOOKUP_FORWARD: lf (dtype) -> img float [n_views][H][W][3].
 *   mode LF_LOOKUP_ADJOINT: img holds d(loss)/d(img); d_lf (float32
 *        [origin_rows][N][3]) is incremented by its transpose (atomics; lf
 *        unused).
 *   nn_out: NULL or int32 [n_views][H][W][2], nearest (i, j), -1 on a miss.
 *   cams: host array of n_views cameras, each eye outside S.
 *   ws / ws_bytes: workspace for the point tables of both SF sets (16 bytes
 *   per point) and their lattice bases per zone (768 bytes per set), filled
 *   by the call; ws == NULL only sets *ws_bytes. */
int lf_lookup(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams, int32_t n_views,
              int32_t W, int32_t H, int32_t K, int32_t mode, float* img, float* d_lf, int32_t* nn_out, void* ws,
              size_t* ws_bytes, void* stream);

/* lf_lookup without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and errors as for lf_lookup, minus
 * ws / ws_bytes: the point tables and zone bases of both SF sets live in a
 * fixed device array of the library of 2 MiB + 1.5 KiB (room for 2 x 65536
 * points, so every valid M, N fits; larger tables would be rejected with
 * LF_E_RANGE), which each
 * device holds from its first call until the process ends.  The first call
 * on a device looks up that array's address with the device current; the
 * call allocates nothing.  `stream` must belong to the current device
 * (LF_E_ARG otherwise).  Every call overwrites the whole table it uses
 * before reading it, so nothing carries over from an earlier call; but all
 * calls on one device share the array, so calls that overlap in time on one
 * device (different streams, or threads) race and must be serialised by the
 * caller. */
int lf_lookup_static(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams,
                     int32_t n_views, int32_t W, int32_t H, int32_t K, int32_t mode, float* img, float* d_lf,
                     int32_t* nn_out, void* stream);

/* Lookup, loss gradient and adjoint in one pass (Sec. 2 lookup and its
 * transpose, for an L2 image loss): img receives the views of lf exactly as
 * lf_lookup's forward mode writes them, and d_lf (float32
 * [origin_rows][N][3]) is incremented by the transpose applied to
 * img - target, the gradient of 1/2 |img - target|^2 (atomics).  target:
 * float32 [n_views][H][W][3], read only.  Other arguments as for lf_lookup. */
int lf_lookup_l2(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams, int32_t n_views,
                 int32_t W, int32_t H, int32_t K, const float* target, float* img, float* d_lf, void* ws,
                 size_t* ws_bytes, void* stream);

/* Ground-truth views: the path tracer of lf_generate along pinhole camera
 * rays, the reference the paper compares its light-field views with (Sec. 3
 * evaluation).  For each pixel (x, y) of each of the n_views cameras (host
 * array, consumed before return; pixel centres, row 0 at the top, as in
 * lf_lookup) img[((v * H + y) * W + x) * 3 + c] (device float32) receives
 * the mean over params->spp samples of the radiance along the ray from the
 * eye through the pixel centre.  The ray starts at the eye with no jitter;
 * the random streams are those of a light-field ray with key
 * (v * H + y) * W + x.  Uses spp, max_bounces, hg_g, majorant,
 * majorant_grid and seed of params (M, N, center, radius, jitter and the
 * row range are ignored).  n_views * W * H < 2^32.  Workspace as for
 * lf_generate (size query with ws == NULL). */
int lf_render_views(const lf_volume* vol, const lf_medium* medium, const lf_light* light,
                    const lf_gen_params* params, const lf_camera* cams, int32_t n_views, int32_t W, int32_t H,
                    float* img, void* ws, size_t* ws_bytes, void* stream);

/* Mean SSIM (Wang et al. 2004; the image index the paper reports in its
 * evaluation) of n_images pairs of RGB float32 images a, b (device,
 * [n_images][H][W][3]): 11 x 11 Gaussian window of sigma 1.5 normalised to
 * sum 1, C1 = (0.01 data_range)^2, C2 = (0.03 data_range)^2, SSIM terms at
 * every window position inside the image ((W - 10) x (H - 10) per channel),
 * averaged over positions and the three channels.  out: device float64
 * [n_images].  W, H >= 11, 1 <= n_images <= 21845.  The result does not
 * depend on scheduling (fixed-order FP64 sums of FP32 terms).  Workspace:
 * size query with ws == NULL. */
int lf_ssim(const float* a, const float* b, int32_t n_images, int32_t W, int32_t H, float data_range, double* out,
            void* ws, size_t* ws_bytes, void* stream);

/* Mean CW-SSIM (complex-wavelet SSIM, Wang & Simoncelli 2005, Sampat et
 * al. 2009; the second index the paper reports in its image-quality
 * evaluation, Sec. 3) of n_images pairs of RGB float32 images a, b
 * (device, [n_images][H][W][3]).  The paper names only a steerable pyramid
 * of eight levels in total; here: eight complex subbands (2 scales x 4
 * orientations) of a filter bank defined on the DFT grid of the image, with
 * signed frequency f = u (2u < n) or u - n, w = 2 pi f / n, r = |w|,
 * theta = atan2(w_y, w_x): radial window cos(pi/2 log2(r / r_s)) for
 * |log2(r / r_s)| < 1, r_s = pi / 2^(s+1), s = 0, 1; one-sided angular
 * window cos(d)^3 for |d| < pi/2, d = theta - pi k / 4 wrapped to
 * (-pi, pi], k = 0..3.  For each channel and subband the local index
 * (2 |sum c_a conj(c_b)| + K) / (sum |c_a|^2 + sum |c_b|^2 + K) over every
 * 7 x 7 window inside the image, K = 49 (0.01 data_range)^2 (data_range 0:
 * K = 0, and a window with 0 / 0 counts as 1), averaged over positions,
 * subbands and channels.  out: device float64 [n_images].  7 <= W, H <=
 * 4096; data_range >= 0.  A direct DFT (O(W H (W + H)) per plane) in FP32
 * with FP64 sums of the local terms in a fixed order: the result is the same
 * on every run.  Workspace: size query with ws == NULL (about 150 W H
 * bytes).  Stream-ordered on `stream`. */
int lf_cw_ssim(const float* a, const float* b, int32_t n_images, int32_t W, int32_t H, float data_range,
               double* out, void* ws, size_t* ws_bytes, void* stream);

/* Cell majorants of the majorant grid that lf_generate and
 * lf_generate_backward track against (piecewise-constant majorant; the grid
 * and its bound are defined with lf_gen_params): out (device float
 * [G][G][G], x fastest, G = params->majorant_grid >= 1) for the medium
 * `sample`.  params->majorant is not consulted.  Stream-ordered on `stream`. */
int lf_majorant_grid(const lf_volume* vol, const lf_medium* sample, const lf_gen_params* params, float* out,
                     void* stream);

/* Adjoint of lf_generate (path-replay extension): given d_lf = d(loss)/d(Lhat)
 * (float32 [origin_rows][N][3]), overwrites d_lut (float32 [lut_size][4]) and d_scale
 * (float32 [1]) with d(loss)/d(LUT) and d(loss)/d(density_scale) of the
 * estimator for the same random stream, majorant held fixed.  Each sample is
 * traced twice (total radiance, then scores times radiance gathered after
 * each event); nothing is stored per path.  With params->sample_radiance
 * (the samples' radiance kept by lf_generate) the first trace is skipped.  Accumulation uses float atomics:
 * reproducible to rounding only.  Rows with zero adjoint are skipped.
 * Workspace as for lf_generate. */
int lf_generate_backward(const lf_volume* vol, const lf_medium* medium, const lf_light* light,
                         const lf_gen_params* params, const float* d_lf, float* d_lut,
                         float* d_scale, void* ws, size_t* ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LUMIPATH_H */
