// surface.hip -- isosurface variant of generation and of the ground-truth
// views: the paper path-traces segmented surfaces; here the surface is where
// the trilinear raw field crosses an isovalue, shaded as a Lambertian
// reflector with the LUT colour at the isovalue.
//
// Path (per sample, up to max_bounces vertices):
//   - first crossing along the segment inside the box: the field minus the
//     isovalue is sampled every half voxel from the segment start, the first
//     pair of samples with different signs is bisected, and the bracket end
//     on the incoming side is the vertex (a path always continues on the
//     side it came from);
//   - normal: central differences of the field over a quarter voxel, turned
//     to face the incoming ray;
//   - next-event estimation: one light sample (vertex stream, pair 0) with a
//     visibility march towards it, BRDF rho / pi;
//   - bounce: cosine-weighted about the normal (pair 1), throughput * rho;
//   - a segment with no crossing adds the environment.
// Samples inside a majorant-grid cell whose raw range excludes the isovalue
// have a known sign and are not fetched: the cell range covers every point
// of the cell plus a voxel, so the march finds the same crossing as a march
// that fetches every sample.
//
// One lane per ray (light-field ray or view pixel), 8 x 8 tiles per wave,
// all samples of the ray in order, so the texel sum is deterministic.
#include "internal.hpp"

namespace lp {

struct SurfCtx {
    const TraceParams& P;
    const float2* rng;      // LDS: raw [lo, hi] per grid cell
    float iso, h;
};

template <int VT>
__device__ __forceinline__ float field(const SurfCtx& S, f3 y) {
    return sample_volume<VT>(S.P, y) - S.iso;
}

// Sign of field - iso at y: from the cell range when it excludes the
// isovalue, else fetched.  Returns true for "non-negative".
template <int VT>
__device__ __forceinline__ bool field_sign(const SurfCtx& S, f3 y) {
    const TraceParams& P = S.P;
    const int G = P.grid_n, Gm = G - 1;
    const int cx = min(max((int)floorf((y.x - P.bmin[0]) * P.gcell[0]), 0), Gm);
    const int cy = min(max((int)floorf((y.y - P.bmin[1]) * P.gcell[1]), 0), Gm);
    const int cz = min(max((int)floorf((y.z - P.bmin[2]) * P.gcell[2]), 0), Gm);
    const float2 r = S.rng[(cz * G + cy) * G + cx];
    if (S.iso < r.x) return true;
    if (S.iso > r.y) return false;
    return field<VT>(S, y) >= 0.0f;
}

// First crossing on [t0, t1] of x + t d: true and *th = incoming-side end.
template <int VT>
__device__ bool surface_hit(const SurfCtx& S, f3 x, f3 d, float t0, float t1, float& th) {
    bool sa = field_sign<VT>(S, fma3(d, t0, x));
    float ta = t0;
    for (int m = 1;; ++m) {
        float tb = fmaf((float)m, S.h, t0);
        if (tb > t1) tb = t1;
        const bool sb = field_sign<VT>(S, fma3(d, tb, x));
        if (sb != sa) {
            float lo = ta, hi = tb;
            for (int it = 0; it < 24; ++it) {
                const float mid = 0.5f * (lo + hi);
                if ((field<VT>(S, fma3(d, mid, x)) >= 0.0f) == sa) lo = mid;
                else hi = mid;
            }
            th = lo;
            return true;
        }
        if (tb >= t1) return false;
        ta = tb;
    }
}

template <int VT>
__device__ __forceinline__ f3 surface_normal(const SurfCtx& S, f3 y, f3 d) {
    const float e = 0.5f * S.h;
    const float gx = sample_volume<VT>(S.P, mk3(y.x + e, y.y, y.z)) - sample_volume<VT>(S.P, mk3(y.x - e, y.y, y.z));
    const float gy = sample_volume<VT>(S.P, mk3(y.x, y.y + e, y.z)) - sample_volume<VT>(S.P, mk3(y.x, y.y - e, y.z));
    const float gz = sample_volume<VT>(S.P, mk3(y.x, y.y, y.z + e)) - sample_volume<VT>(S.P, mk3(y.x, y.y, y.z - e));
    f3 n = mk3(gx, gy, gz);
    const float l2 = dot(n, n);
    if (!(l2 > 0.0f)) return d * -1.0f;
    n = n * rsq(l2);
    return dot(n, d) > 0.0f ? n * -1.0f : n;
}

template <int VT>
__global__ __launch_bounds__(256) void surface_kernel(TraceParams P) {
    __shared__ float2 rng[16 * 16 * 16];
    const int ncell = P.grid_n * P.grid_n * P.grid_n;
    for (int e = threadIdx.x; e < ncell; e += blockDim.x) rng[e] = ((const float2*)P.srange)[e];
    __syncthreads();
    SurfCtx S{P, rng, P.iso, P.half_voxel};
    // albedo: the LUT colour at the isovalue's window position, clamped
    f3 rho;
    {
        const float sw = fminf(fmaxf((P.iso - P.vmin) * P.vscale, 0.0f), 1.0f);
        const float u = sw * P.lut_last;
        const int l0 = min((int)u, P.lut_n - 2);
        const float w = u - (float)l0;
        const float4 A = ((const float4*)P.lut_e)[l0], B = ((const float4*)P.lut_e)[l0 + 1];
        rho = mk3(fminf(fmaxf(fmaf(w, B.x - A.x, A.x), 0.0f), 1.0f), fminf(fmaxf(fmaf(w, B.y - A.y, A.y), 0.0f), 1.0f),
                  fminf(fmaxf(fmaf(w, B.z - A.z, A.z), 0.0f), 1.0f));
    }

    const int lane = threadIdx.x & 63;
    const long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t K0 = P.key0, K1 = P.key1;
    const f3 bmin = mk3(P.bmin[0], P.bmin[1], P.bmin[2]), bmax = mk3(P.bmax[0], P.bmax[1], P.bmax[2]);
    const f3 env = mk3(P.env[0], P.env[1], P.env[2]);
    // the work item: a light-field ray or a view pixel
    bool active = false;
    uint32_t k = 0;
    f3 po = mk3(0, 0, 0), d0 = po;
    bool lf_ray = !P.views;
    if (P.views) {
        const uint32_t t = (uint32_t)tile;
        const uint32_t v = t / (uint32_t)P.vtiles, rem = t - v * (uint32_t)P.vtiles;
        const uint32_t ty = rem / (uint32_t)P.vtx, tx = rem - ty * (uint32_t)P.vtx;
        const int py = (int)ty * 8 + (lane >> 3), px = (int)tx * 8 + (lane & 7);
        if (v < (uint32_t)P.nviews && py < P.H && px < P.W) {
            const ViewCam& cam = P.views[v];
            const float ndx = (2.0f * ((float)px + 0.5f) / (float)P.W - 1.0f) * cam.sx;
            const float ndy = (1.0f - 2.0f * ((float)py + 0.5f) / (float)P.H) * cam.sy;
            k = (v * (uint32_t)P.H + (uint32_t)py) * (uint32_t)P.W + (uint32_t)px;
            po = mk3(cam.eye[0], cam.eye[1], cam.eye[2]);
            d0 = normalize(mk3(cam.fwd[0], cam.fwd[1], cam.fwd[2]) + mk3(cam.right[0], cam.right[1], cam.right[2]) * ndx +
                           mk3(cam.up[0], cam.up[1], cam.up[2]) * ndy);
            active = true;
        }
    } else {
        const int rows = P.row_end - P.row_begin;
        const int tiles_i = (rows + 7) / 8, tiles_j = (P.N + 7) / 8;
        if (tile < (long long)tiles_i * tiles_j) {
            int ti, tj;
            tile_coords(tile, tiles_i, tiles_j, ti, tj);
            const int oi = ti * 8 + (lane >> 3), dj = tj * 8 + (lane & 7);
            if (oi < rows && dj < P.N) {
                const int i = P.perm_o[oi], j = P.perm_d[dj];
                k = (uint32_t)i * (uint32_t)P.N + (uint32_t)j;
                if (P.M == P.N && i == j) {
                    store_texel(P.out, P.dtype, k, mk3(0.0f, 0.0f, 0.0f));  // no direction: texel 0
                } else {
                    po = sf_point(P.M, i, 1.0f / (float)P.M);
                    d0 = normalize(sf_point(P.N, j, 1.0f / (float)P.N) - po);
                    active = true;
                }
            }
        }
    }
    if (!active) return;

    Counters cnt = {0, 0, 0, 0, 0};
    f3 acc = mk3(0.0f, 0.0f, 0.0f);
    f3 t1 = po, t2 = po;
    if (lf_ray) frame(po, t1, t2);
    for (int s = 0; s < P.spp; ++s) {
        cnt.samples++;
        f3 x = po, dir = d0, T = mk3(1.0f, 1.0f, 1.0f), L = mk3(0.0f, 0.0f, 0.0f);
        if (lf_ray) {
            x = mk3(P.O[0], P.O[1], P.O[2]) + po * P.R;
            if (P.jitter) {
                const u4 rj = philox(k, (uint32_t)s, kPurFlight, 0u, K0, K1);
                const float rr = P.jit_rad * sqrtf(u01(rj.x));
                float sa, ca;
                sincospif(2.0f * u01(rj.y), &sa, &ca);
                x = x + (t1 * (rr * ca) + t2 * (rr * sa));
            }
        }
        for (int b = 0; b < P.maxb; ++b) {
            float tn, tf, th;
            if (!clip_box(bmin, bmax, x, dir, tn, tf) || !surface_hit<VT>(S, x, dir, tn, tf, th)) {
                L = L + T * env;
                break;
            }
            cnt.real++;
            const f3 y = fma3(dir, th, x);
            const f3 n = surface_normal<VT>(S, y, dir);
            const u4 r = philox(k, (uint32_t)s, ((uint32_t)b << 8) | kPurVertex, 0u, K0, K1);
            if (P.light_on) {
                f3 om, Le;
                float tend = 0.0f;
                if (P.light_kind == 0) {
                    om = mk3(P.ldir[0], P.ldir[1], P.ldir[2]);
                    Le = mk3(P.lrad[0], P.lrad[1], P.lrad[2]);
                    float a0, a1;
                    if (clip_box(bmin, bmax, y, om, a0, a1)) tend = a1;
                } else {
                    const f3 yl = mk3(P.lcorner[0], P.lcorner[1], P.lcorner[2]) +
                                  mk3(P.le1[0], P.le1[1], P.le1[2]) * u01(r.x) + mk3(P.le2[0], P.le2[1], P.le2[2]) * u01(r.y);
                    const f3 v = yl - y;
                    const float d2 = dot(v, v);
                    const float rinv = rsq(d2);
                    const float dist = d2 * rinv;
                    om = v * rinv;
                    const float cl = fmaxf(0.0f, -dot(mk3(P.lnrm[0], P.lnrm[1], P.lnrm[2]), om));
                    Le = mk3(P.lrad[0], P.lrad[1], P.lrad[2]) * (cl * P.larea * rcp(d2));
                    float a0, a1;
                    tend = dist;
                    if (clip_box(bmin, bmax, y, om, a0, a1)) tend = fminf(tend, a1);
                    else tend = 0.0f;
                }
                const float cosl = dot(n, om);
                float tv;
                if (cosl > 0.0f && !(tend > 0.0f && surface_hit<VT>(S, y, om, 0.0f, tend, tv)))
                    L = L + T * rho * Le * (cosl * 0.318309886183790672f);
            }
            if (b == P.maxb - 1) break;
            // cosine-weighted bounce about n
            const float u0 = u01(r.z), rr = sqrtf(u0);
            float sp, cp;
            sincospif(2.0f * u01(r.w), &sp, &cp);
            f3 b1, b2;
            frame(n, b1, b2);
            dir = normalize(b1 * (rr * cp) + b2 * (rr * sp) + n * sqrtf(fmaxf(0.0f, 1.0f - u0)));
            T = T * rho;
            if (T.x == 0.0f && T.y == 0.0f && T.z == 0.0f) break;
            x = y;
        }
        acc = acc + L;
    }
    const float fs = (float)P.spp;
    store_texel(P.out, P.dtype, k, mk3(acc.x / fs, acc.y / fs, acc.z / fs));
    if (P.stats) {
        atomicAdd(&P.stats[2], (unsigned long long)cnt.real);
        atomicAdd(&P.stats[3], (unsigned long long)cnt.samples);
    }
}

hipError_t launch_surface(const TraceParams& P, int vtype, hipStream_t s) {
    long long ntiles;
    if (P.views) {
        ntiles = (long long)P.nviews * P.vtiles;
    } else {
        const long long rows = P.row_end - P.row_begin;
        ntiles = ((rows + 7) / 8) * (long long)((P.N + 7) / 8);
    }
    if (ntiles <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((ntiles + 3) / 4);
    if (vtype == 0) surface_kernel<0><<<blocks, 256, 0, s>>>(P);
    else if (vtype == 1) surface_kernel<1><<<blocks, 256, 0, s>>>(P);
    else surface_kernel<2><<<blocks, 256, 0, s>>>(P);
    return hipGetLastError();
}

}  // namespace lp
