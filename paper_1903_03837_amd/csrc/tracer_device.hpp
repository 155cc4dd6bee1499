// tracer_device.hpp -- building blocks of the volumetric path tracer behind
// lf_generate and lf_generate_backward (the kernel itself is in wave.hip).
//
// Each ray r_k of the SF ray set (Sec. 2, ray equation) is traced by one
// lane, all of its samples in order, so the FP32 sum per texel is
// deterministic.  Transport (the volumetric reading of Sec. 2's "conventional
// path tracer"):
//   - origin jitter on the disk of area 4 pi R^2 / M in the tangent plane;
//   - delta tracking against a majorant: one global sigma_bar, or a grid of
//     cell majorants walked cell by cell;
//   - real collision: throughput times the albedo, next-event estimation
//     towards the light with ratio-tracking transmittance, Henyey-Greenstein
//     direction for the next segment; escape: constant environment.
// Random numbers: Philox4x32-10 keyed by the seed, counter (ray, sample,
// bounce << 8 | purpose, block); a block holds two word pairs.  Purpose 1
// ("flight" of segment b): pair 0 of segment 0 jitters the origin, then one
// pair per tentative collision (distance, acceptance).  Purpose 2 ("vertex"
// b): pair 0 samples the light, pair 1 the phase function, then one pair per
// shadow step (first word: distance).
//
// The kernel runs in three modes:
//   kFwd     plain estimator;
//   kFrozen  decisions with the sampling medium, importance weights to the
//            evaluated medium (finite-difference hook of the adjoint);
//   kGrad    path replay: every event scatters its score times the radiance
//            gathered after it into LDS accumulators (dLUT, dscale).
#pragma once

#include <hip/hip_fp16.h>

#include "sf_device.hpp"

namespace lp {

enum { kFwd = 0, kFrozen = 1, kGrad = 2 };
enum { kPurFlight = 1, kPurVertex = 2 };
// At most 2^20 word pairs (2^19 blocks) per stream.  Valid scenes stay orders
// of magnitude below; a segment that reaches it ends absorbed (free flight)
// or fully blocked (shadow), so no lane can spin.
constexpr uint32_t kMaxBlocks = 1u << 19;

// Pinhole view for ground-truth rendering: eye, orthonormal basis and the
// half-extents tan(vfov / 2) * aspect, tan(vfov / 2) of the image plane.
struct ViewCam {
    float eye[3], fwd[3], right[3], up[3];
    float sx, sy;
};

struct TraceParams {
    // volume: the library's halo-brick copy (4^3-voxel bricks every 3
    // voxels, bricks x-fastest, voxels x-fastest inside a brick)
    const void* vol;
    int32_t nx, ny;
    int32_t brick_row, brick_slab;   // 64 * bricks per row, 64 * bricks per slab
    float ga[3], gb[3];              // grid coordinate = x * ga + gb
    float gmax[3];                   // n - 1
    int32_t imax[3];                 // n - 2
    float vmin, vscale;              // s = (v - vmin) * vscale
    int32_t lut_n;
    float lut_last;                  // lut_n - 1
    const float* lut_e;              // [lut_n][4]
    const float* lut_s;
    float scale_e, scale_s;
    float bmin[3], bmax[3];
    // light
    int32_t light_kind, light_on;
    float ldir[3], lcorner[3], le1[3], le2[3], lrad[3], lnrm[3];
    float larea;
    float env[3];
    // ray set
    int32_t M, N;
    float O[3], R;
    int32_t spp, maxb;
    float g;
    uint32_t key0, key1;
    int32_t jitter;
    float jit_rad;                   // 2 R / sqrt(M)
    int32_t row_begin, row_end;
    const float* sigbar;             // device scalar
    // outputs
    void* out;
    int32_t dtype;
    unsigned long long* stats;
    int32_t part_log2;  // work items per ray = 2^part_log2 sample ranges
    int32_t waves;      // forward kernels: waves per SIMD the registers are budgeted for (3 or 4)
    float* part_sums;   // forward with several ranges: [rows][N][ranges][3]
    // SF points of both sets (workspace tables filled by sf_point with
    // inv_n = 1/n in FP32, the values the kernel would compute)
    const float4* tab_o;
    const float4* tab_d;
    // per-sample radiance [rows][N][spp][3]: written by the forward,
    // read by the adjoint in place of its first pass (or NULL)
    float* srad;
    // adjoint
    const float* d_lf;
    float* d_lut;
    float* d_scale;
    // persistent forward kernel: spatial orders of the origin rows and the
    // directions, and the per-XCD tile counters (workspace)
    const int32_t* perm_o;
    const int32_t* perm_d;
    unsigned int* tile_ctr;
    // majorant grid: grid_n^3 cell majorants (x fastest) over the volume box;
    // grid_n = 1 with maj = sigbar is the global majorant
    int32_t grid_n, nz;
    // isosurface variant: isovalue, half the smallest voxel extent, raw
    // [lo, hi] per grid cell
    int32_t surface;
    float iso, half_voxel;
    const float* srange;
    // ground-truth views (views != nullptr): camera rays instead of the SF ray
    // set, 8 x 8 pixel tiles, stream key = (view * H + y) * W + x
    const ViewCam* views;
    int32_t nviews, W, H;
    int32_t vtx, vtiles;             // tiles per image row, tiles per view
    float gcell[3];                  // cells per world unit
    float gcw[3];                    // cell width
    const float* maj;
    // adjoint: compacted list of rays with a nonzero adjoint and its length
    uint32_t* ray_list;
    unsigned int* ray_count;
};

// The kernel arguments seen through the kernarg segment (constant address
// space): fields read through such a reference load with scalar loads.  The
// persistent kernels read their parameters this way inside their main loop,
// behind an empty asm barrier per iteration that keeps the loads from being
// hoisted: the compiler then reloads parameters where they are needed
// instead of holding ~100 uniform values in scalar registers and spilling
// them to vector-register lanes (one VALU instruction per spilled read).
typedef const __attribute__((address_space(4))) TraceParams KTraceParams;

// Ray tiles: 8 origins x 8 directions, taken in groups of 16 origin tiles
// sweeping the direction tiles; the tile sequence is cut into 8 parts, one
// per XCD (workgroups are dispatched round-robin over the XCDs).
constexpr int kGroupTiles = 16;
constexpr int kParts = 8;

// Tile t of the row slab -> (origin tile, direction tile).  Tile counts are
// below 2^32 (M, N <= 65535), so 32-bit unsigned division suffices.
__device__ __forceinline__ void tile_coords(long long t, int tiles_i, int tiles_j, int& ti, int& tj) {
    const uint32_t tu = (uint32_t)t;
    const uint32_t per_group = (uint32_t)kGroupTiles * (uint32_t)tiles_j;
    const uint32_t gi = tu / per_group;
    const uint32_t gsz = (uint32_t)min(kGroupTiles, tiles_i - (int)gi * kGroupTiles);
    const uint32_t off = tu - gi * per_group;
    const uint32_t q = off / gsz;
    tj = (int)q;
    ti = (int)(gi * kGroupTiles + (off - q * gsz));
}

// Lane states of the persistent kernels (kDone: the sample's radiance is
// complete and waits to be added to its texel).
enum : int { kIdle = 0, kStart = 1, kFlight = 2, kVertex = 3, kShadow = 4, kShadow2 = 5, kScatter = 6, kDone = 7 };
// A further tracking pass runs while at least this many lanes of a wave are
// still tracking a segment.
constexpr int kTrackPass = 36;

// Next tile for a wave whose home part is `home`; -1 when all are taken.
__device__ __forceinline__ long long next_tile(unsigned int* ctr, long long ntiles, int home, unsigned& dry) {
    const long long part = (ntiles + kParts - 1) / kParts;
    for (int q = 0; q < kParts; ++q) {
        const int p = (home + q) % kParts;
        if (dry & (1u << p)) continue;
        const long long lo = (long long)p * part;
        const long long n = min(part, ntiles - lo);
        if (n <= 0) {
            dry |= 1u << p;
            continue;
        }
        const unsigned got = atomicAdd(&ctr[p], 1u);
        if ((long long)got < n) return lo + got;
        dry |= 1u << p;
    }
    return -1;
}

// Hardware reciprocal / reciprocal square root (1 ulp).  Used where the
// result only moves a continuous quantity (slab bounds, frames, directions);
// the texel mean and the importance weights keep IEEE division.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct Counters {
    uint32_t tent, shadow, real, samples, cells;
};

// ---------------------------------------------------------------------------
// Medium
// ---------------------------------------------------------------------------
template <int VT>
__device__ __forceinline__ float vox(const void* v, uint32_t idx) {
    if constexpr (VT == 0) return (float)((const uint8_t*)v)[idx];
    else if constexpr (VT == 1) return (float)((const uint16_t*)v)[idx];
    else return ((const float*)v)[idx];
}

// Trilinear raw value at world point y (edge-clamped grid coordinates) from
// the library's halo-brick copy of the volume: bricks of 4^3 voxels placed
// every 3 voxels, so that neighbouring bricks share one layer.  The 2 x 2 x 2
// footprint of base voxel (ix, iy, iz) then lies whole in brick
// (ix/3, iy/3, iz/3) at local offset (ix%3, iy%3, iz%3): one 128-byte line
// for u16, half a line for u8, and one of two lines for f32 (or both, in one
// case of three).  Its eight voxels sit at fixed offsets from the first.
template <int VT, class PT>
__device__ __forceinline__ float sample_volume(const PT& P, f3 y) {
    // clamp to [0, n - 1] as one median-of-three
    const float gx = __builtin_amdgcn_fmed3f(fmaf(y.x, P.ga[0], P.gb[0]), 0.0f, P.gmax[0]);
    const float gy = __builtin_amdgcn_fmed3f(fmaf(y.y, P.ga[1], P.gb[1]), 0.0f, P.gmax[1]);
    const float gz = __builtin_amdgcn_fmed3f(fmaf(y.z, P.ga[2], P.gb[2]), 0.0f, P.gmax[2]);
    const int ix = min((int)gx, P.imax[0]);
    const int iy = min((int)gy, P.imax[1]);
    const int iz = min((int)gz, P.imax[2]);
    const float fx = gx - (float)ix, fy = gy - (float)iy, fz = gz - (float)iz;
    // i / 3 as (i * 43691) >> 17, exact for i < 2^17 (dimensions are < 2^16)
    const uint32_t bx = ((uint32_t)ix * 43691u) >> 17, by = ((uint32_t)iy * 43691u) >> 17,
                   bz = ((uint32_t)iz * 43691u) >> 17;
    const uint32_t lx = (uint32_t)ix - 3u * bx, ly = (uint32_t)iy - 3u * by, lz = (uint32_t)iz - 3u * bz;
    const uint32_t base = bz * (uint32_t)P.brick_slab + by * (uint32_t)P.brick_row + bx * 64u + lz * 16u + ly * 4u + lx;
    const float v000 = vox<VT>(P.vol, base), v100 = vox<VT>(P.vol, base + 1);
    const float v010 = vox<VT>(P.vol, base + 4), v110 = vox<VT>(P.vol, base + 5);
    const float v001 = vox<VT>(P.vol, base + 16), v101 = vox<VT>(P.vol, base + 17);
    const float v011 = vox<VT>(P.vol, base + 20), v111 = vox<VT>(P.vol, base + 21);
    const float c00 = fmaf(fx, v100 - v000, v000), c10 = fmaf(fx, v110 - v010, v010);
    const float c01 = fmaf(fx, v101 - v001, v001), c11 = fmaf(fx, v111 - v011, v011);
    const float c0 = fmaf(fy, c10 - c00, c00), c1 = fmaf(fy, c11 - c01, c01);
    return fmaf(fz, c1 - c0, c0);
}

struct TF {
    int l0;
    float w;
    float a;        // alpha of the evaluated medium
    float a_s;      // alpha of the sampling medium (kFrozen)
};

// Post-classification: window, clamp, linear LUT interpolation (LUT in LDS).
// The alpha of the point; its colour (needed at real collisions only) comes
// from tf_rgb with the same entries and weight.
template <int MODE, class PT>
__device__ __forceinline__ TF classify(const PT& P, const float4* lut_e, const float4* lut_s, float raw) {
    TF t;
    const float s = __builtin_amdgcn_fmed3f((raw - P.vmin) * P.vscale, 0.0f, 1.0f);
    const float u = s * P.lut_last;
    t.l0 = min((int)u, P.lut_n - 2);
    t.w = u - (float)t.l0;
    const float Aw = lut_e[t.l0].w, Bw = lut_e[t.l0 + 1].w;
    t.a = fmaf(t.w, Bw - Aw, Aw);
    if constexpr (MODE == kFrozen) {
        const float4 C = lut_s[t.l0], D = lut_s[t.l0 + 1];
        t.a_s = fmaf(t.w, D.w - C.w, C.w);
    } else {
        t.a_s = t.a;
    }
    return t;
}

// Evaluated colour (unclamped) of a classified point.
__device__ __forceinline__ f3 tf_rgb(const float4* lut_e, const TF& t) {
    const float4 A = lut_e[t.l0], B = lut_e[t.l0 + 1];
    return mk3(fmaf(t.w, B.x - A.x, A.x), fmaf(t.w, B.y - A.y, A.y), fmaf(t.w, B.z - A.z, A.z));
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
// Hardware reciprocals of a direction's components (used by the clip and by
// the majorant-grid walk of the same segment).
__device__ __forceinline__ f3 rcp3(f3 d) { return mk3(rcp(d.x), rcp(d.y), rcp(d.z)); }

// [tn, tf) of o + t d, t >= 0, inside the box; false when empty.  id: the
// reciprocals of d's components (rcp3).
__device__ __forceinline__ bool clip_box(f3 bmin, f3 bmax, f3 o, f3 d, f3 id, float& tn, float& tf) {
    float t0 = 0.0f, t1 = 3.402823466e38f;
    const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z}, ii[3] = {id.x, id.y, id.z};
    const float lo[3] = {bmin.x, bmin.y, bmin.z}, hi[3] = {bmax.x, bmax.y, bmax.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dd[a] == 0.0f) {
            if (oo[a] < lo[a] || oo[a] > hi[a]) return false;
            continue;
        }
        const float inv = ii[a];
        float ta = (lo[a] - oo[a]) * inv, tb = (hi[a] - oo[a]) * inv;
        if (ta > tb) {
            const float t = ta;
            ta = tb;
            tb = t;
        }
        t0 = fmaxf(t0, ta);
        t1 = fminf(t1, tb);
    }
    tn = t0;
    tf = t1;
    return t0 < t1;
}

__device__ __forceinline__ bool clip_box(f3 bmin, f3 bmax, f3 o, f3 d, float& tn, float& tf) {
    return clip_box(bmin, bmax, o, d, rcp3(d), tn, tf);
}

// True when the light-field ray from SF origin po (unit sphere) along d0
// misses the volume box in every sample.  The jitter moves the origin by less
// than jit_rad, so the test clips against the box grown by jit_rad plus a
// margin far above FP32 rounding; without jitter it is the sample's own clip
// (the same function on the same origin).
template <class PT>
__device__ __forceinline__ bool misses_box(const PT& P, f3 O, f3 bmin, f3 bmax, f3 po, f3 d0) {
    const float pad = P.jitter ? P.jit_rad * 1.001f + 1e-5f * P.R : 0.0f;
    float tn, tf;
    return !clip_box(mk3(bmin.x - pad, bmin.y - pad, bmin.z - pad), mk3(bmax.x + pad, bmax.y + pad, bmax.z + pad),
                     O + po * P.R, d0, tn, tf);
}

// Orthonormal completion of unit n (Duff et al. 2017).
__device__ __forceinline__ void frame(f3 n, f3& t1, f3& t2) {
    const float sg = n.z >= 0.0f ? 1.0f : -1.0f;
    const float a = -rcp(sg + n.z);
    const float b = n.x * n.y * a;
    t1 = mk3(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    t2 = mk3(b, sg + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ float hg_phase(float g, float mu) {
    const float den = 1.0f + g * g - 2.0f * g * mu;
    const float r = rsq(den);
    return (1.0f - g * g) * 0.0795774715459476679f * r * r * r;
}
__device__ __forceinline__ float hg_mu(float g, float u) {
    float mu;
    if (fabsf(g) < 1e-3f) {
        mu = 1.0f - 2.0f * u;
    } else {
        const float s = (1.0f - g * g) * rcp(1.0f - g + 2.0f * g * u);
        mu = (1.0f + g * g - s * s) * rcp(2.0f * g);
    }
    return fminf(fmaxf(mu, -1.0f), 1.0f);
}

__device__ __forceinline__ float neg_log1m(float u) { return -__logf(1.0f - u); }

// ---------------------------------------------------------------------------
// Majorant-grid walk (3-D DDA over the grid_n^3 cells along x + t d).  The
// exponential variate tau of a tentative collision is spent cell by cell at
// each cell's majorant; a cell of majorant 0 spends none.
// The walk is rebuilt from the point reached at the start of each iteration;
// a point that rounds into a neighbouring cell only shortens that cell's
// first piece (the cell majorants cover one voxel beyond each cell).
// ---------------------------------------------------------------------------
struct GridWalk {
    float t, tx, ty, tz, dx, dy, dz;
    int ci;          // cell index in the padded grid (one border cell per side)
    int sx, sy, sz;  // signed index steps along x, y, z (by the sign of d)

    // id: the reciprocals of d's components (rcp3)
    template <class PT>
    __device__ __forceinline__ void init(const PT& P, f3 x, f3 d, f3 id, float t0) {
        const int G = P.grid_n;
        const f3 p = fma3(d, t0, x);
        const float pp[3] = {p.x, p.y, p.z}, dd[3] = {d.x, d.y, d.z}, xx[3] = {x.x, x.y, x.z};
        const float ii[3] = {id.x, id.y, id.z};
        int c[3];
        float tm[3], dl[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = min(max((int)floorf((pp[a] - P.bmin[a]) * P.gcell[a]), 0), G - 1);
            if (fabsf(dd[a]) < 1e-20f) {
                tm[a] = 3.402823466e38f;
                dl[a] = 0.0f;
            } else {
                const float inv = ii[a];
                const float plane = fmaf((float)(c[a] + (dd[a] > 0.0f ? 1 : 0)), P.gcw[a], P.bmin[a]);
                tm[a] = (plane - xx[a]) * inv;
                dl[a] = P.gcw[a] * fabsf(inv);
            }
        }
        t = t0;
        const int Gp = G + 2;
        ci = ((c[2] + 1) * Gp + (c[1] + 1)) * Gp + (c[0] + 1);
        sx = d.x > 0.0f ? 1 : -1;
        sy = d.y > 0.0f ? Gp : -Gp;
        sz = d.z > 0.0f ? Gp * Gp : -Gp * Gp;
        tx = tm[0];
        ty = tm[1];
        tz = tm[2];
        dx = dl[0];
        dy = dl[1];
        dz = dl[2];
    }

    // Both tentative points of one iteration in a single walk: point A for
    // tauA (when wantA), then point B for tauB from A.  One loop for both
    // keeps the wave's trip count at the maximum over lanes of the cells both
    // points need, not the sum of two maxima.  Points past the segment come
    // back as tend (their majorant is then not used).
    // One trip handles one cell: point A if it lies in the cell, then point B
    // if it lies in the rest of the same cell, else the exponential variate
    // left over and either the segment's end or a step into the next cell.
    // The arithmetic is that of one point per trip (B's room in the cell is
    // measured from A, with the same majorant and cell exit), so the points
    // are the same; only trips whose cell holds both points or holds A and is
    // then left are merged.  All outcomes are formed with selects, so lanes
    // that take different ones run a trip's instructions once.  mg holds each
    // padded cell's majorant s and the hardware reciprocal of s.  The face
    // crossed first is the one whose boundary equals the minimum, and the
    // cell index moves by that axis's signed stride.  The grid in LDS carries
    // a border of cells that repeat the edge cells, so a step that rounding
    // carries one cell past the grid reads the edge cell's majorant; the
    // segment ends at the box, within rounding of the last face, so no walk
    // goes two cells past it (the index is clamped to the padded grid all the
    // same).  Every step raises the smallest boundary by one cell width along
    // its axis, so the loop reaches tend within
    // 3 (grid_n * segment length / cell width + 2) steps.
    template <class PT>
    __device__ __forceinline__ void next2(const PT& P, const float2* mg, bool wantA, float tauA,
                                          float tauB, float tend, float& tA, float& sbA, float& tB, float& sbB,
                                          uint32_t& steps) {
        const int Gp = P.grid_n + 2, last = Gp * Gp * Gp - 1;
        bool seekA = wantA;  // still looking for A (else for B)
        float tau = wantA ? tauA : tauB;
        tA = t;
        tend = __builtin_canonicalizef(tend);
        // B is found, if at all, in the last trip: its point and majorant are
        // taken from that trip after the loop; A not found by the end of the
        // segment lies at tend
        float s, thb;
        bool hitB;
        for (;;) {
            const float2 m = mg[ci];
            s = m.x;
            const float tmin = fminf(fminf(tx, ty), tz);
            const float te = __builtin_amdgcn_fmed3f(tmin, tend, -3.402823466e38f);  // min(tmin, tend)
            const float room = s * fmaxf(te - t, 0.0f);
            const float th = fmaf(tau, m.y, t);        // the current target's point (s > 0 when it lies here)
            const bool hitA = seekA && tau < room;     // A lies in this cell
            // B from A in the same cell, or B as the current target
            const float tb0 = hitA ? th : t;
            const float taub = hitA ? tauB : tau;
            const float roomb = hitA ? s * fmaxf(te - th, 0.0f) : room;
            thb = hitA ? fmaf(taub, m.y, tb0) : th;
            hitB = (hitA || !seekA) && taub < roomb;
            const bool end = !hitB && te >= tend;        // the segment ends in this cell
            const bool step = !hitB && !end;             // on into the next cell
            tA = hitA ? th : tA;
            sbA = hitA ? s : sbA;
            t = te;
            tau = taub - roomb;
            seekA = seekA && !hitA;
            steps += step ? 1u : 0u;
            const bool bx = tx == tmin, by = !bx && ty == tmin, bz = !bx && !by;
            // (exactly one of bx, by, bz holds: a sum of selects, not an indexed pick)
            const int st = (bx ? sx : 0) + (by ? sy : 0) + (bz ? sz : 0);
            ci = (int)min((unsigned)(ci + st), (unsigned)last);  // (a wrapped index clamps to last)
            tx += bx ? dx : 0.0f;
            ty += by ? dy : 0.0f;
            tz += bz ? dz : 0.0f;
            if (!step) break;
        }
        tA = seekA ? tend : tA;
        tB = hitB ? thb : tend;
        sbB = s;
    }
};

// ---------------------------------------------------------------------------
// Gradient accumulation (kGrad): per-lane cache of the alpha gradient of the
// last LUT pair, flushed into the workgroup's LDS accumulator when the pair
// changes; scale gradient kept in a register.
// ---------------------------------------------------------------------------
struct GradAcc {
    float* lds;     // [lut_n][4]
    int cl0;
    float c0, c1;
    float dscale;
    __device__ __forceinline__ void flush() {
        if (cl0 >= 0) {
            atomicAdd(&lds[cl0 * 4 + 3], c0);
            atomicAdd(&lds[cl0 * 4 + 7], c1);
        }
        cl0 = -1;
        c0 = c1 = 0.0f;
    }
    // d(sigma) = scale * ((1-w) d alpha[l0] + w d alpha[l0+1]) + alpha d scale,
    // scattered with factor f.
    __device__ __forceinline__ void sigma(const TF& t, float scale, float f) {
        if (t.l0 != cl0) {
            flush();
            cl0 = t.l0;
        }
        c0 = fmaf(f * scale, 1.0f - t.w, c0);
        c1 = fmaf(f * scale, t.w, c1);
        dscale = fmaf(f, t.a, dscale);
    }
};

// ---------------------------------------------------------------------------
// Texel store (FP32 / FP16 / BF16, round to nearest even) and wave sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void store_texel(void* out, int dtype, uint64_t k, f3 v) {
    if (dtype == 0) {
        float* o = (float*)out + 3 * k;
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
    } else if (dtype == 1) {
        __half* o = (__half*)out + 3 * k;
        o[0] = __float2half_rn(v.x);
        o[1] = __float2half_rn(v.y);
        o[2] = __float2half_rn(v.z);
    } else {
        uint16_t* o = (uint16_t*)out + 3 * k;
        o[0] = bf16_rne(v.x);
        o[1] = bf16_rne(v.y);
        o[2] = bf16_rne(v.z);
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum64(uint32_t v) {
    unsigned long long w = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    return w;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace lp
