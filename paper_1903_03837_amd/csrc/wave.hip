// wave.hip -- persistent light-field generation kernel (forward, frozen
// sampling, and the path-replay adjoint).
//
// Paths differ wildly in cost: a ray that misses the volume is done after
// one clip, a ray through dense tissue scatters and casts shadow rays.  With
// one ray per lane and all of a ray's samples in a loop, a wave64 runs as
// long as its most expensive lane; measured lane utilisation was 17 %.  Here
// every lane runs its own state machine
//     IDLE -> START -> FLIGHT -> VERTEX -> SHADOW -> SCATTER -> FLIGHT ... -> IDLE
// and each loop iteration advances every lane by one Philox4x32-10 block
// (further passes of the same iteration advance only the lanes still
// tracking a segment, while at least kTrackPass of the 64 do):
//   START   pair 0 jitters the origin, pair 1 is the first tentative collision;
//   FLIGHT  two tentative collisions (delta tracking; the majorant grid is
//           walked from the current point to each of them);
//   VERTEX  light sample and phase-function words (NEE set-up);
//   SHADOW  two ratio-tracking steps towards the light;
//   SCATTER the new direction from the phase words, then as FLIGHT (pairs 0
//           and 1 of the next segment's block 0).
// START, SCATTER and VERTEX run one shared rotation and one shared clip, so
// a wave that holds all three pays for each once.
// Both tentative points of a block are fetched before either is classified,
// so a lane keeps 16 voxel loads in flight.  A lane whose sample ends starts
// the next sample of its work item (a range of one ray's samples) in the
// next iteration; a lane whose work item is done takes the next one of its
// wave's current 8 x 8 tile of rays, and the wave takes a new tile when the
// current one is used up (one atomic per tile).
//
// Ray order: origins and directions are each sorted into latitude bands of
// ~5 sqrt(n) consecutive SF indices, by azimuth inside a band, so a tile's
// 64 rays run between two small patches of S; tiles are taken in groups of 16
// origin tiles sweeping the direction tiles, and the tile sequence is cut into
// 8 contiguous parts, one per XCD (workgroups are dispatched round-robin over
// the XCDs), so each XCD's L2 sees a narrow bundle of rays.  A part that runs
// dry hands out tiles of the next parts.  Results do not depend on the order:
// every random number is keyed by (ray, sample, bounce).
//
// Adjoint mode: the rays with a nonzero adjoint are first compacted into a
// list (in the same spatial order) and the waves take 64-ray chunks of that
// list.  Every sample runs twice: pass A gathers its radiance L_tot, pass B
// replays the same stream and, at every event, adds the event's score times
// the radiance gathered after it (adjoint . (L_tot - L_so_far)) to per-
// workgroup LDS gradients: real collision d sigma / sigma, null collision and
// ratio-tracking step -d sigma / (sigma_bar - sigma), albedo d rho / rho.  A
// shadow ray in pass B runs twice (transmittance first, then its scores,
// which multiply only its own NEE term).  Nothing is stored per path.
#include "internal.hpp"

namespace lp {

// STATS: the work counters of `stats` are kept (a separate instantiation, so
// the plain kernel spends no registers on them).  VIEWS: ground-truth views
// (pinhole rays of pixel tiles) instead of light-field rays, also a separate
// instantiation so that the light-field kernel carries none of its code.
// WAVES: resident waves per SIMD the registers are budgeted for (3: up to 168
// VGPRs; 4: 128, with a few values spilled).  The code and its results are
// the same; four waves hide more latency where HBM has room to spare.
template <int VT, int MODE, bool STATS, bool VIEWS, int WAVES>
__global__ __launch_bounds__(256, WAVES) void gen_wave_kernel(TraceParams P) {
    extern __shared__ float4 smem[];
    float4* lut_e = smem;
    float4* lut_s = smem + (MODE == kFrozen ? P.lut_n : 0);
    float* glds = (float*)(smem + P.lut_n);  // kGrad: dLUT [lut_n][4], dscale
    // cell majorants and their reciprocals after the tables above (8-byte aligned)
    float2* mg = (float2*)((float*)smem + ((4 * P.lut_n * (MODE == kFrozen ? 2 : 1) +
                                            (MODE == kGrad ? 4 * P.lut_n + 1 : 0) + 1) & ~1));
    const int ncell = (P.grid_n + 2) * (P.grid_n + 2) * (P.grid_n + 2);  // padded grid
    for (int e = threadIdx.x; e < P.lut_n; e += blockDim.x) {
        lut_e[e] = ((const float4*)P.lut_e)[e];
        if constexpr (MODE == kFrozen) lut_s[e] = ((const float4*)P.lut_s)[e];
    }
    // the cell majorants with a border that repeats the edge cells
    for (int e = threadIdx.x; e < ncell; e += blockDim.x) {
        const int Gp = P.grid_n + 2, ex = e % Gp, ey = (e / Gp) % Gp, ez = e / (Gp * Gp);
        const int G1 = P.grid_n - 1;
        const int cx = min(max(ex - 1, 0), G1), cy = min(max(ey - 1, 0), G1), cz = min(max(ez - 1, 0), G1);
        const float m = P.maj[(cz * P.grid_n + cy) * P.grid_n + cx];
        mg[e] = make_float2(m, rcp(m));
    }
    if constexpr (MODE == kGrad)
        for (int e = threadIdx.x; e < 4 * P.lut_n + 1; e += blockDim.x) glds[e] = 0.0f;
    __syncthreads();

    const float sigbar = *P.sigbar;
    const int lane = threadIdx.x & 63;
    // Each ray is split into 2^part_log2 work items, ranges of its samples,
    // for load balance (the rays of the last tiles would otherwise hold the
    // grid long after most waves are done).  Adjoint: the scores add up in
    // any order.  Forward with more than one range: each item leaves its
    // partial sum in part_sums, and a second kernel adds the ranges in order.
    const long long nlist = MODE == kGrad ? (long long)*P.ray_count << P.part_log2 : 0;
    const long long ntiles = MODE == kGrad ? (nlist + 63) / 64
                             : VIEWS     ? ((long long)P.nviews * P.vtiles) << P.part_log2
                                         : ((long long)((P.row_end - P.row_begin + 7) / 8) * ((P.N + 7) / 8))
                                               << P.part_log2;
    const int home = blockIdx.x % kParts;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // wave-uniform queue cursor: rays [cur, end) of the current tile
    long long cur = 0, end = 0;
    unsigned dry = 0;
    bool drained = false;

    // lane state
    int mode = kIdle;
    uint32_t k = 0, blk = 0;
    int s = 0, b = 0;
    int s_end = P.spp;  // end of this work item's sample range
    int part = 0;       // its range index
    f3 po = mk3(0, 0, 0), d0 = po, acc = po, x = po, dir = po, T = po, L = po, om = po, C = po;
    float W = 1.0f, t = 0.0f, tend = 0.0f, Tr = 1.0f, up0 = 0.0f, up1 = 0.0f;
    f3 isd = po;  // reciprocals of the current segment's direction (dir or om)
    Counters cnt = {0, 0, 0, 0, 0};
    // adjoint state: texel adjoint / spp, pass A radiance, pass, NEE score weight
    f3 adj = po, ltot = po;
    int pass = 0;
    float rc = 0.0f;
    GradAcc G;
    G.lds = glds;
    G.cl0 = -1;
    G.c0 = G.c1 = 0.0f;
    G.dscale = 0.0f;

    KTraceParams* Pk = (KTraceParams*)__builtin_amdgcn_kernarg_segment_ptr();
    for (;;) {
        // parameters reloaded in each iteration (scalar loads; see KTraceParams)
        asm volatile("" : "+s"(Pk));
        const KTraceParams& P = *Pk;
        const uint32_t K0 = P.key0, K1 = P.key1;
        const int rows = P.row_end - P.row_begin;
        const int tiles_i = (rows + 7) / 8, tiles_j = (P.N + 7) / 8;
        const int plog = P.part_log2;
        const int parts = 1 << plog;
        const float inv_spp = 1.0f / (float)P.spp;
        const f3 O = mk3(P.O[0], P.O[1], P.O[2]);
        const f3 env = mk3(P.env[0], P.env[1], P.env[2]);
        // adding a zero environment leaves a sum of +0 at +0: such sums are skipped
        const bool env_zero = env.x == 0.0f && env.y == 0.0f && env.z == 0.0f;
        const f3 bmin = mk3(P.bmin[0], P.bmin[1], P.bmin[2]), bmax = mk3(P.bmax[0], P.bmax[1], P.bmax[2]);
        // ------------------------------------------------------ sample end
        // (of the samples that ended in the previous iteration's passes)
        if (mode == kDone) {
            bool next = true;
            if constexpr (MODE == kGrad) {
                if (pass == 0) {  // replay the same sample with scores
                    ltot = L;
                    pass = 1;
                    next = false;
                } else {
                    pass = P.srad ? 1 : 0;
                }
            } else {
                acc = acc + L;
                if (P.srad && !VIEWS) {
                    float* o = P.srad + 3 * ((uint64_t)k * (uint32_t)P.spp + (uint32_t)s);
                    o[0] = L.x;
                    o[1] = L.y;
                    o[2] = L.z;
                }
            }
            if (next && ++s == s_end) {
                if constexpr (MODE != kGrad) {
                    if (parts == 1) {
                        const float fs = (float)P.spp;
                        store_texel(P.out, P.dtype, k, mk3(acc.x / fs, acc.y / fs, acc.z / fs));
                    } else {  // this range's sum, for the combining kernel
                        const uint64_t kl = (uint64_t)k - (uint64_t)P.row_begin * (uint32_t)P.N;
                        float* o = P.part_sums + 3 * (kl * parts + part);
                        o[0] = acc.x;
                        o[1] = acc.y;
                        o[2] = acc.z;
                    }
                }
                mode = kIdle;
            } else {
                mode = kStart;
                b = 0;
                blk = 0;
            }
        }

        // ------------------------------------------------------------ refill
        const uint64_t idle = __ballot(mode == kIdle);
        if (idle) {
            const int nidle = __popcll(idle);
            const int rank = __popcll(idle & lt_mask);
            long long avail = end - cur;
            long long fresh = -1;
            if (nidle > avail && !drained) {
                long long tl = 0;
                if (lane == 0) tl = next_tile(P.tile_ctr, ntiles, home, dry);
                tl = __shfl(tl, 0, 64);
                dry = __shfl(dry, 0, 64);
                if (tl < 0) drained = true;
                else fresh = tl * 64;
            }
            long long q = -1;
            if (mode == kIdle) {
                if (rank < avail) q = cur + rank;
                else if (fresh >= 0) q = fresh + (rank - avail);
            }
            if (fresh >= 0) {
                cur = fresh + (nidle - avail);
                end = fresh + 64;
            } else {
                cur += min((long long)nidle, avail);
            }
            if (q >= 0) {
                int i = -1, j = -1;
                // work item q: sample range q mod parts of ray slot q / parts
                int s_first = 0;
                if constexpr (MODE == kGrad) {
                    if (q < nlist) {
                        part = (int)(q & (parts - 1));
                        s_first = (part * P.spp) >> plog;
                        s_end = ((part + 1) * P.spp) >> plog;
                        const uint32_t kk = P.ray_list[q >> plog];
                        i = (int)(kk / (uint32_t)P.N);
                        j = (int)(kk - (uint32_t)i * (uint32_t)P.N);
                        const float* a = P.d_lf + 3 * (uint64_t)kk;
                        adj = mk3(a[0] * inv_spp, a[1] * inv_spp, a[2] * inv_spp);
                        pass = P.srad ? 1 : 0;
                    }
                } else if constexpr (VIEWS) {
                    // pixel of an 8 x 8 tile of a view: the ray from the eye through its centre
                    const long long slot = q >> plog;
                    part = (int)(q & (parts - 1));
                    s_first = (part * P.spp) >> plog;
                    s_end = ((part + 1) * P.spp) >> plog;
                    const uint32_t t = (uint32_t)(slot >> 6);
                    const uint32_t v = t / (uint32_t)P.vtiles, rem = t - v * (uint32_t)P.vtiles;
                    const uint32_t ty = rem / (uint32_t)P.vtx, tx = rem - ty * (uint32_t)P.vtx;
                    const int py = (int)ty * 8 + (int)((slot >> 3) & 7), px = (int)tx * 8 + (int)(slot & 7);
                    if (py < P.H && px < P.W) {
                        const ViewCam& cam = P.views[v];
                        const float ndx = (2.0f * ((float)px + 0.5f) / (float)P.W - 1.0f) * cam.sx;
                        const float ndy = (1.0f - 2.0f * ((float)py + 0.5f) / (float)P.H) * cam.sy;
                        k = (v * (uint32_t)P.H + (uint32_t)py) * (uint32_t)P.W + (uint32_t)px;
                        po = mk3(cam.eye[0], cam.eye[1], cam.eye[2]);
                        d0 = normalize(mk3(cam.fwd[0], cam.fwd[1], cam.fwd[2]) +
                                       mk3(cam.right[0], cam.right[1], cam.right[2]) * ndx +
                                       mk3(cam.up[0], cam.up[1], cam.up[2]) * ndy);
                        acc = mk3(0.0f, 0.0f, 0.0f);
                        s = s_first;
                        b = 0;
                        blk = 0;
                        mode = kStart;
                    }
                } else {
                    const long long slot = q >> plog;
                    part = (int)(q & (parts - 1));
                    s_first = (part * P.spp) >> plog;
                    s_end = ((part + 1) * P.spp) >> plog;
                    int ti, tj;
                    tile_coords(slot >> 6, tiles_i, tiles_j, ti, tj);
                    const int oi = ti * 8 + (int)((slot >> 3) & 7), dj = tj * 8 + (int)(slot & 7);
                    if (oi < rows && dj < P.N) {
                        i = P.perm_o[oi];
                        j = P.perm_d[dj];
                    }
                }
                if (i >= 0) {
                    k = (uint32_t)i * (uint32_t)P.N + (uint32_t)j;
                    if (P.M == P.N && i == j) {
                        // no direction: texel 0 (never listed for the adjoint;
                        // with several ranges the combining kernel writes it)
                        if constexpr (MODE != kGrad)
                            if (parts == 1) store_texel(P.out, P.dtype, k, mk3(0.0f, 0.0f, 0.0f));
                    } else {
                        const float4 a = P.tab_o[i], c = P.tab_d[j];
                        po = mk3(a.x, a.y, a.z);
                        d0 = normalize(mk3(c.x, c.y, c.z) - po);
                        acc = mk3(0.0f, 0.0f, 0.0f);
                        s = s_first;
                        b = 0;
                        blk = 0;
                        mode = kStart;
                        // A ray that misses the volume box in every sample: all
                        // samples of the range but the last are added here (each
                        // is the environment radiance), and the last one runs as
                        // usual.  (The adjoint's ray list leaves such rays out.)
                        if constexpr (MODE != kGrad) {
                            if (misses_box(P, O, bmin, bmax, po, d0)) {
                                if (!env_zero)
                                    for (int s2 = s_first + 1; s2 < s_end; ++s2) acc = acc + env;
                                cnt.samples += (uint32_t)(s_end - 1 - s_first);
                                s = s_end - 1;
                            }
                        }
                    }
                }
            }
        }
        if (__ballot(mode != kIdle) == 0) {
            if (drained && end <= cur) break;
            continue;
        }

        // Passes: the first one draws a block for every lane and runs the
        // set-up of START, SCATTER and VERTEX lanes; further passes, while at
        // least kTrackPass lanes are still tracking a segment, advance only
        // those lanes by one block each.  A lane whose segment needs a set-up
        // or whose sample ended waits for the next iteration, so the set-up
        // and sample-end code runs once per iteration for all such lanes.
        // Every lane still takes the same steps in the same order.
        for (bool first = true;; first = false) {
            // ------------------------------------------------------ one block
            const bool vstream = mode == kVertex || mode == kShadow || mode == kShadow2;
            const u4 r = philox(k, (uint32_t)s, ((uint32_t)b << 8) | (vstream ? kPurVertex : kPurFlight), blk, K0, K1);
            bool stepA = mode == kFlight || mode == kShadow || mode == kShadow2;
            bool stepB = stepA;
            bool sample_done = false, after_shadow = false;

            if (first) {
                // --------------------------------------------------- segment set-up
                // A sample's first segment (START), the segment after a scatter
                // (SCATTER: b already advanced) and the shadow ray of a vertex
                // (VERTEX) share one rotation (START's jitter disk, SCATTER's phase
                // direction) and one clip against the box.
                const bool seg = mode == kStart || mode == kScatter;
                const bool shadow_ray = mode == kVertex && P.light_on;
                f3 Le = mk3(0.0f, 0.0f, 0.0f);
                float dist = 0.0f;
                if (mode == kVertex) {
                    // next-event estimation: light sample (pair 0); phase words (pair 1) kept for the scatter
                    up0 = u01(r.z);
                    up1 = u01(r.w);
                    if (P.light_on) {
                        if (P.light_kind == 0) {
                            om = mk3(P.ldir[0], P.ldir[1], P.ldir[2]);
                            Le = mk3(P.lrad[0], P.lrad[1], P.lrad[2]);
                        } else {
                            const f3 yl = mk3(P.lcorner[0], P.lcorner[1], P.lcorner[2]) +
                                          mk3(P.le1[0], P.le1[1], P.le1[2]) * u01(r.x) +
                                          mk3(P.le2[0], P.le2[1], P.le2[2]) * u01(r.y);
                            const f3 v = yl - x;
                            const float d2 = dot(v, v);
                            const float rinv = rsq(d2);
                            dist = d2 * rinv;
                            om = v * rinv;
                            const float cl = fmaxf(0.0f, -dot(mk3(P.lnrm[0], P.lnrm[1], P.lnrm[2]), om));
                            Le = mk3(P.lrad[0], P.lrad[1], P.lrad[2]) * (cl * P.larea * rcp(d2));
                        }
                    } else {
                        after_shadow = true;
                    }
                } else if (seg) {
                    // base + A (cos(2 pi u) t1 + sin(2 pi u) t2), (t1, t2) completing n
                    f3 n, base;
                    float A, ua;
                    if (mode == kStart) {
                        cnt.samples++;
                        if constexpr (MODE == kGrad) {
                            if (P.srad) {  // the sample's total radiance, kept by the forward
                                const float* lt = P.srad + 3 * ((uint64_t)k * (uint32_t)P.spp + (uint32_t)s);
                                ltot = mk3(lt[0], lt[1], lt[2]);
                            }
                        }
                        // light-field ray: origin on S (jittered); view ray: the eye
                        base = VIEWS ? po : O + po * P.R;
                        n = po;
                        A = (P.jitter && !VIEWS) ? P.jit_rad * sqrtf(u01(r.x)) : 0.0f;
                        ua = u01(r.y);
                        T = mk3(1.0f, 1.0f, 1.0f);
                        W = 1.0f;
                        L = mk3(0.0f, 0.0f, 0.0f);
                    } else {
                        const float mu = hg_mu(P.g, up0);
                        A = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
                        base = dir * mu;
                        n = dir;
                        ua = up1;
                    }
                    float sa, ca;
                    sincospif(2.0f * ua, &sa, &ca);
                    f3 t1, t2;
                    frame(n, t1, t2);
                    const f3 v = base + t1 * (A * ca) + t2 * (A * sa);
                    if (mode == kStart) {
                        x = v;
                        dir = d0;
                    } else {
                        dir = v;
                    }
                }
                if (seg || shadow_ray) {
                    float tn, tf;
                    const f3 cd = shadow_ray ? om : dir;
                    isd = rcp3(cd);  // kept for the grid walks of this segment
                    const bool hit = clip_box(bmin, bmax, x, cd, isd, tn, tf);
                    if (shadow_ray) {
                        const float te = hit ? (P.light_kind == 0 ? tf : fminf(dist, tf)) : 0.0f;
                        C = T * Le * (W * hg_phase(P.g, dot(dir, om)));
                        Tr = 1.0f;
                        if (sigbar > 0.0f) {
                            t = 0.0f;
                            tend = te;
                            mode = kShadow;
                            blk = 1;
                        } else {
                            L = L + C;
                            after_shadow = true;
                        }
                    } else if (hit && sigbar > 0.0f) {
                        // START: pair 1 is the first tentative collision (pair 0 was the
                        // jitter); SCATTER: pairs 0 and 1
                        stepA = mode == kScatter;
                        stepB = true;
                        t = tn;
                        tend = tf;
                        mode = kFlight;
                    } else {
                        L = L + T * env * W;
                        sample_done = true;
                    }
                }

            }

            // -------------------------------------------- two tentative points
            bool ev_end = false, ev_real = false;
            f3 ynew = x;
            TF te;
            te.l0 = 0;
            te.w = 0.0f;
            te.a = te.a_s = 0.0f;
            if (stepA || stepB) {
                // (stepB always holds here; stepA is off for the first point of a sample)
                const f3 sd = mode == kFlight ? dir : om;
                GridWalk gw;
                gw.init(P, x, sd, isd, t);
                float sbA = 0.0f, sbB = 0.0f, tA, tB;
                // The walk is a chain of dependent steps (an LDS read of the
                // cell's majorant, then ~40 instructions) that the wave's
                // slowest lane drags out; raised wave priority lets it issue
                // ahead of the other waves of its SIMD, whose volume loads are
                // in flight meanwhile.  With 3 waves per SIMD (the HBM-bound
                // budget) the volume fetch that follows runs at that priority
                // too; with 4 it must not (20 % slower).  Scheduling only:
                // the same instructions and results.  Measured in the forward
                // modes (N = 32768 at 3 waves 4524 -> 4465 -> 4370 ms, N = 8192
                // at 4 waves 741 -> 729 ms); the adjoint keeps the default.
                if constexpr (MODE != kGrad) __builtin_amdgcn_s_setprio(2);
                gw.next2(P, mg, stepA, neg_log1m(u01(r.x)), neg_log1m(u01(r.z)), tend, tA, sbA, tB, sbB, cnt.cells);
                if constexpr (MODE != kGrad) __builtin_amdgcn_s_setprio(0);
                const f3 yA = fma3(sd, tA, x), yB = fma3(sd, tB, x);
                if constexpr (MODE != kGrad && WAVES == 3) __builtin_amdgcn_s_setprio(2);
                const float rawA = sample_volume<VT>(P, yA);
                const float rawB = sample_volume<VT>(P, yB);
                if constexpr (MODE != kGrad && WAVES == 3) __builtin_amdgcn_s_setprio(0);
                bool more = true;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bool use = h ? stepB : stepA;
                    if (!use || !more) continue;
                    const float th = h ? tB : tA;
                    if (th >= tend) {
                        ev_end = true;
                        more = false;
                        continue;
                    }
                    const TF tf = classify<MODE>(P, lut_e, lut_s, h ? rawB : rawA);
                    const float sig_e = P.scale_e * tf.a;
                    const float sb = h ? sbB : sbA;  // majorant of the point's cell
                    t = th;
                    if (mode == kFlight) {
                        cnt.tent++;
                        const float sig_s = MODE == kFrozen ? P.scale_s * tf.a_s : sig_e;
                        if (u01(h ? r.w : r.y) * sb < sig_s) {
                            ev_real = true;
                            more = false;
                            ynew = h ? yB : yA;
                            te = tf;
                            if constexpr (MODE == kFrozen) W *= sig_e / sig_s;
                            if constexpr (MODE == kGrad)
                                if (pass) G.sigma(tf, P.scale_e, dot(adj, ltot - L) / sig_e);
                        } else {
                            if constexpr (MODE == kFrozen) W *= (sb - sig_e) / (sb - sig_s);
                            if constexpr (MODE == kGrad)
                                if (pass) G.sigma(tf, P.scale_e, -dot(adj, ltot - L) / (sb - sig_e));
                        }
                    } else if (mode == kShadow) {
                        cnt.shadow++;
                        Tr *= 1.0f - sig_e * rcp(sb);
                    } else {
                        if constexpr (MODE == kGrad) G.sigma(tf, P.scale_e, -rc / (sb - sig_e));
                    }
                }
                if (ev_end) {
                    if (mode == kFlight) {
                        L = L + T * env * W;
                        sample_done = true;
                    } else if (MODE == kGrad && mode == kShadow && pass) {
                        // transmittance known: replay the shadow ray for its scores
                        rc = dot(adj, C * Tr);
                        if (rc != 0.0f) {
                            mode = kShadow2;
                            blk = 1;
                            t = 0.0f;
                        } else {
                            L = L + C * Tr;
                            after_shadow = true;
                        }
                    } else {
                        L = L + C * Tr;
                        after_shadow = true;
                    }
                } else if (ev_real) {
                    cnt.real++;
                    const f3 rgb = tf_rgb(lut_e, te);
                    if constexpr (MODE == kGrad) {
                        if (pass) {
                            // albedo scores d rho_c / rho_c times the channel's later radiance
                            const f3 after = (ltot - L) * adj;
                            const float ra[3] = {rgb.x, rgb.y, rgb.z};
                            const float af[3] = {after.x, after.y, after.z};
#pragma unroll
                            for (int c = 0; c < 3; ++c)
                                if (ra[c] > 0.0f && ra[c] < 1.0f && af[c] != 0.0f) {
                                    const float f = af[c] / ra[c];
                                    atomicAdd(&glds[te.l0 * 4 + c], f * (1.0f - te.w));
                                    atomicAdd(&glds[te.l0 * 4 + 4 + c], f * te.w);
                                }
                        }
                    }
                    x = ynew;
                    T = T * mk3(__builtin_amdgcn_fmed3f(rgb.x, 0.0f, 1.0f), __builtin_amdgcn_fmed3f(rgb.y, 0.0f, 1.0f),
                                __builtin_amdgcn_fmed3f(rgb.z, 0.0f, 1.0f));
                    if (T.x == 0.0f && T.y == 0.0f && T.z == 0.0f) {
                        sample_done = true;
                    } else {
                        mode = kVertex;
                        blk = 0;
                    }
                } else if (++blk >= kMaxBlocks) {
                    // stream exhausted: the segment ends absorbed / blocked
                    if (mode == kFlight) {
                        sample_done = true;
                    } else {
                        Tr = 0.0f;  // C * 0 adds nothing
                        after_shadow = true;
                    }
                }
            }

            // ------------------------------------------------ scatter direction
            // (drawn at the start of the next iteration, from the phase words)
            if (after_shadow) {
                if (b == P.maxb - 1) {
                    sample_done = true;
                } else {
                    ++b;
                    blk = 0;
                    mode = kScatter;
                }
            }

            if (sample_done) mode = kDone;
            if (__popcll(__ballot(mode == kFlight || mode == kShadow || mode == kShadow2)) < kTrackPass) break;
        }
    }

    if constexpr (MODE == kGrad) {
        G.flush();
        const float ds = wave_sumf(G.dscale);
        if (lane == 0) atomicAdd(&glds[4 * P.lut_n], ds);
        __syncthreads();
        for (int e = threadIdx.x; e < 4 * P.lut_n; e += blockDim.x)
            if (glds[e] != 0.0f) atomicAdd(&P.d_lut[e], glds[e]);
        if (threadIdx.x == 0 && glds[4 * P.lut_n] != 0.0f) atomicAdd(P.d_scale, glds[4 * P.lut_n]);
        return;
    }

    if (STATS) {
        const uint32_t a = wave_sum(cnt.tent), c = wave_sum(cnt.shadow), e = wave_sum(cnt.real),
                       f = wave_sum(cnt.samples);
        const unsigned long long cs = wave_sum64(cnt.cells);
        if (lane == 0) {
            atomicAdd(&P.stats[0], (unsigned long long)a);
            atomicAdd(&P.stats[1], (unsigned long long)c);
            atomicAdd(&P.stats[2], (unsigned long long)e);
            atomicAdd(&P.stats[3], (unsigned long long)f);
            atomicAdd(&P.stats[4], cs);
        }
    }
}

// Spatial order of count consecutive SF indices base..base+count-1 of a set
// of n points: bands of B indices, each sorted by azimuth (rank counting).
// One workgroup per band, its azimuths staged in LDS (B <= 1272 for
// n <= 65535).
constexpr int kMaxBand = 1280;
__global__ __launch_bounds__(256) void sf_order_kernel(int base, int count, int band, int32_t* out) {
    __shared__ float fr[kMaxBand];
    const int lo = blockIdx.x * band;
    const int cnt = min(count - lo, band);
    for (int t = (int)threadIdx.x; t < cnt; t += 256) fr[t] = sf_frac(base + lo + t);
    __syncthreads();
    for (int t = (int)threadIdx.x; t < cnt; t += 256) {
        const float fe = fr[t];
        int rank = 0;
        for (int f = 0; f < cnt; ++f) {
            const float ff = fr[f];
            rank += ff < fe || (ff == fe && f < t);
        }
        out[lo + rank] = base + lo + t;
    }
}

// Compacts the rays (in the spatial tile order) whose adjoint is nonzero and
// which can reach the volume box (a ray that misses it in every sample has no
// collision and so no score).
// One atomic per workgroup and trip claims the list slots of its four waves
// (one per wave made the single counter the bottleneck).
__global__ __launch_bounds__(256) void active_rays_kernel(TraceParams P) {
    __shared__ unsigned wave_n[4], wave_at[4];
    const int rows = P.row_end - P.row_begin;
    const int tiles_i = (rows + 7) / 8, tiles_j = (P.N + 7) / 8;
    const long long total = (long long)tiles_i * tiles_j * 64;
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long base = (long long)blockIdx.x * blockDim.x; base < total; base += stride) {
        const long long q = base + threadIdx.x;
        bool take = false;
        uint32_t k = 0;
        if (q < total) {
            int ti, tj;
            tile_coords(q >> 6, tiles_i, tiles_j, ti, tj);
            const int oi = ti * 8 + (int)((q >> 3) & 7), dj = tj * 8 + (int)(q & 7);
            if (oi < rows && dj < P.N) {
                const int i = P.perm_o[oi], j = P.perm_d[dj];
                k = (uint32_t)i * (uint32_t)P.N + (uint32_t)j;
                const float* a = P.d_lf + 3 * (uint64_t)k;
                take = !(P.M == P.N && i == j) && (a[0] != 0.0f || a[1] != 0.0f || a[2] != 0.0f);
                if (take) {
                    const float4 a = P.tab_o[i], c = P.tab_d[j];
                    const f3 po = mk3(a.x, a.y, a.z);
                    const f3 d0 = normalize(mk3(c.x, c.y, c.z) - po);
                    take = !misses_box(P, mk3(P.O[0], P.O[1], P.O[2]), mk3(P.bmin[0], P.bmin[1], P.bmin[2]),
                                       mk3(P.bmax[0], P.bmax[1], P.bmax[2]), po, d0);
                }
            }
        }
        const uint64_t m = __ballot(take);
        const int wave = threadIdx.x >> 6;
        if (lane == 0) wave_n[wave] = (unsigned)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned n0 = wave_n[0], n1 = wave_n[1], n2 = wave_n[2], n3 = wave_n[3];
            const unsigned tot = n0 + n1 + n2 + n3;
            const unsigned at = tot ? atomicAdd(P.ray_count, tot) : 0u;
            wave_at[0] = at;
            wave_at[1] = at + n0;
            wave_at[2] = at + n0 + n1;
            wave_at[3] = at + n0 + n1 + n2;
        }
        __syncthreads();
        if (take) P.ray_list[wave_at[wave] + __popcll(m & lt_mask)] = k;
        __syncthreads();  // wave_n / wave_at are rewritten by the next trip
    }
}

__global__ void wave_setup_kernel(const float* lut, int n, float scale, float given, float* sigbar,
                                  unsigned int* ctr) {
    __shared__ float red[256];
    float m = 0.0f;
    for (int e = threadIdx.x; e < n; e += 256) m = fmaxf(m, lut[4 * e + 3]);
    red[threadIdx.x] = m;
    if (threadIdx.x < kParts + 1) ctr[threadIdx.x] = 0u;  // tile counters, then the list length
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) sigbar[0] = given > 0.0f ? given : 1.25f * scale * red[0];
}

static int band_size(int n) {
    int b = (int)(5.0 * std::sqrt((double)n));
    b &= ~7;
    return b < 8 ? 8 : b;
}

hipError_t launch_wave_setup(const TraceParams& P, const float* sample_lut, int lut_n, float sample_scale,
                             float given, float* sigbar, unsigned int* ctr, int32_t* perm_o, int32_t* perm_d,
                             hipStream_t s) {
    wave_setup_kernel<<<1, 256, 0, s>>>(sample_lut, lut_n, sample_scale, given, sigbar, ctr);
    const int rows = P.row_end - P.row_begin;
    const int bo = band_size(P.M), bd = band_size(P.N);
    if (rows > 0) sf_order_kernel<<<(rows + bo - 1) / bo, 256, 0, s>>>(P.row_begin, rows, bo, perm_o);
    sf_order_kernel<<<(P.N + bd - 1) / bd, 256, 0, s>>>(0, P.N, bd, perm_d);
    return hipGetLastError();
}

hipError_t launch_active_rays(const TraceParams& P, hipStream_t s) {
    const long long rows = P.row_end - P.row_begin;
    const long long total = ((rows + 7) / 8) * (long long)((P.N + 7) / 8) * 64;
    if (total <= 0) return hipSuccess;
    long long blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    active_rays_kernel<<<(unsigned)blocks, 256, 0, s>>>(P);
    return hipGetLastError();
}

template <int VT, int MODE, bool STATS, bool VIEWS, int WAVES>
static hipError_t launch_wave_w(const TraceParams& P, hipStream_t s) {
    const long long rows = P.row_end - P.row_begin;
    const long long ntiles = (P.views ? (long long)P.nviews * P.vtiles : ((rows + 7) / 8) * (long long)((P.N + 7) / 8))
                             << P.part_log2;
    if (ntiles <= 0) return hipSuccess;
    const size_t ncell = (size_t)(P.grid_n + 2) * (P.grid_n + 2) * (P.grid_n + 2);  // padded grid in LDS
    const size_t lds = sizeof(float4) * (size_t)P.lut_n * (MODE == kFrozen ? 2 : 1) +
                       (MODE == kGrad ? sizeof(float) * (4 * (size_t)P.lut_n + 1) : 0) + sizeof(float) +
                       sizeof(float2) * ncell;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gen_wave_kernel<VT, MODE, STATS, VIEWS, WAVES>, 256,
                                                         lds);
    if (e != hipSuccess) return e;
    long long blocks = (long long)cus * (per_cu > 0 ? per_cu : 1);
    // at least one tile per wave (list lengths are only known on the device;
    // waves that find no chunk exit at once)
    const long long need = (ntiles + 3) / 4;
    if (blocks > need) blocks = need;
    gen_wave_kernel<VT, MODE, STATS, VIEWS, WAVES><<<(unsigned)blocks, 256, lds, s>>>(P);
    return hipGetLastError();
}

// The adjoint is budgeted for three waves (at four it spills ~32 values and
// runs slower); the forward modes take P.waves.
template <int VT, int MODE, bool STATS, bool VIEWS>
static hipError_t launch_wave_t(const TraceParams& P, hipStream_t s) {
    if constexpr (MODE != kGrad)
        if (P.waves == 4) return launch_wave_w<VT, MODE, STATS, VIEWS, 4>(P, s);
    return launch_wave_w<VT, MODE, STATS, VIEWS, 3>(P, s);
}

template <int VT>
static hipError_t launch_wave_mode(const TraceParams& P, int mode, hipStream_t s) {
    if (P.views) return launch_wave_t<VT, kFwd, false, true>(P, s);  // ground-truth views: plain forward
    if (mode == kGrad) return launch_wave_t<VT, kGrad, false, false>(P, s);
    if (P.stats)
        return mode == kFrozen ? launch_wave_t<VT, kFrozen, true, false>(P, s)
                               : launch_wave_t<VT, kFwd, true, false>(P, s);
    return mode == kFrozen ? launch_wave_t<VT, kFrozen, false, false>(P, s)
                           : launch_wave_t<VT, kFwd, false, false>(P, s);
}

// Light-field texels from the sample ranges: the ranges' sums in range
// order, divided by spp (texels i == j are 0).
__global__ void combine_parts_kernel(TraceParams P, long long n) {
    const long long kl = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (kl >= n) return;
    const int parts = 1 << P.part_log2;
    bool none = false;  // texel i == j of the light field
    uint32_t k = (uint32_t)kl;  // views: the pixel
    if (!P.views) {
        const uint32_t i = (uint32_t)P.row_begin + (uint32_t)(kl / P.N), j = (uint32_t)(kl % P.N);
        k = i * (uint32_t)P.N + j;
        none = P.M == P.N && i == j;
    }
    f3 acc = mk3(0.0f, 0.0f, 0.0f);
    if (!none) {
        const float* p = P.part_sums + 3 * (uint64_t)kl * parts;
        acc = mk3(p[0], p[1], p[2]);
        for (int q = 1; q < parts; ++q) acc = acc + mk3(p[3 * q], p[3 * q + 1], p[3 * q + 2]);
        const float fs = (float)P.spp;
        acc = mk3(acc.x / fs, acc.y / fs, acc.z / fs);
    }
    store_texel(P.out, P.dtype, k, acc);
}

hipError_t launch_combine_parts(const TraceParams& P, hipStream_t s) {
    const long long n = P.views ? (long long)P.nviews * P.H * P.W : (long long)(P.row_end - P.row_begin) * P.N;
    if (n <= 0) return hipSuccess;
    combine_parts_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, n);
    return hipGetLastError();
}

hipError_t launch_generate_wave(const TraceParams& P, int vtype, int mode, hipStream_t s) {
    switch (vtype) {
        case 0: return launch_wave_mode<0>(P, mode, s);
        case 1: return launch_wave_mode<1>(P, mode, s);
        default: return launch_wave_mode<2>(P, mode, s);
    }
}

}  // namespace lp
