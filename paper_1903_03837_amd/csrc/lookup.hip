// lookup.hip -- image synthesis from the light field (Sec. 2, Fig. 2) and
// its transpose.
//
// One lane per pixel; a wave64 covers an 8 x 8 pixel tile and a workgroup a
// 16 x 16 tile, so neighbouring lanes query neighbouring points of both SF
// sets and their K x K texel gathers hit the same cache lines.  Per pixel:
// view ray -> front/back hits on S (tangential rays discarded) -> O(1)
// inverse SF mapping of each hit -> K nearest of the nine lattice
// candidates -> tent weights -> K x K gathers (25 at K = 5) -> normalised
// blend.  The adjoint sums each wave's contributions before its atomics:
// as a dense contraction over the wave's 64 pixels on MFMA when the wave's
// distinct origin and direction neighbours fit dictionaries of 8 (most
// waves at view resolution), else over each half of the wave's tile, and
// for a half that still overflows per pair slot after sorting each
// pixel's neighbour lists by index (neighbouring pixels then hold equal
// texels in equal slots, which are summed across the wave with DPP).  One
// float atomic per channel is issued per distinct texel of each
// contraction or pair slot.
#include <hip/hip_fp16.h>

#include <mutex>

#include "internal.hpp"
#include "sf_search.hpp"

namespace lp {

// Texel at byte address p of a light field of type DT.
template <int DT>
__device__ __forceinline__ f3 load_texel_at(const char* p) {
    if constexpr (DT == 0) {
        const float* q = (const float*)p;
        return mk3(q[0], q[1], q[2]);
    } else if constexpr (DT == 1) {
        const __half* q = (const __half*)p;
        return mk3(__half2float(q[0]), __half2float(q[1]), __half2float(q[2]));
    } else {
        const uint16_t* q = (const uint16_t*)p;
        return mk3(__uint_as_float((uint32_t)q[0] << 16), __uint_as_float((uint32_t)q[1] << 16),
                   __uint_as_float((uint32_t)q[2] << 16));
    }
}
template <int DT>
constexpr int texel_bytes() { return DT == 0 ? 12 : 6; }

template <int DT>
__device__ __forceinline__ f3 load_texel(const void* lf, uint64_t t) {
    if constexpr (DT == 0) {
        const float* p = (const float*)lf + 3 * t;
        return mk3(p[0], p[1], p[2]);
    } else if constexpr (DT == 1) {
        const __half* p = (const __half*)lf + 3 * t;
        return mk3(__half2float(p[0]), __half2float(p[1]), __half2float(p[2]));
    } else {
        const uint16_t* p = (const uint16_t*)lf + 3 * t;
        return mk3(__uint_as_float((uint32_t)p[0] << 16), __uint_as_float((uint32_t)p[1] << 16),
                   __uint_as_float((uint32_t)p[2] << 16));
    }
}

// Sort (idx, w) pairs by index (static compare-exchange passes, registers
// only).  In the adjoint this makes neighbouring pixels, which share their
// neighbour sets, list the same texel in the same pair slot.
template <int KMAX>
__device__ __forceinline__ void sort_by_index(int* idx, float* w) {
#pragma unroll
    for (int p = 0; p < KMAX; ++p)
#pragma unroll
        for (int a = (p & 1); a + 1 < KMAX; a += 2) {
            const unsigned ia = (unsigned)idx[a], ib = (unsigned)idx[a + 1];  // -1 sorts last
            if (ib < ia) {
                const int ti = idx[a];
                idx[a] = idx[a + 1];
                idx[a + 1] = ti;
                const float tw = w[a];
                w[a] = w[a + 1];
                w[a + 1] = tw;
            }
        }
}

// The pixel's view ray and its front and back hits on the unit sphere S,
// with the same arithmetic in every lookup kernel, so that the forward
// lookup, the fused lookup + loss and the transpose weigh the same
// neighbours by the same weights.  Square roots, normalisations and
// divisions use the hardware square root, reciprocal square root and
// reciprocal (v_sqrt_f32, v_rsq_f32, v_rcp_f32, about an ulp each; 1-2
// instructions where a correctly rounded square root or an IEEE division
// takes ~10): a hit moves by a few 1e-7 of the radius either way.  Returns false for a ray that misses S or grazes
// it (discriminant at most thr).
__device__ __forceinline__ f3 normalize_rsq(f3 a) { return a * __builtin_amdgcn_rsqf(dot(a, a)); }
__device__ __forceinline__ bool view_hits(const LookupParams& P, const ViewGeom& G, int px, int py, f3& qo, f3& qd) {
    const float ndx = (2.0f * ((float)px + 0.5f) * __builtin_amdgcn_rcpf((float)P.W) - 1.0f) * G.sx;
    const float ndy = (1.0f - 2.0f * ((float)py + 0.5f) * __builtin_amdgcn_rcpf((float)P.H)) * G.sy;
    const f3 d = normalize_rsq(mk3(G.fwd[0], G.fwd[1], G.fwd[2]) + mk3(G.right[0], G.right[1], G.right[2]) * ndx +
                               mk3(G.up[0], G.up[1], G.up[2]) * ndy);
    const f3 oc = mk3(G.oc[0], G.oc[1], G.oc[2]);
    const float b = dot(d, oc);
    const float disc = b * b - G.c;
    if (!(disc > P.thr)) return false;
    const float sq = __builtin_amdgcn_sqrtf(disc);
    qo = normalize_rsq(fma3(d, -b - sq, oc));
    qd = normalize_rsq(fma3(d, -b + sq, oc));
    return true;
}
// 1 / (sum of a pixel's pair weights), positive and normal, by the hardware
// reciprocal.
__device__ __forceinline__ float inv_weight_sum(float wsum) { return __builtin_amdgcn_rcpf(wsum); }
// Tent weight of a neighbour at squared chord d2 (filter radius 1 / inv_r),
// with the hardware square root.
__device__ __forceinline__ float tent_weight_hw(float d2, float inv_r) {
    return fmaxf(0.0f, 1.0f - __builtin_amdgcn_sqrtf(d2) * inv_r);
}

// Separable blend.  When no pair (a, c) of a pixel is degenerate (origin
// and direction neighbour the same point of one set), its pair weights are
// the products wa[a] wb[c], so the weight sum is (sum wa)(sum wb) and the
// view is sum_a wa[a] (sum_c wb[c] T[a][c]) / that sum: 3 multiply-adds per
// texel and 3 per row, against a product, a scaled product and 3
// multiply-adds per texel and a product and a sum per pair for the
// per-pair form.  A pair's point would lie within sqrt(da) of q_o and
// sqrt(db) of q_d, so |q_o - q_d|^2 <= 2 (da + db); with a 10 % margin
// over the FP32 roundings, a chord above 2.2 (da + db) of the farthest kept
// neighbours (the selection leaves distances in ascending order, invalid
// entries last) rules every pair out.  The decision is taken per wave (a
// ballot over the lanes with a pixel on S), in the same way in the forward
// lookup and the fused lookup + loss, so both form each view value with
// the same arithmetic.
// The light field (stored origin rows x N texels of its storage type)
// spans at most 4 GiB.
__host__ __device__ inline bool field_within_4gib(const LookupParams& P) {
    return (uint64_t)P.orows * (uint64_t)P.N * (uint64_t)(P.dtype == 0 ? 12 : 6) <= (1ull << 32);
}
template <int KMAX>
__device__ __forceinline__ bool separable_wave(const LookupParams& P, f3 qo, f3 qd, const float* da, const float* db) {
    const bool maybe_bad = P.degenerate && !(dist2(qo, qd) > 2.2f * (da[KMAX - 1] + db[KMAX - 1]));
    return __ballot(maybe_bad) == 0;
}
template <int KMAX>
__device__ __forceinline__ float separable_weight_sum(const float* wa, const float* wb) {
    float sa = 0.0f, sb = 0.0f;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        sa += wa[a];
        sb += wb[a];
    }
    return sa * sb;
}
// Per-pair weight sum: degenerate pairs left out when the sets are one.
template <int KMAX>
__device__ __forceinline__ float pair_weight_sum(const LookupParams& P, const int* ia, const float* wa, const int* jb,
                                                 const float* wb) {
    float wsum = 0.0f;
#pragma unroll
    for (int a = 0; a < KMAX; ++a)
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            const bool bad = P.degenerate && ia[a] == jb[c];
            wsum += bad ? 0.0f : wa[a] * wb[c];
        }
    return wsum;
}
// One origin row of the separable blend: acc += wa (sum_c wb[c] T[c]).
template <int KMAX>
__device__ __forceinline__ f3 blend_row(const f3* T, const float* wb, float wa, f3 acc) {
    f3 r = mk3(0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int c = 0; c < KMAX; ++c) r = fma3(T[c], wb[c], r);
    return fma3(r, wa, acc);
}

// DPP lane move (a v_mov_b32_dpp): lanes that the row / bank masks disable,
// or whose source lies outside the row under bound_ctrl, read `old`.
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_CTRL>
__device__ __forceinline__ float dpp(float old, float src) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, ROW_MASK, BANK_MASK, BOUND_CTRL));
}

// Sum over the 64 lanes of a wave (all lanes active), left in lane 63:
// prefix sums of 4 inside each 16-lane row, then of 8 and 16 (row_shr), then
// the rows joined by the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ float wave_sum_lane63(float v) {
    float s = v + dpp<0x111, 0xf, 0xf, true>(0.0f, v);  // row_shr:1
    s = s + dpp<0x112, 0xf, 0xf, true>(0.0f, v);        // row_shr:2
    s = s + dpp<0x113, 0xf, 0xf, true>(0.0f, v);        // row_shr:3
    s = s + dpp<0x114, 0xf, 0xe, false>(0.0f, s);       // row_shr:4, lanes 4..15 of each row
    s = s + dpp<0x118, 0xf, 0xc, false>(0.0f, s);       // row_shr:8, lanes 8..15
    s = s + dpp<0x142, 0xa, 0xf, false>(0.0f, s);       // row_bcast:15 into rows 1 and 3
    s = s + dpp<0x143, 0xc, 0xf, false>(0.0f, s);       // row_bcast:31 into rows 2 and 3
    return s;
}

// Wave-aggregated scatter-add of a 3-vector: lanes holding the same texel
// are summed across the wave (DPP) and lane 63 issues the three atomics.
// Each pass retires every lane whose key equals the first pending lane's.
// Called with every lane of the wave active.
__device__ __forceinline__ void wave_scatter_add(float* d_lf, bool pending, uint64_t key, f3 v) {
    const int lane = threadIdx.x & 63;
    uint64_t live = __ballot(pending);
    while (live) {
        const int leader = __ffsll((long long)live) - 1;
        const uint64_t lk = __shfl(key, leader, 64);
        const bool mine = pending && key == lk;
        const float a = wave_sum_lane63(mine ? v.x : 0.0f);
        const float b = wave_sum_lane63(mine ? v.y : 0.0f);
        const float c = wave_sum_lane63(mine ? v.z : 0.0f);
        if (lane == 63) {
            float* dl = d_lf + 3 * lk;
            atomicAdd(dl + 0, a);
            atomicAdd(dl + 1, b);
            atomicAdd(dl + 2, c);
        }
        pending = pending && !mine;
        live = __ballot(pending);
    }
}

// Per-wave LDS of the MFMA scatter: the weight rows of the wave's 64 pixels
// over its dictionaries of distinct origin and direction texel indices.
constexpr int kDict = 8;
struct ScatterLds {
    float u[64 * kDict];  // [pixel][origin entry]: w_a / sum of pair weights
    float v[64 * kDict];  // [pixel][direction entry]: w_b
    float g[64 * 3];      // [pixel][channel]: the pixel's adjoint dimg
    int dict[2 * kDict];  // origin indices, then direction indices
};

// Builds the wave's dictionary of the distinct values among the flagged
// entries val[s] of all lanes, and each entry's position in it (-1 for an
// unflagged entry).  The loop is wave-uniform: each pass takes the value of
// the first lane with a pending entry in slot s and retires every entry
// equal to it.  Returns the dictionary size, or -1 if it would exceed kDict.
template <int KMAX>
__device__ __forceinline__ int wave_dictionary(const int (&val)[KMAX], bool (&pend)[KMAX], int (&pos)[KMAX],
                                               int* dict) {
    int n = 0;
#pragma unroll
    for (int s = 0; s < KMAX; ++s) pos[s] = -1;
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        uint64_t m = __ballot(pend[s]);
        while (m) {
            if (n == kDict) return -1;
            const int leader = __ffsll((long long)m) - 1;
            const int x = __builtin_amdgcn_readlane(val[s], leader);
            // slots before s hold no pending entry, and no value twice in a lane
#pragma unroll
            for (int t = s; t < KMAX; ++t) {
                const bool hit = pend[t] && val[t] == x;
                pos[t] = hit ? n : pos[t];
                pend[t] = pend[t] && !hit;
            }
            if ((threadIdx.x & 63) == 0) dict[n] = x;
            ++n;
            m = __ballot(pend[s]);
        }
    }
    return n;
}

// Wave-level LDS ordering: every lane's writes before, every lane's reads after.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The adjoint scatter of a wave as a dense contraction over its 64 pixels:
// with dictionaries A (origin indices) and B (direction indices) of the
// wave's texels, d_lf[A_x][B_y][ch] += sum_p u_p[x] v_p[y] g_p[ch], where
// u_p / v_p hold pixel p's normalised origin / direction weights at its own
// entries and 0 elsewhere.  A pair (a, b) that no pixel holds gets exactly
// 0, and a degenerate pair (a == b, same SF set) only ever collects
// excluded pairs, so both are skipped, as the per-pair scatter skips them.
// Two v_mfma_f32_16x16x4_f32 chains over the pixels, 4 per instruction:
// rows are u (rows 8..15 repeat 0..7); the first chain's columns are v * g0
// (0..7) and v * g1 (8..15), the second's v * g2, so rows 0..7 of the first
// hold channels 0 and 1 and the top-left block of the second channel 2 (one
// product per instruction cannot hold all three: a fourth block of scaled
// rows times scaled columns would need a quotient of channels).
// Returns false (nothing written to d_lf) when a
// dictionary would exceed kDict entries or an adjoint value is not finite
// (a zero weight times an infinite one would spread NaN over other texels).
template <int KMAX>
__device__ __forceinline__ bool mfma_scatter(const LookupParams& P, ScatterLds& L, bool live, const int (&ia)[KMAX],
                                             const float (&wa)[KMAX], const int (&jb)[KMAX],
                                             const float (&wb)[KMAX], float inv, f3 gi) {
    const int lane = threadIdx.x & 63;
    const bool finite = isfinite(gi.x) && isfinite(gi.y) && isfinite(gi.z);
    if (__ballot(!finite)) return false;
    float u[KMAX];
    bool pa[KMAX], pb[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        u[a] = wa[a] * inv;
        pa[a] = live && ia[a] >= 0 && ia[a] < P.orows && u[a] != 0.0f;
        pb[a] = live && jb[a] >= 0 && wb[a] != 0.0f;
    }
    int xa[KMAX], xb[KMAX];
    const int na = wave_dictionary<KMAX>(ia, pa, xa, L.dict);
    if (na < 0) return false;
    const int nb = wave_dictionary<KMAX>(jb, pb, xb, L.dict + kDict);
    if (nb < 0) return false;
    if (na == 0 || nb == 0) return true;  // no weighted pair in the wave

    float* ur = L.u + lane * kDict;
    float* vr = L.v + lane * kDict;
    *(float4*)ur = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    *(float4*)(ur + 4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    *(float4*)vr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    *(float4*)(vr + 4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        if (xa[a] >= 0) ur[xa[a]] = u[a];
        if (xb[a] >= 0) vr[xb[a]] = wb[a];
    }
    L.g[3 * lane + 0] = gi.x;
    L.g[3 * lane + 1] = gi.y;
    L.g[3 * lane + 2] = gi.z;
    wave_lds_sync();

    // A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k (k: pixel 4 kb + k)
    const int col = lane & 7, kq = lane >> 4;
    const bool hi = (lane & 15) >= kDict;
    const int g01 = hi ? 1 : 0;
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f c01 = {0.0f, 0.0f, 0.0f, 0.0f}, c2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
        const int p = 4 * kb + kq;
        const float uu = L.u[p * kDict + col];
        const float vv = L.v[p * kDict + col];
        c01 = __builtin_amdgcn_mfma_f32_16x16x4f32(uu, vv * L.g[3 * p + g01], c01, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(uu, vv * L.g[3 * p + 2], c2, 0, 0, 0);
    }

    // D[i][j] in lane j + 16 (i / 4), register i % 4; rows 0..7 are in lanes 0..31
    if (kq < 2) {
        const int j = lane & 15, y = j & 7;
        const int db = L.dict[kDict + y];
        const uint64_t col_off = (uint64_t)db;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = 4 * kq + r;
            const int da = L.dict[x];
            bool pair = x < na && y < nb;
            if (KMAX > 1 && P.degenerate && da == db) pair = false;
            float* t = P.d_lf + 3 * ((uint64_t)da * (uint64_t)P.N + col_off);
            if (pair && c01[r] != 0.0f) atomicAdd(t + (j < kDict ? 0 : 1), c01[r]);
            if (pair && j < kDict && c2[r] != 0.0f) atomicAdd(t + 2, c2[r]);
        }
    }
    wave_lds_sync();  // the rows and dictionaries are rewritten by the next call
    return true;
}

// Adjoint of one pixel: d_lf[a][b] += w_ab * dimg for its K x K pairs.
// L2: the pixel's view value is formed first, exactly as the forward lookup
// forms it, and written to img; dimg = value - target (the gradient of
// 1/2 |img - target|^2).  Otherwise dimg is read from img.
template <int KMAX, int DT, bool L2>
__device__ __forceinline__ void lookup_adjoint_pixel(const LookupParams& P, ScatterLds& L, int px, int py, int v) {
    bool live = px < P.W && py < P.H;
    int ia[KMAX], jb[KMAX];
    float wa[KMAX], wb[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        ia[a] = jb[a] = -1;
        wa[a] = wb[a] = 0.0f;
    }
    f3 gi = mk3(0.0f, 0.0f, 0.0f);
    float inv = 0.0f;
    if (live) {
        const ViewGeom& G = P.v[v];
        const uint64_t pix = ((uint64_t)(P.view0 + v) * P.H + py) * P.W + px;
        f3 qo, qd;
        if (view_hits(P, G, px, py, qo, qd)) {
            float da[KMAX], db[KMAX];
            // (one search after the other: the scatter's registers leave no room
            // for both searches' candidate sets at once)
            {
                const int ko = sf_zone(P.M, qo.z);
                sf_knn<KMAX>(P.M, P.invM, SfTable{P.tab_o}, qo, P.zone_o[ko], P.K, ia, da);
            }
            {
                const int kd = sf_zone(P.N, qd.z);
                sf_knn<KMAX>(P.N, P.invN, SfTable{P.tab_d}, qd, P.zone_d[kd], P.K, jb, db);
            }
            if constexpr (!L2) {
                const float* g = P.img + 3 * pix;
                gi = mk3(g[0], g[1], g[2]);
            }
            if constexpr (KMAX == 1) {
                wa[0] = ia[0] < P.orows ? 1.0f : 0.0f;
                wb[0] = 1.0f;
                inv = 1.0f;
                if constexpr (L2) {
                    const bool covered = ia[0] < P.orows;
                    const uint64_t t = (uint64_t)(covered ? ia[0] : 0) * (uint64_t)P.N + (uint64_t)jb[0];
                    gi = covered ? load_texel<DT>(P.lf, t) : mk3(0.0f, 0.0f, 0.0f);
                }
            } else {
#pragma unroll
                for (int a = 0; a < KMAX; ++a) {
                    wa[a] = (ia[a] >= 0 && ia[a] < P.orows) ? tent_weight_hw(da[a], P.inv_rM) : 0.0f;
                    wb[a] = jb[a] >= 0 ? tent_weight_hw(db[a], P.inv_rN) : 0.0f;
                }
                // the forward's weight sum and blend, term for term in the
                // same order (separable on a field within 4 GiB when the wave
                // has no degenerate pair)
                const bool sep = field_within_4gib(P) && separable_wave<KMAX>(P, qo, qd, da, db);
                const float wsum = sep ? separable_weight_sum<KMAX>(wa, wb) : pair_weight_sum<KMAX>(P, ia, wa, jb, wb);
                inv = wsum > 0.0f ? inv_weight_sum(wsum) : 0.0f;
                if constexpr (L2) {
                    f3 acc = mk3(0.0f, 0.0f, 0.0f);
                    if (wsum > 0.0f) {
                        if (sep) {
                            // (blend_row's arithmetic, a texel loaded per step:
                            // fewer live registers in this kernel)
#pragma unroll
                            for (int a = 0; a < KMAX; ++a) {
                                const int ai = (ia[a] >= 0 && ia[a] < P.orows) ? ia[a] : 0;
                                f3 r = mk3(0.0f, 0.0f, 0.0f);
#pragma unroll
                                for (int c = 0; c < KMAX; ++c)
                                    r = fma3(load_texel<DT>(P.lf, (uint64_t)ai * (uint64_t)P.N + (uint64_t)max(jb[c], 0)),
                                             wb[c], r);
                                acc = fma3(r, wa[a], acc);
                            }
                            acc = acc * inv;
                        } else {
#pragma unroll
                            for (int a = 0; a < KMAX; ++a)
#pragma unroll
                                for (int c = 0; c < KMAX; ++c) {
                                    const bool bad = P.degenerate && ia[a] == jb[c];
                                    const float w = bad ? 0.0f : wa[a] * wb[c] * inv;
                                    const int ai = (ia[a] >= 0 && ia[a] < P.orows) ? ia[a] : 0;
                                    const uint64_t t = (uint64_t)ai * (uint64_t)P.N + (uint64_t)max(jb[c], 0);
                                    acc = fma3(load_texel<DT>(P.lf, t), w, acc);
                                }
                        }
                    }
                    gi = acc;
                }
                sort_by_index<KMAX>(ia, wa);
                sort_by_index<KMAX>(jb, wb);
            }
            if constexpr (L2) {
                float* o = P.img + 3 * pix;
                o[0] = gi.x;
                o[1] = gi.y;
                o[2] = gi.z;
                const float* tg = P.target + 3 * pix;
                gi = gi - mk3(tg[0], tg[1], tg[2]);
            }
        } else {
            live = false;
            if constexpr (L2) {
                float* o = P.img + 3 * pix;
                o[0] = o[1] = o[2] = 0.0f;
            }
        }
    }
    // K = 9 lists alone fill a dictionary: only the per-pair path below
    if constexpr (KMAX < kDict) {
        if (mfma_scatter<KMAX>(P, L, live, ia, wa, jb, wb, inv, gi)) return;
        // The wave's texels overflow a dictionary: each half of its tile (8 x 4
        // pixels, with fewer distinct neighbours) on its own; only a half
        // that still overflows (or a non-finite adjoint) takes the per-pair
        // path.
        const bool low = (threadIdx.x & 63) < 32;
        if (mfma_scatter<KMAX>(P, L, live && low, ia, wa, jb, wb, inv, gi)) live = live && !low;
        if (mfma_scatter<KMAX>(P, L, live && !low, ia, wa, jb, wb, inv, gi)) live = live && low;
        if (__ballot(live) == 0) return;
    }
#pragma unroll
    for (int a = 0; a < KMAX; ++a)
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            // nearest sampling (K = 1) copies the texel even when i == j
            const bool bad = KMAX > 1 && P.degenerate && ia[a] == jb[c];
            const float w = bad ? 0.0f : wa[a] * wb[c] * inv;
            const bool pend = live && w != 0.0f && ia[a] >= 0 && ia[a] < P.orows && jb[c] >= 0;
            const uint64_t key = (uint64_t)max(ia[a], 0) * (uint64_t)P.N + (uint64_t)max(jb[c], 0);
            wave_scatter_add(P.d_lf, pend, key, gi * w);
        }
}

// Adjoint (and the fused L2 variant): every lane of the wave takes part in
// the aggregated scatter (no early exit).  K <= 5: 8 waves per SIMD (64
// VGPRs, a few values spilled) ran 3 % faster than 7 waves with no spills;
// K = 9 (per-pair scatter of 81 pairs) is held to 3, where it has no spills.
template <int KMAX, int DT, bool L2>
__global__ __launch_bounds__(256, KMAX <= 5 ? 8 : 3) void lookup_adjoint_kernel(LookupParams P) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ ScatterLds lds[4];
    const int px = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int py = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    lookup_adjoint_pixel<KMAX, DT, L2>(P, lds[wave], px, py, blockIdx.z);
}

// Bound by VALU issue (the searches, the selection and the blend) and the
// gathers' latency while the field stays in the caches; on a field of many
// GB the gathers' misses to HBM take their share too.  K <= 5 is held to 7
// waves per SIMD on fields within 4 GiB (72 VGPRs) and 6 on larger ones
// (80: the per-pair blend holds more texels), K = 9 to 3.
// OFF32: the field spans at most 4 GiB (field_within_4gib), so a texel is
// addressed by a 32-bit byte offset from the field's (uniform) base, one add
// per texel; there the neighbours blend separably in a wave without
// degenerate pairs, by pairs otherwise.  Larger fields blend by pairs (on a
// field of many GB, whose gathers miss to HBM, the compiler's own load
// order beats the row-ahead loads).
template <int KMAX, int DT, bool OFF32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KMAX <= 5 ? (OFF32 ? 7 : 6) : 3))) void lookup_kernel(
    LookupParams P) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int py = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int v = blockIdx.z;
    // zone bases of both sets, in LDS
    __shared__ SfZone zb[2 * kZones];
    if (threadIdx.x < 2 * kZones) zb[threadIdx.x] = threadIdx.x < kZones ? P.zone_o[threadIdx.x] : P.zone_d[threadIdx.x - kZones];
    __syncthreads();
    if (px >= P.W || py >= P.H) return;
    const ViewGeom& G = P.v[v];
    const uint64_t pix = ((uint64_t)(P.view0 + v) * P.H + py) * P.W + px;
    f3 qo, qd;
    if (!view_hits(P, G, px, py, qo, qd)) {
        {
            float* o = P.img + 3 * pix;
            o[0] = o[1] = o[2] = 0.0f;
        }
        if (P.nn) {
            P.nn[2 * pix] = -1;
            P.nn[2 * pix + 1] = -1;
        }
        return;
    }

    int ia[KMAX], jb[KMAX];
    float da[KMAX], db[KMAX];
    {
        const int ko = sf_zone(P.M, qo.z), kd = sf_zone(P.N, qd.z);
        sf_knn_pair<KMAX>(P.K, P.M, P.invM, SfTable{P.tab_o}, qo, zb[ko], ia, da, P.N, P.invN, SfTable{P.tab_d}, qd,
                          zb[kZones + kd], jb, db);
    }
    if (P.nn) {
        P.nn[2 * pix] = ia[0];
        P.nn[2 * pix + 1] = jb[0];
    }

    if constexpr (KMAX == 1) {
        const bool covered = ia[0] < P.orows;
        const uint64_t t = (uint64_t)(covered ? ia[0] : 0) * (uint64_t)P.N + (uint64_t)jb[0];
        {
            const f3 c = covered ? load_texel<DT>(P.lf, t) : mk3(0.0f, 0.0f, 0.0f);
            float* o = P.img + 3 * pix;
            o[0] = c.x;
            o[1] = c.y;
            o[2] = c.z;
        }
        return;
    }

    float wa[KMAX], wb[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        wa[a] = (ia[a] >= 0 && ia[a] < P.orows) ? tent_weight_hw(da[a], P.inv_rM) : 0.0f;
        wb[a] = jb[a] >= 0 ? tent_weight_hw(db[a], P.inv_rN) : 0.0f;
    }
    f3 acc = mk3(0.0f, 0.0f, 0.0f);
    // per-pair form: every pair tested, the compiler's own load order
    auto blend_pairs = [&]() {
        const float wsum = pair_weight_sum<KMAX>(P, ia, wa, jb, wb);
        if (wsum > 0.0f) {
            const float inv = inv_weight_sum(wsum);
#pragma unroll
            for (int a = 0; a < KMAX; ++a)
#pragma unroll
                for (int c = 0; c < KMAX; ++c) {
                    const bool bad = P.degenerate && ia[a] == jb[c];
                    const float w = bad ? 0.0f : wa[a] * wb[c] * inv;
                    const int ai = (ia[a] >= 0 && ia[a] < P.orows) ? ia[a] : 0;
                    const uint64_t t = (uint64_t)ai * (uint64_t)P.N + (uint64_t)max(jb[c], 0);
                    acc = fma3(load_texel<DT>(P.lf, t), w, acc);
                }
        }
    };
    if constexpr (OFF32) {
        if (separable_wave<KMAX>(P, qo, qd, da, db)) {  // wave-uniform
            const float wsum = separable_weight_sum<KMAX>(wa, wb);
            if (wsum > 0.0f) {
                const float inv = inv_weight_sum(wsum);
                // Uncovered or missing neighbours read texel 0 (weight 0), so
                // every gather is in range.  A texel is a 32-bit byte offset
                // from the field's base, origin row a at ai * row_bytes plus
                // direction column c at co[c] (24-bit multiplies: indices
                // below 2^16, rows below 2^24 bytes, products below 2^32).
                constexpr uint32_t TB = texel_bytes<DT>();
                const char* const lf = (const char*)P.lf;
                const uint32_t row_bytes = (uint32_t)P.N * TB;
                uint32_t co[KMAX];
#pragma unroll
                for (int c = 0; c < KMAX; ++c) co[c] = __umul24((uint32_t)max(jb[c], 0), TB);
                auto load_row = [&](int a, f3* row) {
                    const int ai = (ia[a] >= 0 && ia[a] < P.orows) ? ia[a] : 0;
                    const uint32_t ro = __umul24((uint32_t)ai, row_bytes);
#pragma unroll
                    for (int c = 0; c < KMAX; ++c) row[c] = load_texel_at<DT>(lf + (ro + co[c]));
                };
                // origin rows in turn, the next row's loads in flight while a
                // row is blended (two rows of texels held)
                f3 row[2][KMAX];
                load_row(0, row[0]);
#pragma unroll
                for (int a = 0; a < KMAX; ++a) {
                    if (a + 1 < KMAX) load_row(a + 1, row[(a + 1) & 1]);
                    __builtin_amdgcn_sched_barrier(0);
                    acc = blend_row<KMAX>(row[a & 1], wb, wa[a], acc);
                    __builtin_amdgcn_sched_barrier(0);
                }
                acc = acc * inv;
            }
        } else {
            blend_pairs();
        }
    } else {
        blend_pairs();
    }
    float* o = P.img + 3 * pix;
    o[0] = acc.x;
    o[1] = acc.y;
    o[2] = acc.z;
}

template <int KMAX, int DT>
static hipError_t launch_lookup_mode(const LookupParams& P, int mode, hipStream_t s) {
    dim3 grid((P.W + 15) / 16, (P.H + 15) / 16, P.nviews);
    if (mode == 0 && field_within_4gib(P)) lookup_kernel<KMAX, DT, true><<<grid, 256, 0, s>>>(P);
    else if (mode == 0) lookup_kernel<KMAX, DT, false><<<grid, 256, 0, s>>>(P);
    else if (mode == 1) lookup_adjoint_kernel<KMAX, 0, false><<<grid, 256, 0, s>>>(P);
    else lookup_adjoint_kernel<KMAX, DT, true><<<grid, 256, 0, s>>>(P);
    return hipGetLastError();
}

template <int KMAX>
static hipError_t launch_lookup_dt(const LookupParams& P, int mode, hipStream_t s) {
    if (mode == 1) return launch_lookup_mode<KMAX, 0>(P, mode, s);  // the plain adjoint reads no texels
    switch (P.dtype) {
        case 0: return launch_lookup_mode<KMAX, 0>(P, mode, s);
        case 1: return launch_lookup_mode<KMAX, 1>(P, mode, s);
        default: return launch_lookup_mode<KMAX, 2>(P, mode, s);
    }
}

// Point table of an SF set (float4 per point, w unused) for the lookups.
__global__ void sf_table_kernel(int n, float inv_n, float4* t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const f3 p = sf_point(n, i, inv_n);
    t[i] = make_float4(p.x, p.y, p.z, 0.0f);
}

hipError_t launch_sf_table(int n, float inv_n, float4* out, hipStream_t s) {
    sf_table_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, inv_n, out);
    return hipGetLastError();
}

// Zone bases of both SF sets (sf_zone_basis for k = 0 .. kZones - 1).
__global__ void sf_zone_kernel(float inv_m, float inv_n, SfZone* zo, SfZone* zd) {
    const int k = threadIdx.x;
    if (k < kZones) zo[k] = sf_zone_basis(k, inv_m);
    else if (k < 2 * kZones) zd[k - kZones] = sf_zone_basis(k - kZones, inv_n);
}

hipError_t launch_sf_tables(const LookupParams& P, hipStream_t s) {
    hipError_t e = launch_sf_table(P.M, P.invM, (float4*)P.tab_o, s);
    if (e == hipSuccess) e = launch_sf_table(P.N, P.invN, (float4*)P.tab_d, s);
    if (e != hipSuccess) return e;
    sf_zone_kernel<<<1, 64, 0, s>>>(P.invM, P.invN, (SfZone*)P.zone_o, (SfZone*)P.zone_d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of the lookup entry point that allocates nothing: the point
// tables of both SF sets, 16 bytes per point, each set below 65536 points
// (2 MiB per device, held until the process ends).  Host code never passes
// `scratch` itself to a kernel (on the host it names a stand-in, not device
// memory): the address each device gives for it is looked up once per
// device, with that device current, and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float4 scratch[kLookupScratchPoints];

hipError_t lookup_scratch(int dev, void** ptr) {
    static std::mutex mu;
    static void* addr[kMaxScratchDevices] = {};
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_lookup(const LookupParams& P, int mode, hipStream_t s) {
    if (P.K == 1) return launch_lookup_dt<1>(P, mode, s);
    if (P.K <= 5) return launch_lookup_dt<5>(P, mode, s);
    return launch_lookup_dt<9>(P, mode, s);
}

// ---------------------------------------------------------------------------
// lf_points: the point set and the inverse query
// ---------------------------------------------------------------------------
__global__ void points_kernel(int n, float inv_n, float* xyz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const f3 p = sf_point(n, i, inv_n);
    xyz[3 * i] = p.x;
    xyz[3 * i + 1] = p.y;
    xyz[3 * i + 2] = p.z;
}

template <int KMAX>
__global__ void query_kernel(int n, float inv_n, float inv_r, const float* query, long long nq, int K, int* idx,
                             float* w) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const f3 v = normalize(mk3(query[3 * q], query[3 * q + 1], query[3 * q + 2]));
    const int k = sf_zone(n, v.z);
    int id[KMAX];
    float d2[KMAX];
    sf_knn<KMAX>(n, inv_n, SfEval{n, inv_n}, v, sf_zone_basis(k, inv_n), K, id, d2);
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        if (a >= K) break;
        idx[q * K + a] = id[a];
        if (w) w[q * K + a] = id[a] >= 0 ? tent_weight(d2[a], inv_r) : 0.0f;
    }
}

hipError_t launch_points(int n, float* xyz, const float* query, long long nq, int K, int* idx, float* w,
                         hipStream_t s) {
    const float inv_n = 1.0f / (float)n;
    if (xyz) points_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, inv_n, xyz);
    if (query && nq > 0) {
        const float inv_r = 1.0f / sqrtf(4.0f * kPi * inv_n);
        const unsigned blocks = (unsigned)((nq + 255) / 256);
        if (K == 1) query_kernel<1><<<blocks, 256, 0, s>>>(n, inv_n, inv_r, query, nq, K, idx, w);
        else if (K <= 5) query_kernel<5><<<blocks, 256, 0, s>>>(n, inv_n, inv_r, query, nq, K, idx, w);
        else query_kernel<9><<<blocks, 256, 0, s>>>(n, inv_n, inv_r, query, nq, K, idx, w);
    }
    return hipGetLastError();
}

}  // namespace lp
