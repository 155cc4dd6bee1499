// sf_search.hpp -- the inverse spherical-Fibonacci mapping of the lookups:
// nearest point of a set and the K nearest of its lattice neighbours.
//
// Inverse mapping (Keinert et al. 2015, used in Sec. 2): in the (phi, z)
// plane the points form a lattice spanned by the index steps F(k), F(k+1)
// (consecutive Fibonacci numbers) of the zone k around the query height.
// Solving for the lattice cell that holds the query and testing its four
// corners gives the nearest point; a short descent over the eight lattice
// neighbours then absorbs FP32 slips at cell boundaries.
#pragma once

#include "sf_device.hpp"

namespace lp {

constexpr double kPiD = 3.14159265358979323846;
constexpr float kInvLog2Phi2 = 0.72021004520627820f;  // 1 / log2(Phi^2)
constexpr float kPiSqrt5 = 7.0248147310f;     // pi * sqrt(5)

// Point sources for the inverse mapping: evaluated on the fly, or read from
// a table the same function filled (identical values, so identical
// decisions).
struct SfEval {
    int n;
    float inv_n;
    __device__ __forceinline__ f3 operator()(uint32_t i) const { return sf_point(n, (int)i, inv_n); }
};
struct SfTable {
    const float4* t;
    __device__ __forceinline__ f3 operator()(uint32_t i) const {
        const float4 v = t[i];
        return {v.x, v.y, v.z};
    }
};

__device__ __forceinline__ int fib(int k) {
    // F(0..24); k stays below 20 for n <= 65535 (F(-1) = 1)
    constexpr int t[25] = {0,   1,   1,   2,    3,    5,    8,    13,   21,   34,    55,    89,   144,
                           233, 377, 610, 987, 1597, 2584, 4181, 6765, 10946, 17711, 28657, 46368};
    return k < 0 ? 1 : t[k];
}

// Zone number k = max(2, floor(log_{Phi^2}(n pi sqrt5 (1 - z^2)))), with
// the hardware base-2 logarithm (v_log_f32, about an ulp; arg is a normal
// number or zero): the zone only picks the lattice basis, and an ulp moves
// k only for heights within ~1e-7 of a zone boundary, where either basis
// serves: the candidate offsets F(k-1) .. F(k+2) hold both zones' steps.
__device__ __forceinline__ int sf_zone(int n, float qz) {
    const float arg = (float)n * kPiSqrt5 * ((1.0f - qz) * (1.0f + qz));
    if (!(arg > 0.0f)) return 2;
    const int k = (int)floorf(__builtin_amdgcn_logf(arg) * kInvLog2Phi2);
    return k < 2 ? 2 : (k > 20 ? 20 : k);
}

// Signed azimuth step of the index step F: 2 pi (F (Phi-1) - round(F (Phi-1))).
__device__ __forceinline__ float sf_dphi(int F) {
    double x = (double)F * kPhiM1;
    return (float)(2.0 * kPiD * (x - rint(x)));
}

// |q - p|^2 with its roundings fixed (y^2 first, then x and z by fused
// multiply-add), so that a distance reused from another step of the search
// is the one the step itself would compute.
__device__ __forceinline__ float dist2(f3 q, f3 p) {
    const f3 d = q - p;
    return fmaf(d.z, d.z, fmaf(d.x, d.x, d.y * d.y));
}
__device__ __forceinline__ bool closer(float da, int ia, float db, int ib) {
    return da < db || (da == db && ia < ib);
}

__device__ __forceinline__ SfZone sf_zone_basis(int k, float inv_n) {
    SfZone Z;
    const int F0 = fib(k), F1 = fib(k + 1);
    Z.b00 = sf_dphi(F0);
    Z.b01 = sf_dphi(F1);
    Z.b10 = -2.0f * (float)F0 * inv_n;
    Z.b11 = -2.0f * (float)F1 * inv_n;
    Z.inv_det = 1.0f / (Z.b00 * Z.b11 - Z.b01 * Z.b10);
    Z.f_km1 = fib(k - 1);
    Z.f_k = F0;
    Z.f_kp1 = F1;
    return Z;
}

// Azimuth atan2(y, x) in [-pi, pi], to 4e-7 rad (the FP32 spacing near pi
// included; a host test checks the coefficients below): reduced to
// t = min(|x|, |y|) / max(|x|, |y|) in [0, 1], then atan t = t P(t^2) with
// P of degree 7, a minimax fit of atan(t) / t on [0, 1] (relative error
// 1e-7; coefficients fitted for this file), then unfolded by octant.  About
// 20 instructions where atan2f takes 55.  The azimuth only places the query
// in a lattice cell, and the corner and candidate steps that follow find the
// same nearest point for azimuth errors far larger than this (measured:
// an azimuth moved by 1e-3 rad changed no nearest point among 8e5 random
// queries at n = 2048 and 32768).
__device__ __forceinline__ float sf_azimuth(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float s = t * t;
    float p = -0.00469326926f;
    p = fmaf(p, s, 0.0242523793f);
    p = fmaf(p, s, -0.0594863594f);
    p = fmaf(p, s, 0.0991429016f);
    p = fmaf(p, s, -0.140194803f);
    p = fmaf(p, s, 0.199697241f);
    p = fmaf(p, s, -0.333319902f);
    p = fmaf(p, s, 0.999999881f);
    float r = t * p;
    r = ay > ax ? 1.57079632679489662f - r : r;
    r = x < 0.0f ? 3.14159265358979324f - r : r;
    return copysignf(r, y);
}

// Corners of the lattice cell that holds q, corner s at cell offset
// (s & 1, s >> 1), zone k with basis Z (sf_zone_basis): returns the nearest corner's index
// and leaves which corner it is in best_s and the squared distance of each
// corner in d2.  lattice: the corner indices follow the lattice (corner s at
// index i_0 + (s & 1) F(k) + (s >> 1) F(k+1): no clamp or mirror at a pole)
// and k >= 3 (F(k-1) < F(k)), so that the other three corners are
// candidates of the nearest one (sf_candidates_at_corner).
template <class Pts>
__device__ __forceinline__ int sf_cell_corners(int n, float inv_n, const Pts& pts, f3 q, const SfZone& Z,
                                               float* d2, int& best_s, bool& lattice) {
    const float b00 = Z.b00, b01 = Z.b01, b10 = Z.b10, b11 = Z.b11, inv_det = Z.inv_det;
    const float z0 = 1.0f - inv_n;
    const float v0 = sf_azimuth(q.y, q.x), v1 = q.z - z0;
    const float c0 = floorf((b11 * v0 - b01 * v1) * inv_det);
    const float c1 = floorf((b00 * v1 - b10 * v0) * inv_det);
    int best = -1, idx[4];
    float bd = 3.402823466e38f;
    best_s = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float zc = b10 * (c0 + (float)(s & 1)) + b11 * (c1 + (float)(s >> 1)) + z0;
        zc = fminf(fmaxf(zc, -1.0f), 1.0f) * 2.0f - zc;  // mirror heights past a pole
        int i = (int)floorf(0.5f * (float)n * (1.0f - zc));
        i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
        idx[s] = i;
        const float d = dist2(q, pts(i));
        d2[s] = d;
        if (closer(d, i, bd, best)) {
            bd = d;
            best = i;
            best_s = s;
        }
    }
    const int F0 = Z.f_k, F1 = Z.f_kp1;
    lattice = Z.f_km1 != F0 && idx[1] == idx[0] + F0 && idx[2] == idx[0] + F1 && idx[3] == idx[0] + F0 + F1;
    return best;
}

// Candidate set of a centre index: c + {0, +-F(k-1), +-F(k), +-F(k+1),
// +-F(k+2)} inside [0, n), duplicates (zone 2: F(1) = F(2)) replaced by
// invalid entries (d2 = +inf, distinct large keys).
struct Cand9 {
    int idx[9];
    float d2[9];
};
template <class Pts>
__device__ __forceinline__ void sf_candidates(int n, const Pts& pts, f3 q, const SfZone& Z, int c, Cand9& C) {
    const int f1 = Z.f_km1, f2 = Z.f_k, f3v = Z.f_kp1, f4 = Z.f_k + Z.f_kp1;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        int off = 0;
        if (t > 0) {
            const int m = (t - 1) >> 1;
            const int f = m == 0 ? f1 : (m == 1 ? f2 : (m == 2 ? f3v : f4));
            off = (t & 1) ? f : -f;
        }
        const int ci = c + off;
        const bool dup = (t == 1 || t == 2) && f1 == f2;
        const bool ok = (unsigned)ci < (unsigned)n && !dup;
        // every lane loads (an index clamped into the set), so that the nine
        // loads are issued back to back without branches
        const float d = dist2(q, pts(min((uint32_t)ci, (uint32_t)(n - 1))));
        C.idx[t] = ok ? ci : 0x7fffff00 + t;
        C.d2[t] = ok ? d : 3.402823466e38f;
    }
}

// v[s] for s in 0..3, as selects on the two bits of s
template <class T>
__device__ __forceinline__ T sel4(int s, T v0, T v1, T v2, T v3) {
    return (s & 2) ? ((s & 1) ? v3 : v2) : ((s & 1) ? v1 : v0);
}

// sf_candidates for the centre c = the nearest corner best_s of a lattice
// cell whose corners follow the lattice (sf_cell_corners): the centre and
// the other three corners sit at four of the nine slots (which four depends
// on best_s), so their distances are taken from cd2 and only the other five
// points are loaded.  The same set, to the bit, as sf_candidates(c).
template <class Pts>
__device__ __forceinline__ void sf_candidates_at_corner(int n, const Pts& pts, f3 q, const SfZone& Z, int c,
                                                        int best_s, const float* cd2, Cand9& C) {
    const int f1 = Z.f_km1, f2 = Z.f_k, f3v = Z.f_kp1, f4 = Z.f_k + Z.f_kp1;
    const int off[9] = {0, f1, -f1, f2, -f2, f3v, -f3v, f4, -f4};
    // slot of corner s' seen from the nearest corner s (0: the centre)
    constexpr int kCornerSlot[4][4] = {{0, 3, 5, 7}, {4, 0, 1, 5}, {6, 2, 0, 3}, {8, 6, 4, 0}};
    // the five slots that hold no corner, per nearest corner
    constexpr int kOpenSlot[4][5] = {{1, 2, 4, 6, 8}, {2, 3, 6, 7, 8}, {1, 4, 5, 7, 8}, {1, 2, 3, 5, 7}};
    float du[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) {
        const int o = sel4(best_s, off[kOpenSlot[0][u]], off[kOpenSlot[1][u]], off[kOpenSlot[2][u]],
                           off[kOpenSlot[3][u]]);
        du[u] = dist2(q, pts(min((uint32_t)(c + o), (uint32_t)(n - 1))));
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        // the distance at slot t for each nearest corner s: a corner's, or a
        // loaded one (both fixed at compile time per (t, s))
        float ds[4];
#pragma unroll
        for (int sc = 0; sc < 4; ++sc) {
            ds[sc] = 0.0f;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
                if (kCornerSlot[sc][s2] == t) ds[sc] = cd2[s2];
#pragma unroll
            for (int u = 0; u < 5; ++u)
                if (kOpenSlot[sc][u] == t) ds[sc] = du[u];
        }
        const float d = sel4(best_s, ds[0], ds[1], ds[2], ds[3]);
        const int ci = c + off[t];
        const bool ok = (unsigned)ci < (unsigned)n;
        C.idx[t] = ok ? ci : 0x7fffff00 + t;
        C.d2[t] = ok ? d : 3.402823466e38f;
    }
}

// Index of the nearest candidate of a set.
__device__ __forceinline__ int cand_best(const Cand9& C) {
    int best = C.idx[0];
    float bdd = C.d2[0];
#pragma unroll
    for (int t = 1; t < 9; ++t)
        if (closer(C.d2[t], C.idx[t], bdd, best)) {
            bdd = C.d2[t];
            best = C.idx[t];
        }
    return best;
}

// Comparators (a, b), a < b, that leave the five smallest of nine keys in
// positions 0..4 in order: Batcher's odd-even merge sort of 16 inputs
// restricted to 9, then pruned of every comparator the first five outputs do
// not need.  By the 0-1 principle it suffices that this holds for all 512
// inputs of zeros and ones, which a host test checks.
constexpr int kSel5of9 = 23;
__device__ constexpr int kSel5of9Net[kSel5of9][2] = {
    {0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5},
    {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {0, 8}, {4, 8}, {2, 4}, {1, 2}, {3, 4}};

// Comparators (a, b) over eight keys that leave the four smallest in positions
// 0..3 in order: Batcher's odd-even merge sort of 8 inputs, pruned of every
// comparator the first four outputs do not need (18 of 19; a host test checks
// all 256 inputs of zeros and ones).  When the descent has converged, the
// centre (candidate 0) is the unique smallest key, and the five nearest are
// the centre followed by the four smallest of the other eight.
constexpr int kSel4of8 = 18;
__device__ constexpr int kSel4of8Net[kSel4of8][2] = {
    {0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}, {4, 5}, {6, 7}, {4, 6}, {5, 7},
    {5, 6}, {0, 4}, {2, 6}, {2, 4}, {1, 5}, {3, 7}, {3, 5}, {1, 2}, {3, 4}};

// One 64-bit key per candidate, (d2 bits, index): a squared distance is a
// non-negative float, so its bits order like the value, and keys compare in
// (distance, index) order with one unsigned comparison.
__device__ __forceinline__ void cand_keys(const Cand9& C, uint64_t* key) {
#pragma unroll
    for (int a = 0; a < 9; ++a) key[a] = ((uint64_t)__float_as_uint(C.d2[a]) << 32) | (uint32_t)C.idx[a];
}
// The first KMAX keys as (index, d2); positions from K on, and invalid
// candidates, give index -1.  Returns the number of valid ones.
template <int KMAX>
__device__ __forceinline__ int keys_out(const uint64_t* key, int K, int* out_idx, float* out_d2) {
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < KMAX; ++r) {
        const int id = (int)(uint32_t)key[r];
        const bool ok = r < K && id >= 0 && id < 0x7fffff00;
        out_idx[r] = ok ? id : -1;
        out_d2[r] = __uint_as_float((uint32_t)(key[r] >> 32));
        cnt += ok;
    }
    return cnt;
}

// Keep the K nearest candidates in (distance^2, index) order, on the keys
// of cand_keys.  Up to five kept: the selection network above (23
// compare-exchanges); nine: nine rounds of odd-even transposition (36).
// Registers only.
// centre_min: candidate 0 is known to be the smallest key (the descent
// converged on it); then only the other eight are ordered.
template <int KMAX>
__device__ __forceinline__ int select_k(const Cand9& C, int K, int* out_idx, float* out_d2, bool centre_min = false) {
    uint64_t key[9];
    cand_keys(C, key);
    if constexpr (KMAX == 1) {
        if (!centre_min) {
#pragma unroll
            for (int a = 1; a < 9; ++a) key[0] = key[a] < key[0] ? key[a] : key[0];
        }
    } else if constexpr (KMAX <= 5) {
        if (centre_min) {
#pragma unroll
            for (int c = 0; c < kSel4of8; ++c) {
                const int a = kSel4of8Net[c][0] + 1, b = kSel4of8Net[c][1] + 1;
                const uint64_t lo = key[a] < key[b] ? key[a] : key[b];
                const uint64_t hi = key[a] < key[b] ? key[b] : key[a];
                key[a] = lo;
                key[b] = hi;
            }
        } else {
#pragma unroll
            for (int c = 0; c < kSel5of9; ++c) {
                const int a = kSel5of9Net[c][0], b = kSel5of9Net[c][1];
                const uint64_t lo = key[a] < key[b] ? key[a] : key[b];
                const uint64_t hi = key[a] < key[b] ? key[b] : key[a];
                key[a] = lo;
                key[b] = hi;
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < 9; ++p)
#pragma unroll
            for (int a = (p & 1); a + 1 < 9; a += 2) {
                const uint64_t lo = key[a] < key[a + 1] ? key[a] : key[a + 1];
                const uint64_t hi = key[a] < key[a + 1] ? key[a + 1] : key[a];
                key[a] = lo;
                key[a + 1] = hi;
            }
    }
    return keys_out<KMAX>(key, K, out_idx, out_d2);
}

// Tent filter of radius sqrt(4 pi / n) on the unit chord (Sec. 2 filter
// kernel of size R sqrt(4 pi / N), with R scaled out).
__device__ __forceinline__ float tent_weight(float d2, float inv_r) {
    return fmaxf(0.0f, 1.0f - sqrtf(d2) * inv_r);
}

// ---------------------------------------------------------------------------
// K nearest points of a query: the lattice corners, the candidate set of the
// nearest corner, then the descent, which moves the centre to the set's
// nearest candidate until the centre is its own set's nearest (at most 16
// sets), and the selection over the last set (select_k, centre_min when the
// descent converged).  The first set is nearly always centred on its own
// nearest candidate; the selection that keeps the K nearest when it is also
// tells whether it is, at the cost of one comparison, so the common case
// runs no separate nearest-candidate scan, and only a query whose first set
// is not centred descends and selects again.
// ---------------------------------------------------------------------------

// 32-bit keys for the selection over a first set: the squared distance's
// bits with the low four replaced by the candidate's slot t (0..8).  The
// keys order like the distances rounded down to 20 significant bits, ties
// broken by slot (the centre, slot 0, first); an invalid candidate
// (d2 = FLT_MAX) keys above every valid one.  Rounding a squared distance
// down by at most 2^-19 of itself moves a tent weight by below 1e-6, and a
// decision only between candidates whose distances agree to that
// precision.  A compare-exchange is one unsigned minimum and one maximum,
// where the 64-bit (distance, index) keys of select_k take two 64-bit
// compares and four selects.
constexpr uint32_t kInvalidKey = 0x7f7ffff0u;  // FLT_MAX's bits, slot field cleared
__device__ __forceinline__ uint32_t slot_key(float d2, int t) { return (__float_as_uint(d2) & ~15u) | (uint32_t)t; }
// Index of slot t of the set centred on c (offsets 0, +-F(k-1), +-F(k),
// +-F(k+1), +-F(k+2) in slot order) as c + a F(k-1) + b F(k): F(k+1) =
// F(k-1) + F(k) and F(k+2) = F(k-1) + 2 F(k).  a and b per slot are 2- and
// 3-bit signed fields of two constants (a: 0 1 -1 0 0 1 -1 1 -1; b: 0 0 0
// 1 -1 1 -1 2 -2), extracted by a signed bit-field extract; a host test
// checks the constants against the offsets.
constexpr int kSlotA[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int kSlotB[9] = {0, 0, 0, 1, -1, 1, -1, 2, -2};
constexpr uint32_t pack_fields(const int* v, int bits) {
    uint32_t r = 0;
    for (int t = 0; t < 9; ++t) r |= ((uint32_t)v[t] & ((1u << bits) - 1u)) << (bits * t);
    return r;
}
constexpr uint32_t kSlotAF = pack_fields(kSlotA, 2), kSlotBF = pack_fields(kSlotB, 3);
__device__ __forceinline__ int slot_index(int c, uint32_t t, int f_km1, int f_k) {
    const int a = __builtin_amdgcn_sbfe((int)kSlotAF, 2 * t, 2);
    const int b = __builtin_amdgcn_sbfe((int)kSlotBF, 3 * t, 3);
    return c + __mul24(a, f_km1) + __mul24(b, f_k);
}

// Selection over a first set, centred on c, assumed centred on its nearest
// candidate.  Returns whether it is; best is the set's nearest candidate
// either way.  out_idx and out_d2 hold the K nearest (out_d2 rounded down as
// above) only when it returns true.
template <int KMAX>
__device__ __forceinline__ bool select_k_centred(const Cand9& C, const SfZone& Z, int c, int K, int* out_idx,
                                                 float* out_d2, int& best) {
    if constexpr (KMAX <= 5) {
        uint32_t key[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) key[t] = slot_key(C.d2[t], t);
        if constexpr (KMAX == 1) {
            uint32_t m = key[1];
#pragma unroll
            for (int a = 2; a < 9; ++a) m = min(m, key[a]);
            key[1] = m;
        } else {
            // the network over candidates 1..8 leaves their four smallest in
            // positions 1..4, in order
#pragma unroll
            for (int e = 0; e < kSel4of8; ++e) {
                const int a = kSel4of8Net[e][0] + 1, b = kSel4of8Net[e][1] + 1;
                const uint32_t lo = min(key[a], key[b]), hi = max(key[a], key[b]);
                key[a] = lo;
                key[b] = hi;
            }
        }
        // (the Fibonacci steps read once: decoded indices are plain
        // arithmetic, which the compiler keeps out of branches)
        const int f_km1 = Z.f_km1, f_k = Z.f_k;
        int id[KMAX];
#pragma unroll
        for (int r = 1; r < KMAX; ++r) id[r] = slot_index(c, key[r] & 15u, f_km1, f_k);
        const bool centred = key[0] < key[1];
        best = centred ? c : (KMAX > 1 ? id[1] : slot_index(c, key[1] & 15u, f_km1, f_k));
        // the centre first, then the smallest of the others
        out_idx[0] = c;  // (K >= 1 and the centre is a valid candidate)
        out_d2[0] = __uint_as_float(key[0] & ~15u);
#pragma unroll
        for (int r = 1; r < KMAX; ++r) {
            const bool ok = r < K && key[r] < kInvalidKey;
            out_idx[r] = ok ? id[r] : -1;
            out_d2[r] = __uint_as_float(key[r] & ~15u);
        }
        return centred;
    } else {
        // all nine sorted by nine rounds of odd-even transposition; the set
        // is centred when its smallest key is the centre's (slot 0)
        uint32_t key[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) key[t] = slot_key(C.d2[t], t);
#pragma unroll
        for (int p = 0; p < 9; ++p)
#pragma unroll
            for (int a = (p & 1); a + 1 < 9; a += 2) {
                const uint32_t lo = min(key[a], key[a + 1]), hi = max(key[a], key[a + 1]);
                key[a] = lo;
                key[a + 1] = hi;
            }
        const int f_km1 = Z.f_km1, f_k = Z.f_k;
        int id[KMAX];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) id[r] = slot_index(c, key[r] & 15u, f_km1, f_k);
        best = id[0];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) {
            const bool ok = r < K && key[r] < kInvalidKey;
            out_idx[r] = ok ? id[r] : -1;
            out_d2[r] = __uint_as_float(key[r] & ~15u);
        }
        return (key[0] & 15u) == 0u;
    }
}

// The descent from a first set centred on c whose nearest candidate is
// best != c, then the selection over the set it ends on.
template <int KMAX, class Pts>
__device__ __forceinline__ void sf_descend_select(int n, const Pts& pts, f3 q, const SfZone& Z, int c, int best,
                                                  int K, int* out_idx, float* out_d2) {
    Cand9 C;
    bool conv = true;  // the final set is centred on its own nearest candidate
    for (int it = 1; best != c; ++it) {  // it: sets examined so far
        c = best;
        if (it == 16) {
            conv = false;
            break;
        }
        sf_candidates(n, pts, q, Z, c, C);
        best = cand_best(C);
    }
    select_k<KMAX>(C, K, out_idx, out_d2, conv);
}

// K nearest of one query, Z the basis of its zone (sf_zone_basis).
template <int KMAX, class Pts>
__device__ __forceinline__ void sf_knn(int n, float inv_n, const Pts& pts, f3 q, const SfZone& Z, int K,
                                       int* out_idx, float* out_d2) {
    float cd[4];
    int s;
    bool lat;
    const int c = sf_cell_corners(n, inv_n, pts, q, Z, cd, s, lat);
    Cand9 C;
    if (__ballot(!lat) == 0) sf_candidates_at_corner(n, pts, q, Z, c, s, cd, C);  // wave-uniform
    else sf_candidates(n, pts, q, Z, c, C);
    int best;
    if (!select_k_centred<KMAX>(C, Z, c, K, out_idx, out_d2, best))
        sf_descend_select<KMAX>(n, pts, q, Z, c, best, K, out_idx, out_d2);
}

// sf_knn for two independent queries (the front and the back hit of a view
// ray): the corners and first candidate sets of both in straight-line code,
// so that the point-table loads of the two searches are in flight together;
// the rare descents follow per query.
template <int KMAX, class Pts>
__device__ __forceinline__ void sf_knn_pair(int K, int n1, float inv1, const Pts& p1, f3 q1, const SfZone& Z1,
                                            int* i1, float* d1, int n2, float inv2, const Pts& p2, f3 q2,
                                            const SfZone& Z2, int* i2, float* d2) {
    float cd1[4], cd2[4];
    int s1, s2;
    bool lat1, lat2;
    const int c1 = sf_cell_corners(n1, inv1, p1, q1, Z1, cd1, s1, lat1);
    const int c2 = sf_cell_corners(n2, inv2, p2, q2, Z2, cd2, s2, lat2);
    Cand9 C1, C2;
    if (__ballot(!(lat1 && lat2)) == 0) {  // wave-uniform
        sf_candidates_at_corner(n1, p1, q1, Z1, c1, s1, cd1, C1);
        sf_candidates_at_corner(n2, p2, q2, Z2, c2, s2, cd2, C2);
    } else {
        sf_candidates(n1, p1, q1, Z1, c1, C1);
        sf_candidates(n2, p2, q2, Z2, c2, C2);
    }
    // (both sets' distances before either selection: fewer live registers
    // than the loaded points of one set held across the other's selection)
    __builtin_amdgcn_sched_barrier(0);
    int b1, b2;
    const bool ok1 = select_k_centred<KMAX>(C1, Z1, c1, K, i1, d1, b1);
    const bool ok2 = select_k_centred<KMAX>(C2, Z2, c2, K, i2, d2, b2);
    if (!ok1) sf_descend_select<KMAX>(n1, p1, q1, Z1, c1, b1, K, i1, d1);
    if (!ok2) sf_descend_select<KMAX>(n2, p2, q2, Z2, c2, b2, K, i2, d2);
}

}  // namespace lp
