// sf_device.hpp -- device building blocks shared by the light-field kernels:
// small vector algebra, Philox4x32-10, the spherical-Fibonacci point set and
// its O(1) inverse (nearest point and at most nine neighbours).
//
// Spherical Fibonacci set (Fink et al. 2019, Sec. 2, SF point equation):
//   p_i = (cos phi_i sin theta_i, sin phi_i sin theta_i, z_i),
//   phi_i = 2 pi frac(i (Phi - 1)), z_i = 1 - (2i + 1) / n.
// frac(i (Phi - 1)) is the one step computed in FP64: in FP32 its error grows
// with i and reaches half the point spacing near n = 32768.
//
// Inverse mapping (Keinert et al. 2015, used in Sec. 2): in the (phi, z)
// plane the points form a lattice spanned by the index steps F(k), F(k+1)
// (consecutive Fibonacci numbers) of the zone k around the query height.
// Solving for the lattice cell that holds the query and testing its four
// corners gives the nearest point; a short descent over the eight lattice
// neighbours then absorbs FP32 slips at cell boundaries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

constexpr float kPi = 3.14159265358979323846f;
constexpr double kPiD = 3.14159265358979323846;
constexpr double kPhiM1 = 0.61803398874989484820;       // Phi - 1 = 1 / Phi
constexpr float kInvLogPhi2 = 1.0390834931f;             // 1 / ln(Phi^2)
constexpr float kPiSqrt5 = 7.0248147310f;                // pi * sqrt(5)

struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 operator*(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 normalize(f3 a) { return a * (1.0f / sqrtf(dot(a, a))); }

// Correctly rounded square root of x = +0 or finite x >= 2^-96: the hardware
// square root (within 1 ulp), then its lower or upper neighbour by the sign
// of the fma residual.  For such x this is the value sqrtf gives (sqrtf also
// rescales inputs below 2^-96 and passes special values through, which costs
// another seven instructions).
__device__ __forceinline__ float sqrt_big(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float lo = __uint_as_float(__float_as_uint(s) - 1u), hi = __uint_as_float(__float_as_uint(s) + 1u);
    float r = fmaf(-lo, s, x) <= 0.0f ? lo : s;
    r = fmaf(-hi, s, x) > 0.0f ? hi : r;
    return r;
}
// normalize() of a vector whose squared length is at least 2^-96.
__device__ __forceinline__ f3 normalize_big(f3 a) { return a * (1.0f / sqrt_big(dot(a, a))); }
__device__ __forceinline__ f3 fma3(f3 a, float s, f3 b) {  // a * s + b
    return {fmaf(a.x, s, b.x), fmaf(a.y, s, b.y), fmaf(a.z, s, b.z)};
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The 32x32->64 products
// map to v_mad_u64_u32.
// ---------------------------------------------------------------------------
struct u4 {
    uint32_t x, y, z, w;
};
__device__ __forceinline__ u4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi_a = (uint32_t)(a >> 32), lo_a = (uint32_t)a;
        const uint32_t hi_b = (uint32_t)(b >> 32), lo_b = (uint32_t)b;
        c0 = hi_b ^ c1 ^ k0;
        c2 = hi_a ^ c3 ^ k1;
        c1 = lo_b;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}
// 24-bit uniform in [0, 1), exact in binary32.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-08f; }

// ---------------------------------------------------------------------------
// Spherical-Fibonacci points
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sf_frac(int i) {
    double f = (double)i * kPhiM1;
    return (float)(f - floor(f));
}
__device__ __forceinline__ f3 sf_point(int n, int i, float inv_n) {
    float s, c;
    sincospif(2.0f * sf_frac(i), &s, &c);
    const uint32_t a = 2u * (uint32_t)i + 1u;
    const uint32_t b = 2u * (uint32_t)n - a;
    const float st = sqrtf((float)((uint64_t)a * b)) * inv_n;
    const float z = (float)(n - 2 * i - 1) * inv_n;
    return {c * st, s * st, z};
}

// Point sources for the inverse mapping: evaluated on the fly, or read from
// a table the same function filled (identical values, so identical
// decisions).
struct SfEval {
    int n;
    float inv_n;
    __device__ __forceinline__ f3 operator()(int i) const { return sf_point(n, i, inv_n); }
};
struct SfTable {
    const float4* t;
    __device__ __forceinline__ f3 operator()(int i) const {
        const float4 v = t[i];
        return {v.x, v.y, v.z};
    }
};

__device__ __forceinline__ int fib(int k) {
    // F(0..24); k stays below 20 for n <= 65535
    constexpr int t[25] = {0,   1,   1,   2,    3,    5,    8,    13,   21,   34,    55,    89,   144,
                           233, 377, 610, 987, 1597, 2584, 4181, 6765, 10946, 17711, 28657, 46368};
    return t[k];
}

// Zone number k = max(2, floor(log_{Phi^2}(n pi sqrt5 (1 - z^2)))).
__device__ __forceinline__ int sf_zone(int n, float qz) {
    const float arg = (float)n * kPiSqrt5 * ((1.0f - qz) * (1.0f + qz));
    if (!(arg > 0.0f)) return 2;
    const int k = (int)floorf(logf(arg) * kInvLogPhi2);
    return k < 2 ? 2 : (k > 20 ? 20 : k);
}

// Signed azimuth step of the index step F: 2 pi (F (Phi-1) - round(F (Phi-1))).
__device__ __forceinline__ float sf_dphi(int F) {
    double x = (double)F * kPhiM1;
    return (float)(2.0 * kPiD * (x - rint(x)));
}

__device__ __forceinline__ float dist2(f3 q, f3 p) {
    const f3 d = q - p;
    return dot(d, d);
}
__device__ __forceinline__ bool closer(float da, int ia, float db, int ib) {
    return da < db || (da == db && ia < ib);
}

// Lattice basis of zone k of an SF set of n points in (azimuth, height): the
// index steps F(k) and F(k+1) move by (b00, b10) and (b01, b11); inv_det is
// the inverse of the basis determinant.
struct SfZone {
    float b00, b01, b10, b11, inv_det, pad0, pad1, pad2;
};
constexpr int kZones = 21;  // k = 0 .. 20 (zones 0 and 1 are never used)
__device__ __forceinline__ SfZone sf_zone_basis(int k, float inv_n) {
    SfZone Z;
    const int F0 = fib(k), F1 = fib(k + 1);
    Z.b00 = sf_dphi(F0);
    Z.b01 = sf_dphi(F1);
    Z.b10 = -2.0f * (float)F0 * inv_n;
    Z.b11 = -2.0f * (float)F1 * inv_n;
    Z.inv_det = 1.0f / (Z.b00 * Z.b11 - Z.b01 * Z.b10);
    Z.pad0 = Z.pad1 = Z.pad2 = 0.0f;
    return Z;
}

// Nearest point by the lattice-cell corners (no descent yet), the zone's
// basis given.
template <class Pts>
__device__ __forceinline__ int sf_cell_nearest_z(int n, float inv_n, const Pts& pts, f3 q, const SfZone& Z,
                                                 float& best_d2) {
    const float b00 = Z.b00, b01 = Z.b01, b10 = Z.b10, b11 = Z.b11, inv_det = Z.inv_det;
    const float z0 = 1.0f - inv_n;
    const float v0 = atan2f(q.y, q.x), v1 = q.z - z0;
    const float c0 = floorf((b11 * v0 - b01 * v1) * inv_det);
    const float c1 = floorf((b00 * v1 - b10 * v0) * inv_det);
    int best = -1;
    float bd = 3.402823466e38f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float zc = b10 * (c0 + (float)(s & 1)) + b11 * (c1 + (float)(s >> 1)) + z0;
        zc = fminf(fmaxf(zc, -1.0f), 1.0f) * 2.0f - zc;  // mirror heights past a pole
        int i = (int)floorf(0.5f * (float)n * (1.0f - zc));
        i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
        const float d = dist2(q, pts(i));
        if (closer(d, i, bd, best)) {
            bd = d;
            best = i;
        }
    }
    best_d2 = bd;
    return best;
}

// Nearest point by the lattice-cell corners (no descent yet).
template <class Pts>
__device__ __forceinline__ int sf_cell_nearest(int n, float inv_n, const Pts& pts, f3 q, int k, float& best_d2) {
    return sf_cell_nearest_z(n, inv_n, pts, q, sf_zone_basis(k, inv_n), best_d2);
}

// Candidate set of a centre index: c + {0, +-F(k-1), +-F(k), +-F(k+1),
// +-F(k+2)} inside [0, n), duplicates (zone 2: F(1) = F(2)) replaced by
// invalid entries (d2 = +inf, distinct large keys).
struct Cand9 {
    int idx[9];
    float d2[9];
};
template <class Pts>
__device__ __forceinline__ void sf_candidates(int n, const Pts& pts, f3 q, int k, int c, Cand9& C) {
    const int f1 = fib(k - 1), f2 = fib(k), f3v = fib(k + 1), f4 = fib(k + 2);
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
        C.idx[t] = ok ? ci : 0x7fffff00 + t;
        C.d2[t] = ok ? dist2(q, pts(ci)) : 3.402823466e38f;
    }
}

// Nearest point: lattice corners, then descent over the candidate set until
// the centre is the closest candidate.  Leaves that final set in C.  Z: the
// basis of zone k (sf_zone_basis).
template <class Pts>
__device__ __forceinline__ int sf_nearest(int n, float inv_n, const Pts& pts, f3 q, int k, const SfZone& Z, Cand9& C) {
    float bd;
    int c = sf_cell_nearest_z(n, inv_n, pts, q, Z, bd);
    for (int it = 0; it < 16; ++it) {
        sf_candidates(n, pts, q, k, c, C);
        int best = C.idx[0];
        float bdd = C.d2[0];
#pragma unroll
        for (int t = 1; t < 9; ++t)
            if (closer(C.d2[t], C.idx[t], bdd, best)) {
                bdd = C.d2[t];
                best = C.idx[t];
            }
        if (best == c) break;
        c = best;
    }
    return c;
}

template <class Pts>
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

// sf_nearest for two independent queries (the front and the back hit of a
// view ray), each with its zone's basis (sf_zone_basis): the lattice corners of both, then the first candidate sets of
// both, in straight-line code, so that the point-table loads of the two
// searches are in flight together; the rare further descent steps follow
// per query.  Each query takes the same steps as in sf_nearest (the same
// centres and candidate sets, and the same cap of 16 sets), so C1 and C2
// are the sets sf_nearest leaves; conv1 / conv2 tell whether each set is
// centred on its own nearest candidate (always, unless the cap was reached).
template <class Pts>
__device__ __forceinline__ void sf_nearest_pair(int n1, float inv1, const Pts& p1, f3 q1, int k1, const SfZone& Z1,
                                                Cand9& C1, int n2, float inv2, const Pts& p2, f3 q2, int k2,
                                                const SfZone& Z2, Cand9& C2, bool& conv1, bool& conv2) {
    float bd1, bd2;
    int c1 = sf_cell_nearest_z(n1, inv1, p1, q1, Z1, bd1);
    int c2 = sf_cell_nearest_z(n2, inv2, p2, q2, Z2, bd2);
    sf_candidates(n1, p1, q1, k1, c1, C1);
    sf_candidates(n2, p2, q2, k2, c2, C2);
    int b1 = cand_best<Pts>(C1), b2 = cand_best<Pts>(C2);
    conv1 = conv2 = true;  // the final set is centred on its own nearest candidate
    for (int it = 1; b1 != c1; ++it) {
        c1 = b1;
        if (it == 16) {
            conv1 = false;
            break;
        }
        sf_candidates(n1, p1, q1, k1, c1, C1);
        b1 = cand_best<Pts>(C1);
    }
    for (int it = 1; b2 != c2; ++it) {
        c2 = b2;
        if (it == 16) {
            conv2 = false;
            break;
        }
        sf_candidates(n2, p2, q2, k2, c2, C2);
        b2 = cand_best<Pts>(C2);
    }
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

// Keep the K nearest candidates in (distance^2, index) order.  A squared
// distance is a non-negative float, so its bits order like the value: each
// candidate becomes one 64-bit key (d2 bits, index), and keys compare in
// (distance, index) order with one unsigned comparison.  Up to five kept:
// the selection network above (23 compare-exchanges); nine: nine rounds of
// odd-even transposition (36).  Registers only.
// centre_min: candidate 0 is known to be the smallest key (the descent
// converged on it); then only the other eight are ordered.
template <int KMAX>
__device__ __forceinline__ int select_k(const Cand9& C, int K, int* out_idx, float* out_d2, bool centre_min = false) {
    uint64_t key[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) key[a] = ((uint64_t)__float_as_uint(C.d2[a]) << 32) | (uint32_t)C.idx[a];
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

// Tent filter of radius sqrt(4 pi / n) on the unit chord (Sec. 2 filter
// kernel of size R sqrt(4 pi / N), with R scaled out).
__device__ __forceinline__ float tent_weight(float d2, float inv_r) {
    return fmaxf(0.0f, 1.0f - sqrtf(d2) * inv_r);
}
// The same weight with the short square root: a d2 below 2^-96 gives weight 1
// with either square root (sqrt(d2) * inv_r < 2^-41 for n <= 65535).
__device__ __forceinline__ float tent_weight_big(float d2, float inv_r) {
    return fmaxf(0.0f, 1.0f - sqrt_big(d2) * inv_r);
}

}  // namespace lp
