// sf_device.hpp -- device building blocks shared by the light-field kernels:
// small vector algebra, Philox4x32-10 and the spherical-Fibonacci point set
// (its inverse mapping, used by the lookups only, is in sf_search.hpp).
//
// Spherical Fibonacci set (Fink et al. 2019, Sec. 2, SF point equation):
//   p_i = (cos phi_i sin theta_i, sin phi_i sin theta_i, z_i),
//   phi_i = 2 pi frac(i (Phi - 1)), z_i = 1 - (2i + 1) / n.
// frac(i (Phi - 1)) is the one step computed in FP64: in FP32 its error grows
// with i and reaches half the point spacing near n = 32768.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

constexpr float kPi = 3.14159265358979323846f;
constexpr double kPhiM1 = 0.61803398874989484820;       // Phi - 1 = 1 / Phi

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

// Lattice basis of zone k of an SF set of n points in (azimuth, height): the
// index steps F(k) and F(k+1) move by (b00, b10) and (b01, b11); inv_det is
// the inverse of the basis determinant; f_km1, f_k, f_kp1 are the Fibonacci
// numbers F(k-1), F(k), F(k+1) themselves.
struct SfZone {
    float b00, b01, b10, b11, inv_det;
    int32_t f_km1, f_k, f_kp1;
};
constexpr int kZones = 21;  // k = 0 .. 20 (zones 0 and 1 are never used)

}  // namespace lp
