// generate.hip -- small set-up kernels of light-field generation: the
// default majorant, zero fill, and the copy of the volume into 4^3 bricks.
#include <hip/hip_fp16.h>

#include "internal.hpp"

namespace lp {

__global__ void majorant_kernel(const float* lut, int n, float scale, float given, float* out) {
    __shared__ float red[256];
    float m = 0.0f;
    for (int e = threadIdx.x; e < n; e += 256) m = fmaxf(m, lut[4 * e + 3]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = given > 0.0f ? given : 1.25f * scale * red[0];
}

__global__ void zero_kernel(float* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

hipError_t launch_majorant(const float* lut, int lut_n, float scale, float given, float* out, hipStream_t s) {
    majorant_kernel<<<1, 256, 0, s>>>(lut, lut_n, scale, given, out);
    return hipGetLastError();
}

hipError_t launch_zero(float* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// Copy of the input volume (x-fastest, or 8^3 bricks) into 4^3 bricks; the
// padding beyond nx, ny, nz is never read (fetch coordinates are clamped).
template <typename T>
__global__ void brick4_kernel(const T* src, int layout, int nx, int ny, int nz, int nbx, int nby, long long total,
                              T* dst) {
    const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= total) return;
    const long long bk = d >> 6;
    const int w = (int)(d & 63);
    const int bx = (int)(bk % nbx), by = (int)((bk / nbx) % nby), bz = (int)(bk / ((long long)nbx * nby));
    const int x = bx * 4 + (w & 3), y = by * 4 + ((w >> 2) & 3), z = bz * 4 + (w >> 4);
    T v = T(0);
    if (x < nx && y < ny && z < nz) {
        long long si;
        if (layout == 8) {
            const long long b8 = (x >> 3) + (long long)(nx >> 3) * ((y >> 3) + (long long)(ny >> 3) * (z >> 3));
            si = b8 * 512 + (x & 7) + 8 * ((y & 7) + 8 * (z & 7));
        } else {
            si = x + (long long)nx * (y + (long long)ny * z);
        }
        v = src[si];
    }
    dst[d] = v;
}

hipError_t launch_brick4(const void* src, int vtype, int layout, int nx, int ny, int nz, void* dst, hipStream_t s) {
    const int nbx = (nx + 3) / 4, nby = (ny + 3) / 4, nbz = (nz + 3) / 4;
    const long long total = 64ll * nbx * nby * nbz;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (vtype == 0)
        brick4_kernel<uint8_t><<<blocks, 256, 0, s>>>((const uint8_t*)src, layout, nx, ny, nz, nbx, nby, total,
                                                       (uint8_t*)dst);
    else if (vtype == 1)
        brick4_kernel<uint16_t><<<blocks, 256, 0, s>>>((const uint16_t*)src, layout, nx, ny, nz, nbx, nby, total,
                                                        (uint16_t*)dst);
    else
        brick4_kernel<float><<<blocks, 256, 0, s>>>((const float*)src, layout, nx, ny, nz, nbx, nby, total,
                                                     (float*)dst);
    return hipGetLastError();
}

}  // namespace lp
