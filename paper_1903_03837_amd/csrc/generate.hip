// generate.hip -- small set-up kernels of light-field generation: zero fill,
// the halo-brick copy of the volume, and the cell majorants of the
// majorant grid.
#include <hip/hip_fp16.h>

#include "internal.hpp"

namespace lp {

__global__ void zero_kernel(float* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

hipError_t launch_zero(float* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// Halo-brick copy of the input volume (x-fastest, or 8^3 bricks): brick
// (bx, by, bz) holds the 4^3 voxels from (3 bx, 3 by, 3 bz), so neighbouring
// bricks share a layer and every trilinear footprint lies in one brick.
// Voxels past the last index repeat the edge (no valid footprint reads them).
// One workgroup: 4 consecutive bricks along x, one lane per voxel (no
// integer division: the grid is the brick grid).
template <typename T>
__global__ __launch_bounds__(256) void halo_brick_kernel(const T* src, int layout, int nx, int ny, int nz, int nbx,
                                                         int nby, T* dst) {
    const int bx = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (bx >= nbx) return;
    const int by = blockIdx.y, bz = blockIdx.z;
    const int w = threadIdx.x & 63;
    const int x = min(bx * 3 + (w & 3), nx - 1), y = min(by * 3 + ((w >> 2) & 3), ny - 1),
              z = min(bz * 3 + (w >> 4), nz - 1);
    long long si;
    if (layout == 8) {
        const long long b8 = (x >> 3) + (long long)(nx >> 3) * ((y >> 3) + (long long)(ny >> 3) * (z >> 3));
        si = b8 * 512 + (x & 7) + 8 * ((y & 7) + 8 * (z & 7));
    } else {
        si = x + (long long)nx * (y + (long long)ny * z);
    }
    dst[(((long long)bz * nby + by) * nbx + bx) * 64 + w] = src[si];
}

hipError_t launch_halo_bricks(const void* src, int vtype, int layout, int nx, int ny, int nz, void* dst,
                              hipStream_t s) {
    const int nbx = halo_bricks(nx), nby = halo_bricks(ny), nbz = halo_bricks(nz);
    const dim3 grid((unsigned)((nbx + 3) / 4), (unsigned)nby, (unsigned)nbz);
    if (vtype == 0)
        halo_brick_kernel<uint8_t><<<grid, 256, 0, s>>>((const uint8_t*)src, layout, nx, ny, nz, nbx, nby,
                                                         (uint8_t*)dst);
    else if (vtype == 1)
        halo_brick_kernel<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)src, layout, nx, ny, nz, nbx, nby,
                                                          (uint16_t*)dst);
    else
        halo_brick_kernel<float><<<grid, 256, 0, s>>>((const float*)src, layout, nx, ny, nz, nbx, nby, (float*)dst);
    return hipGetLastError();
}

// Majorant grid: one workgroup per cell (x fastest).  Every point of cell c
// along an axis has grid coordinate g = x * n / extent - 1/2 in
// [c n / G - 1/2, (c + 1) n / G - 1/2), so its trilinear footprint lies in
// voxels floor(c n / G - 1/2) .. floor((c + 1) n / G - 1/2) + 1; one more
// voxel on each side absorbs the FP32 rounding of the cell a point is
// assigned to.  The raw range [lo, hi] of that block bounds the
// interpolated value, and the LUT entries bracketing its window position
// bound alpha.  Majorant = max(1.25 scale max alpha, global / 256).
__device__ __forceinline__ int floor_div_i(int a, int b) {  // b > 0
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

template <typename T>
__global__ __launch_bounds__(1024) void majorant_grid_kernel(const T* vol, int layout, int nx, int ny, int nz, int G,
                                                             const float* lut, int lut_n, float scale, double vmin,
                                                             double vmax, float* out, float* range) {
    __shared__ float rlo[1024], rhi[1024];
    const int cell = blockIdx.x;
    const int c[3] = {cell % G, (cell / G) % G, cell / (G * G)};
    const int n[3] = {nx, ny, nz};
    int lo[3], cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = max(floor_div_i(2 * c[a] * n[a] - G, 2 * G) - 1, 0);
        const int hi = min(floor_div_i(2 * (c[a] + 1) * n[a] - G, 2 * G) + 2, n[a] - 1);
        cnt[a] = hi - lo[a] + 1;
    }
    float vlo = 3.402823466e38f, vhi = -3.402823466e38f;
    // one wave per (y, z) row of the block, lanes along x; eight rows per
    // trip so that eight loads are in flight
    const int rows = cnt[1] * cnt[2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r0 = wave; r0 < rows; r0 += 16 * 8) {
        for (int dx = lane; dx < cnt[0]; dx += 64) {
            const int x = lo[0] + dx;
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = min(r0 + 16 * u, rows - 1);  // a repeated row changes no extreme
                const int y = lo[1] + r % cnt[1], z = lo[2] + r / cnt[1];
                long long at;
                if (layout == 8)
                    at = ((x >> 3) + (long long)(nx >> 3) * ((y >> 3) + (long long)(ny >> 3) * (z >> 3))) * 512 +
                         (x & 7) + 8 * ((y & 7) + 8 * (z & 7));
                else
                    at = x + (long long)nx * (y + (long long)ny * z);
                v[u] = (float)vol[at];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                vlo = fminf(vlo, v[u]);
                vhi = fmaxf(vhi, v[u]);
            }
        }
    }
    rlo[threadIdx.x] = vlo;
    rhi[threadIdx.x] = vhi;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rlo[threadIdx.x] = fminf(rlo[threadIdx.x], rlo[threadIdx.x + w]);
            rhi[threadIdx.x] = fmaxf(rhi[threadIdx.x], rhi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (range) {  // raw range of the cell's block (isosurface variant)
        range[2 * cell] = rlo[0];
        range[2 * cell + 1] = rhi[0];
    }
    if (!out) return;
    // window position of the range ends in double, as the definition states
    const double last = (double)(lut_n - 1);
    const double slo = fmin(fmax(((double)rlo[0] - vmin) / (vmax - vmin), 0.0), 1.0);
    const double shi = fmin(fmax(((double)rhi[0] - vmin) / (vmax - vmin), 0.0), 1.0);
    const int e0 = min((int)floor(slo * last), lut_n - 2);
    const int e1 = min((int)floor(shi * last), lut_n - 2) + 1;
    float amax = 0.0f, aall = 0.0f;
    for (int e = 0; e < lut_n; ++e) {
        const float a = lut[4 * e + 3];
        aall = fmaxf(aall, a);
        if (e >= e0 && e <= e1) amax = fmaxf(amax, a);
    }
    const double m = 1.25 * (double)scale * (double)amax;
    const double fl = 1.25 * (double)scale * (double)aall / 256.0;
    out[cell] = (float)(m > fl ? m : fl);
}

hipError_t launch_majorant_grid(const void* vol, int vtype, int layout, int nx, int ny, int nz, int G,
                                const float* lut, int lut_n, float scale, double vmin, double vmax, float* out,
                                float* range, hipStream_t s) {
    const unsigned cells = (unsigned)(G * G * G);
    if (vtype == 0)
        majorant_grid_kernel<uint8_t><<<cells, 1024, 0, s>>>((const uint8_t*)vol, layout, nx, ny, nz, G, lut, lut_n,
                                                             scale, vmin, vmax, out, range);
    else if (vtype == 1)
        majorant_grid_kernel<uint16_t><<<cells, 1024, 0, s>>>((const uint16_t*)vol, layout, nx, ny, nz, G, lut,
                                                              lut_n, scale, vmin, vmax, out, range);
    else
        majorant_grid_kernel<float><<<cells, 1024, 0, s>>>((const float*)vol, layout, nx, ny, nz, G, lut, lut_n,
                                                           scale, vmin, vmax, out, range);
    return hipGetLastError();
}

__global__ void fill_views_kernel(ViewBatch b, ViewCam* dst) {
    if ((int)threadIdx.x < b.count) dst[b.first + threadIdx.x] = b.v[threadIdx.x];
}

hipError_t launch_fill_views(const ViewBatch& b, ViewCam* dst, hipStream_t s) {
    fill_views_kernel<<<1, kViewBatch, 0, s>>>(b, dst);
    return hipGetLastError();
}

}  // namespace lp
