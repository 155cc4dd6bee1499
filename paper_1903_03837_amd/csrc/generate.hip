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
// A workgroup covers 16 consecutive bricks along x: it stages the 16 rows
// (y, z) x 49 voxels they span in LDS with reads along x, then each lane
// writes one brick row (4 voxels along x) with one vector store, so both the
// reads and the 2 KB of bricks are contiguous (no integer division in the
// stores: the grid is the brick grid).
template <typename T>
struct alignas(4 * sizeof(T)) BrickRow {
    T e[4];
};

constexpr int kHaloSpan = 3 * 16 + 1;  // voxels along x under 16 bricks

template <typename T>
__global__ __launch_bounds__(256) void halo_brick_kernel(const T* src, int layout, int nx, int ny, int nz, int nbx,
                                                         int nby, T* dst) {
    __shared__ T tile[16][kHaloSpan + 3];
    const int bx0 = blockIdx.x * 16;
    const int by = blockIdx.y, bz = blockIdx.z;
    for (int t = (int)threadIdx.x; t < 16 * kHaloSpan; t += 256) {
        const int row = t / kHaloSpan, xo = t - row * kHaloSpan;  // constant divisor
        const int x = min(bx0 * 3 + xo, nx - 1);
        const int y = min(by * 3 + (row & 3), ny - 1), z = min(bz * 3 + (row >> 2), nz - 1);
        long long si;
        if (layout == 8) {
            const long long b8 = (x >> 3) + (long long)(nx >> 3) * ((y >> 3) + (long long)(ny >> 3) * (z >> 3));
            si = b8 * 512 + (x & 7) + 8 * ((y & 7) + 8 * (z & 7));
        } else {
            si = x + (long long)nx * (y + (long long)ny * z);
        }
        tile[row][xo] = src[si];
    }
    __syncthreads();
    const int b = (int)(threadIdx.x >> 4), row = threadIdx.x & 15;  // brick row dy + 4 dz
    const int bx = bx0 + b;
    if (bx >= nbx) return;
    BrickRow<T> r;
#pragma unroll
    for (int dx = 0; dx < 4; ++dx) r.e[dx] = tile[row][3 * b + dx];
    *(BrickRow<T>*)(dst + (((long long)bz * nby + by) * nbx + bx) * 64 + 4 * row) = r;
}

hipError_t launch_halo_bricks(const void* src, int vtype, int layout, int nx, int ny, int nz, void* dst,
                              hipStream_t s) {
    const int nbx = halo_bricks(nx), nby = halo_bricks(ny), nbz = halo_bricks(nz);
    const dim3 grid((unsigned)((nbx + 15) / 16), (unsigned)nby, (unsigned)nbz);
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
    // waves take z-slices of the block, lanes run along x and each lane
    // walks y, 16 rows per trip so that 16 loads are in flight (a row's
    // address is the previous one plus a stride: no division per row)
    constexpr int kRows = 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int zi = wave; zi < cnt[2]; zi += 16) {
        const int z = lo[2] + zi;
        for (int dx = lane; dx < cnt[0]; dx += 64) {
            const int x = lo[0] + dx;
            for (int y0 = 0; y0 < cnt[1]; y0 += kRows) {
                float v[kRows];
#pragma unroll
                for (int u = 0; u < kRows; ++u) {
                    const int y = lo[1] + min(y0 + u, cnt[1] - 1);  // a repeated row changes no extreme
                    long long at;
                    if (layout == 8)
                        at = ((x >> 3) + (long long)(nx >> 3) * ((y >> 3) + (long long)(ny >> 3) * (z >> 3))) * 512 +
                             (x & 7) + 8 * ((y & 7) + 8 * (z & 7));
                    else
                        at = x + (long long)nx * (y + (long long)ny * z);
                    v[u] = (float)vol[at];
                }
#pragma unroll
                for (int u = 0; u < kRows; ++u) {
                    vlo = fminf(vlo, v[u]);
                    vhi = fmaxf(vhi, v[u]);
                }
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
    const float clo = rlo[0], chi = rhi[0];
    if (range && threadIdx.x == 0) {  // raw range of the cell's block (isosurface variant)
        range[2 * cell] = clo;
        range[2 * cell + 1] = chi;
    }
    if (!out) return;
    // window position of the range ends in double, as the definition states
    const double last = (double)(lut_n - 1);
    const double slo = fmin(fmax(((double)clo - vmin) / (vmax - vmin), 0.0), 1.0);
    const double shi = fmin(fmax(((double)chi - vmin) / (vmax - vmin), 0.0), 1.0);
    const int e0 = min((int)floor(slo * last), lut_n - 2);
    const int e1 = min((int)floor(shi * last), lut_n - 2) + 1;
    // alpha maxima over the bracketed entries and over all entries, read by
    // the whole workgroup (one thread walking the LUT waited on every load)
    float amax = 0.0f, aall = 0.0f;
    for (int e = (int)threadIdx.x; e < lut_n; e += 1024) {
        const float a = lut[4 * e + 3];
        aall = fmaxf(aall, a);
        if (e >= e0 && e <= e1) amax = fmaxf(amax, a);
    }
    __syncthreads();  // rlo[0] / rhi[0] are read; the arrays are reused
    rlo[threadIdx.x] = amax;
    rhi[threadIdx.x] = aall;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rlo[threadIdx.x] = fmaxf(rlo[threadIdx.x], rlo[threadIdx.x + w]);
            rhi[threadIdx.x] = fmaxf(rhi[threadIdx.x], rhi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double m = 1.25 * (double)scale * (double)rlo[0];
    const double fl = 1.25 * (double)scale * (double)rhi[0] / 256.0;
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
