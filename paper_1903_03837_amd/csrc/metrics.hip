// metrics.hip -- image similarity of light-field views against ground-truth
// views: mean SSIM (Wang, Bovik, Sheikh, Simoncelli 2004, the index the
// paper reports) with the 11 x 11 Gaussian window of sigma 1.5, over the
// positions where the window lies inside the image, per colour channel, then
// averaged over the channels.
//
// One workgroup computes 16 x 16 window positions of one channel: the 26 x 26
// input tiles of both images go to LDS, a horizontal pass forms the five
// windowed moments (means, second moments, cross moment) for 26 rows, a
// vertical pass finishes them, and each thread evaluates its SSIM term.  The
// workgroup sum (FP64) goes to its own slot; a second kernel adds the slots
// of each image in a fixed order, so the result is the same on every run.
#include "internal.hpp"

namespace lp {

constexpr int kWin = 11, kHalo = kWin - 1, kTile = 16, kIn = kTile + kHalo;

__global__ __launch_bounds__(256) void ssim_tile_kernel(SsimParams P) {
    __shared__ float A[kIn][kIn + 1], B[kIn][kIn + 1];
    __shared__ float Hm[5][kIn][kTile + 1];
    __shared__ double red[256];
    const int Wv = P.W - kHalo, Hv = P.H - kHalo;
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    const int img = blockIdx.z / 3, ch = blockIdx.z % 3;
    const float* a = P.a + (size_t)img * P.H * P.W * 3;
    const float* b = P.b + (size_t)img * P.H * P.W * 3;
    for (int e = threadIdx.x; e < kIn * kIn; e += 256) {
        const int ty = e / kIn, tx = e - ty * kIn;
        const int x = x0 + tx, y = y0 + ty;
        float va = 0.0f, vb = 0.0f;
        if (x < P.W && y < P.H) {
            const size_t o = ((size_t)y * P.W + x) * 3 + ch;
            va = a[o];
            vb = b[o];
        }
        A[ty][tx] = va;
        B[ty][tx] = vb;
    }
    __syncthreads();
    // horizontal pass: 26 rows x 16 columns of the five moments
    for (int e = threadIdx.x; e < kIn * kTile; e += 256) {
        const int ty = e / kTile, tx = e - ty * kTile;
        float ma = 0.0f, mb = 0.0f, aa = 0.0f, bb = 0.0f, ab = 0.0f;
#pragma unroll
        for (int t = 0; t < kWin; ++t) {
            const float w = P.w[t], va = A[ty][tx + t], vb = B[ty][tx + t];
            ma = fmaf(w, va, ma);
            mb = fmaf(w, vb, mb);
            aa = fmaf(w, va * va, aa);
            bb = fmaf(w, vb * vb, bb);
            ab = fmaf(w, va * vb, ab);
        }
        Hm[0][ty][tx] = ma;
        Hm[1][ty][tx] = mb;
        Hm[2][ty][tx] = aa;
        Hm[3][ty][tx] = bb;
        Hm[4][ty][tx] = ab;
    }
    __syncthreads();
    // vertical pass and the SSIM term of this thread's window position
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    double term = 0.0;
    if (x0 + tx < Wv && y0 + ty < Hv) {
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < kWin; ++t) {
            const float w = P.w[t];
#pragma unroll
            for (int q = 0; q < 5; ++q) m[q] = fmaf(w, Hm[q][ty + t][tx], m[q]);
        }
        const float va = m[2] - m[0] * m[0], vb = m[3] - m[1] * m[1], cab = m[4] - m[0] * m[1];
        const float num = (2.0f * m[0] * m[1] + P.c1) * (2.0f * cab + P.c2);
        const float den = (m[0] * m[0] + m[1] * m[1] + P.c1) * (va + vb + P.c2);
        term = (double)(num / den);
    }
    red[threadIdx.x] = term;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t slot = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        P.partial[slot] = red[0];
    }
}

// Mean SSIM of each image: its 3 * tiles slots in order, over 3 Wv Hv terms.
__global__ void ssim_reduce_kernel(SsimParams P, int slots_per_image) {
    const int img = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    for (int e = threadIdx.x; e < slots_per_image; e += 256) s += P.partial[(size_t)img * slots_per_image + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) P.out[img] = red[0] / (3.0 * (double)(P.W - kHalo) * (double)(P.H - kHalo));
}

hipError_t launch_ssim(const SsimParams& P, int n_images, hipStream_t s) {
    const int Wv = P.W - kHalo, Hv = P.H - kHalo;
    dim3 grid((Wv + kTile - 1) / kTile, (Hv + kTile - 1) / kTile, 3 * n_images);
    ssim_tile_kernel<<<grid, 256, 0, s>>>(P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ssim_reduce_kernel<<<n_images, 256, 0, s>>>(P, (int)(3 * grid.x * grid.y));
    return hipGetLastError();
}

size_t ssim_partial_count(int n_images, int W, int H) {
    const size_t gx = (size_t)(W - kHalo + kTile - 1) / kTile, gy = (size_t)(H - kHalo + kTile - 1) / kTile;
    return gx * gy * 3 * (size_t)n_images;
}

}  // namespace lp
