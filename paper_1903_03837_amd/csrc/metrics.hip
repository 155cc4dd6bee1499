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

// ---------------------------------------------------------------------------
// CW-SSIM (Wang & Simoncelli 2005, Sampat et al. 2009; the second index the
// paper reports): complex subbands of a steerable filter bank defined in the
// DFT domain, 2 scales x 4 orientations (the eight levels the paper names),
// and the local index
//     S = (2 |sum c_x conj(c_y)| + K) / (sum |c_x|^2 + sum |c_y|^2 + K)
// over 7 x 7 windows inside the image, averaged over positions, subbands and
// channels.  Filter of scale s, orientation k at DFT index (u, v): signed
// frequencies f = u (2u < n) or u - n, w = 2 pi f / n, r = |w|, theta =
// atan2(w_y, w_x); R_s = cos(pi/2 log2(r / r_s)) for |log2(r / r_s)| < 1,
// r_s = pi / 2^(s+1); A_k = cos(d)^3 for |d| < pi/2, d = theta - pi k / 4
// wrapped to (-pi, pi].
//
// Per image, the six planes (two images x three channels) go through a
// direct separable DFT (rows with the row and the twiddles in LDS, then
// columns coalesced along x; twiddle index (u x) mod n, so no phase
// rounding grows with the index), then per subband: spectrum x filter
// (with the 1 / (W H) of the inverse), inverse columns, inverse rows, and
// the windowed index of 16 x 16 positions per workgroup from LDS tiles.
// Workgroup sums (FP64) go to slots that one kernel adds in a fixed order.
// The DFT costs O(W H (W + H)) per plane: this is a metric for views of a
// few hundred pixels a side, not a hot path.

constexpr int kCwScales = 2, kCwOrients = 4, kCwBands = kCwScales * kCwOrients;
constexpr int kCwWin = 7, kCwHalo = kCwWin - 1, kCwTile = 16, kCwIn = kCwTile + kCwHalo;

__global__ void cw_twiddle_kernel(int n, float2* tw) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    tw[m] = make_float2((float)cs, (float)sn);
}

// planes[p][y][x] = channel p % 3 of image a (p < 3) or b, as complex values
__global__ void cw_planes_kernel(const float* a, const float* b, int W, int H, float2* planes) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)W * H;
    if (e >= n) return;
#pragma unroll
    for (int p = 0; p < 6; ++p) planes[p * n + e] = make_float2((p < 3 ? a : b)[3 * e + p % 3], 0.0f);
}

// out[p][y][u] = sum_x in[p][y][x] exp(-+ 2 pi i u x / W)  (inverse: +)
__global__ __launch_bounds__(256) void cw_dft_rows_kernel(const float2* in, float2* out, const float2* tw, int W,
                                                          int H, int inverse) {
    extern __shared__ float2 cw_lds[];
    float2* row = cw_lds;
    float2* t = cw_lds + W;
    const int y = blockIdx.y, p = blockIdx.z;
    const float2* src = in + ((size_t)p * H + y) * W;
    for (int x = threadIdx.x; x < W; x += 256) {
        row[x] = src[x];
        t[x] = tw[x];
    }
    __syncthreads();
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= W) return;
    const float sg = inverse ? 1.0f : -1.0f;
    float re = 0.0f, im = 0.0f;
    int m = 0;
    for (int x = 0; x < W; ++x) {
        const float2 v = row[x], w = t[m];
        const float ws = sg * w.y;
        re = fmaf(v.x, w.x, fmaf(-v.y, ws, re));
        im = fmaf(v.x, ws, fmaf(v.y, w.x, im));
        m += u;
        if (m >= W) m -= W;
    }
    out[((size_t)p * H + y) * W + u] = make_float2(re, im);
}

// out[p][v][x] = sum_y in[p][y][x] exp(-+ 2 pi i v y / H)  (inverse: +)
__global__ __launch_bounds__(256) void cw_dft_cols_kernel(const float2* in, float2* out, const float2* tw, int W,
                                                          int H, int inverse) {
    const int x = blockIdx.x * 256 + threadIdx.x, v = blockIdx.y, p = blockIdx.z;
    if (x >= W) return;
    const float sg = inverse ? 1.0f : -1.0f;
    const float2* src = in + (size_t)p * H * W + x;
    float re = 0.0f, im = 0.0f;
    int m = 0;
    for (int y = 0; y < H; ++y) {
        const float2 c = src[(size_t)y * W], w = tw[m];
        const float ws = sg * w.y;
        re = fmaf(c.x, w.x, fmaf(-c.y, ws, re));
        im = fmaf(c.x, ws, fmaf(c.y, w.x, im));
        m += v;
        if (m >= H) m -= H;
    }
    out[((size_t)p * H + v) * W + x] = make_float2(re, im);
}

// out[p] = spec[p] * F_sk / (W H) for the six planes
__global__ void cw_filter_kernel(const float2* spec, float2* out, int W, int H, int s, int k) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)W * H;
    if (e >= n) return;
    const int v = (int)(e / W), u = (int)(e - (long long)v * W);
    const double pi = 3.141592653589793;
    const double fu = 2 * u < W ? u : u - W, fv = 2 * v < H ? v : v - H;
    const double wx = 2.0 * pi * fu / W, wy = 2.0 * pi * fv / H;
    const double r = sqrt(wx * wx + wy * wy);
    double f = 0.0;
    if (r > 0.0) {
        const double lr = log2(r / (pi / (double)(2 << s)));
        if (fabs(lr) < 1.0) {
            const double d = remainder(atan2(wy, wx) - pi * k / kCwOrients, 2.0 * pi);
            if (fabs(d) < 0.5 * pi) {
                const double c = cos(d);
                f = cos(0.5 * pi * lr) * c * c * c;
            }
        }
    }
    const float g = (float)(f / ((double)W * (double)H));
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const float2 z = spec[p * n + e];
        out[p * n + e] = make_float2(z.x * g, z.y * g);
    }
}

// windowed index of 16 x 16 positions of channel blockIdx.z of one subband;
// the workgroup's FP64 sum goes to slots[(ch * gy + by) * gx + bx]
__global__ __launch_bounds__(256) void cw_map_kernel(const float2* coef, int W, int H, float K, double* slots) {
    __shared__ float Q[4][kCwIn][kCwIn + 1];     // re, im of c_x conj(c_y), |c_x|^2, |c_y|^2
    __shared__ float Hs[4][kCwIn][kCwTile + 1];  // horizontal 7-sums
    __shared__ double red[256];
    const int Wv = W - kCwHalo, Hv = H - kCwHalo;
    const int x0 = blockIdx.x * kCwTile, y0 = blockIdx.y * kCwTile, ch = blockIdx.z;
    const size_t n = (size_t)W * H;
    const float2* cx = coef + ch * n;
    const float2* cy = coef + (3 + ch) * n;
    for (int e = threadIdx.x; e < kCwIn * kCwIn; e += 256) {
        const int ty = e / kCwIn, tx = e - ty * kCwIn;
        const int x = x0 + tx, y = y0 + ty;
        float2 a = make_float2(0.0f, 0.0f), b = a;
        if (x < W && y < H) {
            a = cx[(size_t)y * W + x];
            b = cy[(size_t)y * W + x];
        }
        Q[0][ty][tx] = a.x * b.x + a.y * b.y;
        Q[1][ty][tx] = a.y * b.x - a.x * b.y;
        Q[2][ty][tx] = a.x * a.x + a.y * a.y;
        Q[3][ty][tx] = b.x * b.x + b.y * b.y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCwIn * kCwTile; e += 256) {
        const int ty = e / kCwTile, tx = e - ty * kCwTile;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float sum = 0.0f;
#pragma unroll
            for (int d = 0; d < kCwWin; ++d) sum += Q[q][ty][tx + d];
            Hs[q][ty][tx] = sum;
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kCwTile, ty = threadIdx.x / kCwTile;
    double term = 0.0;
    if (x0 + tx < Wv && y0 + ty < Hv) {
        float q[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float sum = 0.0f;
#pragma unroll
            for (int d = 0; d < kCwWin; ++d) sum += Hs[c][ty + d][tx];
            q[c] = sum;
        }
        const float num = 2.0f * sqrtf(q[0] * q[0] + q[1] * q[1]) + K;
        const float den = q[2] + q[3] + K;
        term = den > 0.0f ? (double)(num / den) : 1.0;
    }
    red[threadIdx.x] = term;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) slots[((size_t)ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void cw_reduce_kernel(const double* slots, int nslots, double scale, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int e = threadIdx.x; e < nslots; e += 256) s += slots[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

size_t cw_ssim_slots(int W, int H) {
    const size_t gx = (size_t)(W - kCwHalo + kCwTile - 1) / kCwTile, gy = (size_t)(H - kCwHalo + kCwTile - 1) / kCwTile;
    return gx * gy * 3 * kCwBands;
}

hipError_t launch_cw_ssim(const CwParams& P, int n_images, hipStream_t s) {
    const int W = P.W, H = P.H;
    const long long n = (long long)W * H;
    const unsigned eb = (unsigned)((n + 255) / 256);
    const dim3 rows_grid((W + 255) / 256, H, 6), cols_grid((W + 255) / 256, H, 6);
    const size_t rows_lds = 2 * sizeof(float2) * (size_t)W;
    const int gx = (W - kCwHalo + kCwTile - 1) / kCwTile, gy = (H - kCwHalo + kCwTile - 1) / kCwTile;
    const size_t band_slots = (size_t)gx * gy * 3;
    const double scale = 1.0 / (3.0 * kCwBands * (double)(W - kCwHalo) * (double)(H - kCwHalo));
    cw_twiddle_kernel<<<(W + 255) / 256, 256, 0, s>>>(W, P.tw_w);
    cw_twiddle_kernel<<<(H + 255) / 256, 256, 0, s>>>(H, P.tw_h);
    for (int img = 0; img < n_images; ++img) {
        const float* a = P.a + (size_t)img * n * 3;
        const float* b = P.b + (size_t)img * n * 3;
        cw_planes_kernel<<<eb, 256, 0, s>>>(a, b, W, H, P.t1);
        cw_dft_rows_kernel<<<rows_grid, 256, rows_lds, s>>>(P.t1, P.t2, P.tw_w, W, H, 0);
        cw_dft_cols_kernel<<<cols_grid, 256, 0, s>>>(P.t2, P.spec, P.tw_h, W, H, 0);
        for (int band = 0; band < kCwBands; ++band) {
            cw_filter_kernel<<<eb, 256, 0, s>>>(P.spec, P.t1, W, H, band / kCwOrients, band % kCwOrients);
            cw_dft_cols_kernel<<<cols_grid, 256, 0, s>>>(P.t1, P.t2, P.tw_h, W, H, 1);
            cw_dft_rows_kernel<<<rows_grid, 256, rows_lds, s>>>(P.t2, P.t1, P.tw_w, W, H, 1);
            cw_map_kernel<<<dim3(gx, gy, 3), 256, 0, s>>>(P.t1, W, H, P.K, P.slots + band * band_slots);
        }
        cw_reduce_kernel<<<1, 256, 0, s>>>(P.slots, (int)(band_slots * kCwBands), scale, P.out + img);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lp
