// generate.hip -- adjoint of light-field generation (path replay), plus the
// small majorant and zero-fill kernels.
//
// Work decomposition: rays are grouped in 8 x 8 tiles (8 origins i x 8
// directions j) and every wave64 takes whole tiles in a grid-stride loop, one
// ray per lane; each sample is traced twice (its total radiance, then the
// score replay).  Rays whose adjoint is zero are skipped, which removes most
// of the work when the adjoint comes from a few views.  The transfer
// function lives in LDS; the kernel keeps a per-workgroup LDS copy of dLUT
// and flushes it with one atomic per entry at the end.
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

template <int VT, int MODE>
__global__ __launch_bounds__(256) void gen_kernel(TraceParams P) {
    extern __shared__ float4 smem[];
    float4* lut_e = smem;
    float4* lut_s = smem + (MODE == kFrozen ? P.lut_n : 0);
    float* glds = (float*)(smem + (MODE == kFrozen ? 2 : 1) * P.lut_n);
    for (int e = threadIdx.x; e < P.lut_n; e += blockDim.x) {
        lut_e[e] = ((const float4*)P.lut_e)[e];
        if constexpr (MODE == kFrozen) lut_s[e] = ((const float4*)P.lut_s)[e];
    }
    if constexpr (MODE == kGrad)
        for (int e = threadIdx.x; e < 4 * P.lut_n + 1; e += blockDim.x) glds[e] = 0.0f;
    __syncthreads();

    const float sigbar = *P.sigbar;
    const float inv_sigbar = sigbar > 0.0f ? 1.0f / sigbar : 0.0f;
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    const int rows = P.row_end - P.row_begin;
    const long long tiles_j = (P.N + 7) / 8;
    const long long ntiles = (long long)((rows + 7) / 8) * tiles_j;
    const float invM = 1.0f / (float)P.M, invN = 1.0f / (float)P.N;
    Counters cnt = {0, 0, 0, 0};
    GradAcc G;
    G.lds = glds;
    G.cl0 = -1;
    G.c0 = G.c1 = 0.0f;
    G.dscale = 0.0f;

    for (long long t = wave; t < ntiles; t += nwaves) {
        const int ti = (int)(t / tiles_j), tj = (int)(t - (long long)ti * tiles_j);
        const int i = P.row_begin + ti * 8 + (lane >> 3);
        const int j = tj * 8 + (lane & 7);
        if (i >= P.row_end || j >= P.N) continue;
        const uint32_t k = (uint32_t)i * (uint32_t)P.N + (uint32_t)j;
        const bool degenerate = P.M == P.N && i == j;
        f3 adj = mk3(0.0f, 0.0f, 0.0f);
        if constexpr (MODE == kGrad) {
            if (degenerate) continue;
            const float* a = P.d_lf + 3 * (uint64_t)k;
            const float inv_spp = 1.0f / (float)P.spp;
            adj = mk3(a[0] * inv_spp, a[1] * inv_spp, a[2] * inv_spp);
            if (adj.x == 0.0f && adj.y == 0.0f && adj.z == 0.0f) continue;
        }
        f3 acc = mk3(0.0f, 0.0f, 0.0f);
        if (!degenerate) {
            const f3 po = sf_point(P.M, i, invM);
            const f3 pd = sf_point(P.N, j, invN);
            const f3 dir = normalize(pd - po);
            for (int s = 0; s < P.spp; ++s) {
                if constexpr (MODE == kGrad) {
                    const f3 lt = trace_sample<VT, kFwd>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir,
                                                             (uint32_t)s, cnt, acc, adj, G);
                    trace_sample<VT, kGrad>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir, (uint32_t)s, cnt,
                                                lt, adj, G);
                } else {
                    acc = acc + trace_sample<VT, MODE>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir,
                                                           (uint32_t)s, cnt, acc, adj, G);
                }
            }
        }
        if constexpr (MODE != kGrad) {
            const float fs = (float)P.spp;
            store_texel(P, k, mk3(acc.x / fs, acc.y / fs, acc.z / fs));
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
    } else {
        if (P.stats) {
            const uint32_t a = wave_sum(cnt.tent), b = wave_sum(cnt.shadow), c = wave_sum(cnt.real),
                           d = wave_sum(cnt.samples);
            if (lane == 0) {
                atomicAdd(&P.stats[0], (unsigned long long)a);
                atomicAdd(&P.stats[1], (unsigned long long)b);
                atomicAdd(&P.stats[2], (unsigned long long)c);
                atomicAdd(&P.stats[3], (unsigned long long)d);
            }
        }
    }
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

template <int VT>
static hipError_t launch_bwd_t(const TraceParams& P, hipStream_t s) {
    const long long rows = P.row_end - P.row_begin;
    const long long ntiles = ((rows + 7) / 8) * (long long)((P.N + 7) / 8);
    if (ntiles <= 0) return hipSuccess;
    // 4 tiles (waves) per workgroup as a persistent grid, so that only a few
    // thousand workgroups flush their LDS gradients.
    long long blocks = (ntiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    const size_t lds = sizeof(float4) * (size_t)P.lut_n + sizeof(float) * (4 * (size_t)P.lut_n + 1);
    gen_kernel<VT, kGrad><<<(unsigned)blocks, 256, lds, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_backward(const TraceParams& P, int vtype, hipStream_t s) {
    switch (vtype) {
        case 0: return launch_bwd_t<0>(P, s);
        case 1: return launch_bwd_t<1>(P, s);
        default: return launch_bwd_t<2>(P, s);
    }
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
