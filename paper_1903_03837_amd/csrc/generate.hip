// generate.hip -- light-field generation (Sec. 2, Fig. 1) and its adjoint.
//
// Work decomposition: rays are grouped in 8 x 8 tiles (8 origins i x 8
// directions j) and every wave64 takes whole tiles in a grid-stride loop, one
// ray per lane.  All spp samples of a ray run in order in its lane, so the
// texel is a deterministic FP32 sum, written once (12 B FP32 or 6 B
// FP16/BF16 per texel).  The transfer function lives in LDS; the volume is
// read with plain loads (it stays in L2 / the Infinity Cache for the 8-32 MiB
// volumes).  The adjoint kernel keeps a per-workgroup LDS copy of dLUT and
// flushes it with one atomic per entry at the end.
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

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void store_texel(const TraceParams& P, uint64_t k, f3 v) {
    if (P.dtype == 0) {
        float* o = (float*)P.out + 3 * k;
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
    } else if (P.dtype == 1) {
        __half* o = (__half*)P.out + 3 * k;
        o[0] = __float2half_rn(v.x);
        o[1] = __float2half_rn(v.y);
        o[2] = __float2half_rn(v.z);
    } else {
        uint16_t* o = (uint16_t*)P.out + 3 * k;
        o[0] = bf16_rne(v.x);
        o[1] = bf16_rne(v.y);
        o[2] = bf16_rne(v.z);
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int VT, int BR, int MODE>
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
                    const f3 lt = trace_sample<VT, BR, kFwd>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir,
                                                             (uint32_t)s, cnt, acc, adj, G);
                    trace_sample<VT, BR, kGrad>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir, (uint32_t)s, cnt,
                                                lt, adj, G);
                } else {
                    acc = acc + trace_sample<VT, BR, MODE>(P, lut_e, lut_s, sigbar, inv_sigbar, k, po, dir,
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

template <int VT, int BR, int MODE>
static hipError_t launch_gen_t(const TraceParams& P, hipStream_t s) {
    const long long rows = P.row_end - P.row_begin;
    const long long ntiles = ((rows + 7) / 8) * (long long)((P.N + 7) / 8);
    if (ntiles <= 0) return hipSuccess;
    // 4 tiles (waves) per workgroup; the adjoint runs as a persistent grid so
    // that only a few thousand workgroups flush their LDS gradients.
    const long long cap = MODE == kGrad ? 2048 : 16384;
    long long blocks = (ntiles + 3) / 4;
    if (blocks > cap) blocks = cap;
    const size_t lds = sizeof(float4) * (size_t)P.lut_n * (MODE == kFrozen ? 2 : 1) +
                       (MODE == kGrad ? sizeof(float) * (4 * (size_t)P.lut_n + 1) : 0);
    gen_kernel<VT, BR, MODE><<<(unsigned)blocks, 256, lds, s>>>(P);
    return hipGetLastError();
}

template <int VT, int BR>
static hipError_t launch_gen_mode(const TraceParams& P, int mode, hipStream_t s) {
    switch (mode) {
        case kFwd: return launch_gen_t<VT, BR, kFwd>(P, s);
        case kFrozen: return launch_gen_t<VT, BR, kFrozen>(P, s);
        default: return launch_gen_t<VT, BR, kGrad>(P, s);
    }
}

template <int VT>
static hipError_t launch_gen_brick(const TraceParams& P, int brick, int mode, hipStream_t s) {
    return brick ? launch_gen_mode<VT, 1>(P, mode, s) : launch_gen_mode<VT, 0>(P, mode, s);
}

hipError_t launch_generate(const TraceParams& P, int vtype, int brick, int mode, hipStream_t s) {
    switch (vtype) {
        case 0: return launch_gen_brick<0>(P, brick, mode, s);
        case 1: return launch_gen_brick<1>(P, brick, mode, s);
        default: return launch_gen_brick<2>(P, brick, mode, s);
    }
}

}  // namespace lp
