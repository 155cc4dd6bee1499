// internal.hpp -- launch entry points of the kernels, called by the C ABI in
// api.cpp after argument validation.
#pragma once

#include <hip/hip_runtime.h>

#include "tracer_device.hpp"

namespace lp {

constexpr int kMaxViewsPerLaunch = 24;

struct ViewGeom {
    float oc[3];      // eye - O
    float fwd[3], right[3], up[3];
    float c;          // |eye - O|^2 - R^2
    float sx, sy;     // tan(vfov / 2) * aspect, tan(vfov / 2)
};

struct LookupParams {
    int32_t M, N;
    float invM, invN;
    float inv_rM, inv_rN;   // 1 / sqrt(4 pi / n)
    int32_t W, H, K;
    int32_t nviews, view0;
    int32_t dtype, degenerate;
    int32_t orows;          // stored origin rows: neighbours i >= orows are uncovered
    float thr;              // tangent threshold 1e-6 R^2
    const void* lf;
    float* img;
    float* d_lf;
    const float* target;    // fused L2 adjoint: target views
    int32_t* nn;
    const float4* tab_o;    // SF point tables (workspace), float4 per point
    const float4* tab_d;
    const SfZone* zone_o;   // zone bases of both sets (workspace), kZones each
    const SfZone* zone_d;
    ViewGeom v[kMaxViewsPerLaunch];
};

// Mean SSIM of image pairs [n][H][W][3] (metrics.hip).
struct SsimParams {
    const float* a;
    const float* b;
    int32_t W, H;
    float w[11];            // normalised 1-D Gaussian window, sigma 1.5
    float c1, c2;           // (0.01 L)^2, (0.03 L)^2
    double* partial;        // one slot per workgroup
    double* out;            // [n] mean SSIM
};

hipError_t launch_ssim(const SsimParams& P, int n_images, hipStream_t s);
size_t ssim_partial_count(int n_images, int W, int H);

// CW-SSIM of image pairs (metrics.hip): workspace pieces and launch.
struct CwParams {
    const float* a;
    const float* b;
    int32_t W, H;
    float K;           // 49 (0.01 data_range)^2
    float2* tw_w;      // [W] twiddles (cos, sin) of 2 pi m / W
    float2* tw_h;      // [H]
    float2* spec;      // [6][H][W] spectra of the six planes of one image pair
    float2* t1;        // [6][H][W] scratch planes
    float2* t2;        // [6][H][W]
    double* slots;     // workgroup sums of one image pair
    double* out;       // [n_images]
};
size_t cw_ssim_slots(int W, int H);
hipError_t launch_cw_ssim(const CwParams& P, int n_images, hipStream_t s);

hipError_t launch_points(int n, float* xyz, const float* query, long long nq, int K, int* idx, float* w,
                         hipStream_t s);
// Halo bricks along an axis of n >= 2 voxels: base voxels 0 .. n-2, three per brick.
inline int halo_bricks(int n) { return (n - 2) / 3 + 1; }
hipError_t launch_halo_bricks(const void* src, int vtype, int layout, int nx, int ny, int nz, void* dst,
                              hipStream_t s);
hipError_t launch_wave_setup(const TraceParams& P, const float* sample_lut, int lut_n, float sample_scale,
                             float given, float* sigbar, unsigned int* ctr, int32_t* perm_o, int32_t* perm_d,
                             hipStream_t s);
hipError_t launch_majorant_grid(const void* vol, int vtype, int layout, int nx, int ny, int nz, int G,
                                const float* lut, int lut_n, float scale, double vmin, double vmax, float* out,
                                float* range, hipStream_t s);
hipError_t launch_surface(const TraceParams& P, int vtype, hipStream_t s);

// Up to kViewBatch ground-truth views per argument block.
constexpr int kViewBatch = 32;
struct ViewBatch {
    ViewCam v[kViewBatch];
    int32_t first, count;
};
hipError_t launch_fill_views(const ViewBatch& b, ViewCam* dst, hipStream_t s);
hipError_t launch_generate_wave(const TraceParams& P, int vtype, int mode, hipStream_t s);
hipError_t launch_active_rays(const TraceParams& P, hipStream_t s);
hipError_t launch_zero(float* p, long long n, hipStream_t s);
hipError_t launch_lookup(const LookupParams& P, int mode, hipStream_t s);
// Fixed device scratch of lf_lookup_static (lookup.hip): room for the point
// tables and zone bases of two SF sets of up to 65536 points each.  lookup_scratch() gives
// its address on device `dev`, which must be the current device on the first
// call for that device.
// (each zone table: kZones bases of 32 bytes, 768 bytes with alignment)
constexpr size_t kZoneTableBytes = 768;
static_assert(sizeof(SfZone) * kZones <= kZoneTableBytes, "zone table");
constexpr size_t kLookupScratchPoints = 2 * 65536 + 2 * kZoneTableBytes / 16;
constexpr size_t kLookupScratchBytes = kLookupScratchPoints * 16;
constexpr int kMaxScratchDevices = 64;
hipError_t lookup_scratch(int dev, void** ptr);
hipError_t launch_sf_tables(const LookupParams& P, hipStream_t s);
hipError_t launch_combine_parts(const TraceParams& P, hipStream_t s);
// Table of the n SF points sf_point(n, i, inv_n) as float4 (w = 0).
hipError_t launch_sf_table(int n, float inv_n, float4* out, hipStream_t s);

}  // namespace lp
