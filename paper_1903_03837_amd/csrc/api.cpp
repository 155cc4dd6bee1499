// api.cpp -- the C ABI of liblumipath.so (include/lumipath.h): host-side
// argument validation, parameter packing and kernel launches.  Validation
// finishes before any HIP call, so a bad argument never touches the device.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lumipath.h"
#include "internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(LF_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Voxels of the volume's halo-brick copy (4^3-voxel bricks every 3 voxels).
size_t brick_voxels(const lf_volume* v) {
    return 64 * (size_t)lp::halo_bricks(v->nx) * (size_t)lp::halo_bricks(v->ny) * (size_t)lp::halo_bricks(v->nz);
}

size_t brick_copy_bytes(const lf_volume* v) {
    const size_t esz = v->type == LF_VOX_U8 ? 1 : (v->type == LF_VOX_U16 ? 2 : 4);
    return align256(esz * brick_voxels(v));
}

// lf_generate workspace: majorant (offset 0), 8 tile counters (offset 64),
// spatial order of the generated origin rows (offset 256), spatial order of
// the directions, the cell majorants of the grid (when used), the point
// tables of both SF sets, then the brick copy of the volume.
long long stored_rows(const lf_gen_params* p) { return p->origin_rows > 0 ? p->origin_rows : p->M; }

// Sample ranges per ray (log2) of the path tracer's work items.  The
// adjoint (rays with a nonzero adjoint only, often a small share of the
// field) takes at most 16 ranges per ray of at least 2 samples each.  A
// forward takes at most 4 ranges from 32 samples, 2 from 16; it keeps each
// range's sum (12 bytes) until a second kernel adds them; it splits by the
// rays per lane
// of a nominal full grid (256 CUs x 3 waves x 4 SIMDs x 64 lanes = 196608):
// 4 ranges below 8 rays per lane, 2 below 64, else 1, and never when
// M*N*spp > 2^31.  The rule depends on M, N and spp only, so the field does
// not depend on the device or the row split.
int part_log2(const lf_gen_params* p, bool forward) {
    if (!forward) {  // adjoint: at most 16 ranges per ray, at least 2 samples each
        int l = 0;
        while (l < 4 && (p->spp >> (l + 1)) >= 2) ++l;
        return l;
    }
    const int by_spp = p->spp >= 32 ? 2 : (p->spp >= 16 ? 1 : 0);
    const unsigned long long rays = (unsigned long long)p->M * (unsigned long long)p->N;
    if (rays * (unsigned long long)p->spp > (1ull << 31)) return 0;
    const int by_rays = rays < 8ull * 196608 ? 2 : (rays < 64ull * 196608 ? 1 : 0);
    return by_spp < by_rays ? by_spp : by_rays;
}

// The same rule for ground-truth views, by pixels instead of rays.
int view_part_log2(int spp, unsigned long long pixels) {
    if (pixels * (unsigned long long)spp > (1ull << 31)) return 0;
    const int by_spp = spp >= 32 ? 2 : (spp >= 16 ? 1 : 0);
    const int by_px = pixels < 8ull * 196608 ? 2 : (pixels < 64ull * 196608 ? 1 : 0);
    return by_spp < by_px ? by_spp : by_px;
}

size_t part_sums_bytes(const lf_gen_params* p) {
    if (p->surface) return 0;
    const int pl = part_log2(p, true);
    if (pl == 0) return 0;
    const long long re = p->row_end <= 0 ? stored_rows(p) : p->row_end;
    return align256(12 * (size_t)(re - p->row_begin) * (size_t)p->N << pl);
}

// Cells per axis of the majorant grid in use (0: the global majorant).
int grid_cells(const lf_gen_params* p) { return p->majorant > 0.0f ? 0 : p->majorant_grid; }

size_t gen_perm_bytes(const lf_gen_params* p) {
    const long long re = p->row_end <= 0 ? stored_rows(p) : p->row_end;
    const size_t rows = (size_t)(re - p->row_begin);
    return 256 + align256(4 * rows) + align256(4 * (size_t)p->N);
}

size_t gen_grid_bytes(const lf_gen_params* p) {
    const size_t G = (size_t)grid_cells(p);
    return align256(4 * G * G * G);
}

size_t gen_order_bytes(const lf_gen_params* p) {
    return gen_perm_bytes(p) + gen_grid_bytes(p) + align256(16 * (size_t)p->M) + align256(16 * (size_t)p->N);
}

int check_params(const lf_gen_params* p, bool need_rays) {
    if (!p) return fail(LF_E_ARG, "params is NULL");
    if (p->M < 1 || p->N < 1) return fail(LF_E_ARG, "M and N must be >= 1 (got %d, %d)", p->M, p->N);
    if (p->M > 65535 || p->N > 65535) return fail(LF_E_RANGE, "M and N must be <= 65535");
    if ((unsigned long long)p->M * (unsigned long long)p->N >= (1ull << 32))
        return fail(LF_E_RANGE, "M*N must be < 2^32");
    if (!(p->radius > 0.0f) || !std::isfinite(p->radius)) return fail(LF_E_ARG, "radius must be > 0");
    if (!finite3(p->center)) return fail(LF_E_ARG, "center must be finite");
    if (p->origin_rows < 0 || p->origin_rows > p->M) return fail(LF_E_ARG, "origin_rows must be in [0, M]");
    if (!need_rays) return LF_OK;
    if (p->spp < 1) return fail(LF_E_ARG, "spp must be >= 1");
    if (p->max_bounces < 1 || p->max_bounces > 65535) return fail(LF_E_ARG, "max_bounces must be in [1, 65535]");
    if (!(std::fabs(p->hg_g) < 1.0f)) return fail(LF_E_ARG, "|hg_g| must be < 1");
    if (!std::isfinite(p->majorant)) return fail(LF_E_ARG, "majorant must be finite");
    if (p->majorant_grid < 0 || p->majorant_grid > 16)
        return fail(LF_E_ARG, "majorant_grid must be in [0, 16] (got %d)", p->majorant_grid);
    if (p->surface != 0 && p->surface != 1) return fail(LF_E_ARG, "surface must be 0 or 1");
    if (p->waves_per_simd != 0 && p->waves_per_simd != 3 && p->waves_per_simd != 4)
        return fail(LF_E_ARG, "waves_per_simd must be 0, 3 or 4 (got %d)", p->waves_per_simd);
    if (!std::isfinite(p->iso)) return fail(LF_E_ARG, "iso must be finite");
    if (p->sample_radiance && p->surface)
        return fail(LF_E_UNSUPPORTED, "sample_radiance is not available in the isosurface variant");
    if ((uintptr_t)p->sample_radiance % 4) return fail(LF_E_ARG, "sample_radiance is not aligned to 4 bytes");
    const long long rows = p->origin_rows > 0 ? p->origin_rows : p->M;
    const long long re = p->row_end <= 0 ? rows : p->row_end;
    if (p->row_begin < 0 || p->row_begin > re || re > rows)
        return fail(LF_E_ARG, "row range [%lld, %lld) outside [0, %lld)", (long long)p->row_begin, re, rows);
    return LF_OK;
}

int check_volume(const lf_volume* v) {
    if (!v) return fail(LF_E_ARG, "volume is NULL");
    if (!v->data) return fail(LF_E_ARG, "volume data is NULL");
    if (v->type < LF_VOX_U8 || v->type > LF_VOX_F32) return fail(LF_E_ARG, "unknown voxel type %d", v->type);
    if (v->nx < 2 || v->ny < 2 || v->nz < 2) return fail(LF_E_ARG, "volume dimensions must be >= 2");
    if (v->nx > 65535 || v->ny > 65535 || v->nz > 65535 || brick_voxels(v) > 0xFFFFFFFFull)
        return fail(LF_E_RANGE, "volume too large: its halo-brick copy (%zu voxels) needs 32-bit voxel indices",
                    brick_voxels(v));
    const uintptr_t esz = v->type == LF_VOX_U8 ? 1 : (v->type == LF_VOX_U16 ? 2 : 4);
    if ((uintptr_t)v->data % esz) return fail(LF_E_ARG, "volume data is not aligned to its voxel size");
    if (v->brick != 0 && v->brick != 8) return fail(LF_E_UNSUPPORTED, "brick must be 0 or 8");
    if (v->brick == 8 && (v->nx % 8 || v->ny % 8 || v->nz % 8))
        return fail(LF_E_ARG, "bricked volume dimensions must be multiples of 8");
    if (!(v->vmax > v->vmin) || !std::isfinite(v->vmin) || !std::isfinite(v->vmax))
        return fail(LF_E_ARG, "vmax must exceed vmin");
    for (int a = 0; a < 3; ++a)
        if (!(v->box_max[a] > v->box_min[a]) || !std::isfinite(v->box_min[a]) || !std::isfinite(v->box_max[a]))
            return fail(LF_E_ARG, "box_max must exceed box_min on every axis");
    return LF_OK;
}

int check_medium(const lf_medium* m, const char* name) {
    if (!m) return fail(LF_E_ARG, "%s medium is NULL", name);
    if (!m->lut) return fail(LF_E_ARG, "%s lut is NULL", name);
    if ((uintptr_t)m->lut % 16) return fail(LF_E_ARG, "%s lut must be 16-byte aligned", name);
    if (m->lut_size < 2 || m->lut_size > 1024) return fail(LF_E_ARG, "%s lut_size must be in [2, 1024]", name);
    if (!(m->density_scale >= 0.0f) || !std::isfinite(m->density_scale))
        return fail(LF_E_ARG, "%s density_scale must be finite and >= 0", name);
    return LF_OK;
}

int check_light(const lf_light* l) {
    if (!l) return fail(LF_E_ARG, "light is NULL");
    if (!finite3(l->radiance) || !finite3(l->env)) return fail(LF_E_ARG, "light radiance/env must be finite");
    if (l->kind == LF_LIGHT_DIRECTIONAL) {
        const double n = std::sqrt((double)l->dir[0] * l->dir[0] + (double)l->dir[1] * l->dir[1] +
                                   (double)l->dir[2] * l->dir[2]);
        if (!(std::fabs(n - 1.0) < 1e-3)) return fail(LF_E_ARG, "directional light dir must be a unit vector");
    } else if (l->kind == LF_LIGHT_AREA) {
        const double cx = (double)l->e1[1] * l->e2[2] - (double)l->e1[2] * l->e2[1];
        const double cy = (double)l->e1[2] * l->e2[0] - (double)l->e1[0] * l->e2[2];
        const double cz = (double)l->e1[0] * l->e2[1] - (double)l->e1[1] * l->e2[0];
        if (!(cx * cx + cy * cy + cz * cz > 0.0) || !finite3(l->corner))
            return fail(LF_E_ARG, "area light edges must span a parallelogram");
    } else {
        return fail(LF_E_ARG, "unknown light kind %d", l->kind);
    }
    return LF_OK;
}

void pack_trace(lp::TraceParams& T, const lf_volume* v, const lf_medium* e, const lf_medium* s,
                const lf_light* l, const lf_gen_params* p) {
    std::memset(&T, 0, sizeof(T));
    T.waves = p->waves_per_simd == 3 ? 3 : 4;
    T.vol = v->data;  // replaced by the workspace's halo-brick copy
    T.nx = v->nx;
    T.ny = v->ny;
    T.brick_row = 64 * lp::halo_bricks(v->nx);
    T.brick_slab = 64 * lp::halo_bricks(v->nx) * lp::halo_bricks(v->ny);
    const int n[3] = {v->nx, v->ny, v->nz};
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)v->box_max[a] - (double)v->box_min[a];
        T.ga[a] = (float)(n[a] / ext);
        T.gb[a] = (float)(-(double)v->box_min[a] * n[a] / ext - 0.5);
        T.gmax[a] = (float)(n[a] - 1);
        T.imax[a] = n[a] - 2;
        T.bmin[a] = v->box_min[a];
        T.bmax[a] = v->box_max[a];
    }
    T.vmin = v->vmin;
    T.vscale = (float)(1.0 / ((double)v->vmax - (double)v->vmin));
    T.lut_n = e->lut_size;
    T.lut_last = (float)(e->lut_size - 1);
    T.lut_e = e->lut;
    T.lut_s = s ? s->lut : e->lut;
    T.scale_e = e->density_scale;
    T.scale_s = s ? s->density_scale : e->density_scale;
    T.light_kind = l->kind;
    T.light_on = l->radiance[0] != 0.0f || l->radiance[1] != 0.0f || l->radiance[2] != 0.0f;
    for (int a = 0; a < 3; ++a) {
        T.ldir[a] = l->dir[a];
        T.lcorner[a] = l->corner[a];
        T.le1[a] = l->e1[a];
        T.le2[a] = l->e2[a];
        T.lrad[a] = l->radiance[a];
        T.env[a] = l->env[a];
        T.O[a] = p->center[a];
    }
    if (l->kind == LF_LIGHT_DIRECTIONAL) {
        const double nn = std::sqrt((double)l->dir[0] * l->dir[0] + (double)l->dir[1] * l->dir[1] +
                                    (double)l->dir[2] * l->dir[2]);
        for (int a = 0; a < 3; ++a) T.ldir[a] = (float)(l->dir[a] / nn);
    } else {
        const double c[3] = {(double)l->e1[1] * l->e2[2] - (double)l->e1[2] * l->e2[1],
                             (double)l->e1[2] * l->e2[0] - (double)l->e1[0] * l->e2[2],
                             (double)l->e1[0] * l->e2[1] - (double)l->e1[1] * l->e2[0]};
        const double area = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int a = 0; a < 3; ++a) T.lnrm[a] = (float)(c[a] / area);
        T.larea = (float)area;
    }
    T.M = p->M;
    T.N = p->N;
    T.R = p->radius;
    T.spp = p->spp;
    T.maxb = p->max_bounces;
    T.g = p->hg_g;
    T.key0 = (uint32_t)p->seed;
    T.key1 = (uint32_t)(p->seed >> 32);
    T.jitter = p->jitter != 0;
    T.jit_rad = (float)(2.0 * p->radius / std::sqrt((double)p->M));
    T.row_begin = (int32_t)p->row_begin;
    T.row_end = (int32_t)(p->row_end <= 0 ? stored_rows(p) : p->row_end);
    T.stats = (unsigned long long*)p->stats;
    T.srad = p->sample_radiance;
    const int G = grid_cells(p);
    T.grid_n = G > 0 ? G : 1;
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)v->box_max[a] - (double)v->box_min[a];
        T.gcell[a] = (float)(T.grid_n / ext);
        T.gcw[a] = (float)(ext / T.grid_n);
    }
    T.nz = v->nz;
    T.surface = p->surface;
    T.iso = p->iso;
    double hv = 1e300;
    for (int a = 0; a < 3; ++a) hv = std::min(hv, ((double)v->box_max[a] - (double)v->box_min[a]) / n[a]);
    T.half_voxel = (float)(0.5 * hv);
}

// Isosurface variant: cells of the raw-range grid (the majorant grid size,
// 8 when none is set) and their bytes in the workspace.
int surface_cells(const lf_gen_params* p) { return p->majorant_grid > 0 ? p->majorant_grid : 8; }
size_t surface_range_bytes(const lf_gen_params* p) {
    if (!p->surface) return 0;
    const size_t G = (size_t)surface_cells(p);
    return align256(8 * G * G * G);
}

// Set-up and launch of the isosurface variant; `range` is its workspace.
hipError_t run_surface(lp::TraceParams& T, const lf_volume* vol, const lf_medium* m, const lf_gen_params* p,
                       char* w, float* range, hipStream_t s) {
    float* sig = (float*)w;
    unsigned int* ctr = (unsigned int*)(w + 64);
    int32_t* perm_o = (int32_t*)(w + 256);
    int32_t* perm_d = (int32_t*)(w + 256 + align256(4 * (size_t)(T.row_end - T.row_begin)));
    T.sigbar = sig;
    T.tile_ctr = ctr;
    T.perm_o = perm_o;
    T.perm_d = perm_d;
    const int G = surface_cells(p);
    T.grid_n = G;
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)vol->box_max[a] - (double)vol->box_min[a];
        T.gcell[a] = (float)(G / ext);
        T.gcw[a] = (float)(ext / G);
    }
    T.srange = range;
    hipError_t e = lp::launch_wave_setup(T, m->lut, m->lut_size, m->density_scale, p->majorant, sig, ctr, perm_o,
                                         perm_d, s);
    if (e == hipSuccess)
        e = lp::launch_majorant_grid(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, G, m->lut,
                                     m->lut_size, m->density_scale, vol->vmin, vol->vmax, nullptr, range, s);
    if (e == hipSuccess) e = lp::launch_surface(T, vol->type, s);
    return e;
}

// Majorant set-up shared by both entry points: the global majorant, the tile
// counters and spatial orders, then (with a grid) the cell majorants; without
// a grid the one cell's majorant is the global one.
hipError_t setup_tracking(lp::TraceParams& T, const lf_volume* vol, const lf_medium* sm, const lf_gen_params* p,
                          char* w, hipStream_t s) {
    float* sig = (float*)w;
    unsigned int* ctr = (unsigned int*)(w + 64);
    int32_t* perm_o = (int32_t*)(w + 256);
    int32_t* perm_d = (int32_t*)(w + 256 + align256(4 * (size_t)(T.row_end - T.row_begin)));
    T.sigbar = sig;
    T.tile_ctr = ctr;
    T.perm_o = perm_o;
    T.perm_d = perm_d;
    T.maj = sig;
    float4* tab_o = (float4*)(w + gen_perm_bytes(p) + gen_grid_bytes(p));
    float4* tab_d = (float4*)((char*)tab_o + align256(16 * (size_t)p->M));
    T.tab_o = tab_o;
    T.tab_d = tab_d;
    hipError_t e = lp::launch_wave_setup(T, sm->lut, sm->lut_size, sm->density_scale, p->majorant, sig, ctr,
                                         perm_o, perm_d, s);
    if (e == hipSuccess) e = lp::launch_sf_table(p->M, 1.0f / (float)p->M, tab_o, s);
    if (e == hipSuccess) e = lp::launch_sf_table(p->N, 1.0f / (float)p->N, tab_d, s);
    if (e == hipSuccess && grid_cells(p) > 0) {
        float* cells = (float*)(w + gen_perm_bytes(p));
        T.maj = cells;
        e = lp::launch_majorant_grid(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, T.grid_n, sm->lut,
                                     sm->lut_size, sm->density_scale, vol->vmin, vol->vmax, cells, nullptr, s);
    }
    return e;
}

int check_workspace(void* ws, size_t* ws_bytes, size_t need) {
    if (!ws_bytes) return fail(LF_E_ARG, "ws_bytes is NULL");
    if (!ws) return 1;  // size query
    if (*ws_bytes < need)
        return fail(LF_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", *ws_bytes, need);
    if ((uintptr_t)ws % 16) return fail(LF_E_WORKSPACE, "workspace must be 16-byte aligned");
    return LF_OK;
}

}  // namespace

extern "C" {

const char* lf_last_error(void) { return g_err.c_str(); }

int lf_version(void) { return LUMIPATH_VERSION; }

int lf_points(int32_t n, float* xyz_out, const float* query, int64_t nq, int32_t K, int32_t* idx_out,
              float* w_out, void* stream) {
    g_err.clear();
    if (n < 1 || n > 65535) return fail(LF_E_ARG, "n must be in [1, 65535] (got %d)", n);
    if (!xyz_out && !query) return fail(LF_E_ARG, "nothing to do: xyz_out and query are NULL");
    if (query) {
        if (nq < 0) return fail(LF_E_ARG, "nq must be >= 0");
        if (K < 1 || K > 9) return fail(LF_E_ARG, "K must be in [1, 9] (got %d)", K);
        if (!idx_out) return fail(LF_E_ARG, "idx_out is NULL");
        if (nq > (1ll << 40)) return fail(LF_E_RANGE, "too many queries");
    }
    hipError_t e = lp::launch_points(n, xyz_out, query, query ? nq : 0, K, idx_out, w_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lf_points");
    return LF_OK;
}

int lf_generate(const lf_volume* vol, const lf_medium* eval, const lf_medium* sample, const lf_light* light,
                const lf_gen_params* params, int32_t dtype, void* lf_out, void* ws, size_t* ws_bytes,
                void* stream) {
    g_err.clear();
    int r;
    if ((r = check_volume(vol)) || (r = check_medium(eval, "eval")) || (r = check_light(light)) ||
        (r = check_params(params, true)))
        return r;
    if (sample) {
        if ((r = check_medium(sample, "sample"))) return r;
        if (sample->lut_size != eval->lut_size) return fail(LF_E_ARG, "sample and eval LUT sizes differ");
    }
    if (dtype < LF_F32 || dtype > LF_BF16) return fail(LF_E_ARG, "unknown light-field dtype %d", dtype);
    if (!lf_out) return fail(LF_E_ARG, "lf_out is NULL");
    if (params->surface && sample && sample != eval)
        return fail(LF_E_UNSUPPORTED, "frozen sampling does not apply to the isosurface variant");
    const size_t need =
        gen_order_bytes(params) + brick_copy_bytes(vol) + surface_range_bytes(params) + part_sums_bytes(params);
    r = check_workspace(ws, ws_bytes, need);
    if (r == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (r) return r;
    lp::TraceParams T;
    pack_trace(T, vol, eval, sample, light, params);
    T.out = lf_out;
    T.dtype = dtype;
    char* w = (char*)ws;
    T.vol = w + gen_order_bytes(params);
    const lf_medium* sm = sample ? sample : eval;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = lp::launch_halo_bricks(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, (void*)T.vol, s);
    if (params->surface) {
        if (e == hipSuccess)
            e = run_surface(T, vol, eval, params, w, (float*)(w + gen_order_bytes(params) + brick_copy_bytes(vol)), s);
        if (e != hipSuccess) return hip_fail(e, "lf_generate (isosurface)");
        return LF_OK;
    }
    if (e == hipSuccess) e = setup_tracking(T, vol, sm, params, w, s);
    if (e != hipSuccess) return hip_fail(e, "lf_generate (set-up)");
    const int mode = (sample && sample != eval) ? lp::kFrozen : lp::kFwd;
    T.part_log2 = part_log2(params, true);
    T.part_sums = (float*)(w + gen_order_bytes(params) + brick_copy_bytes(vol) + surface_range_bytes(params));
    e = lp::launch_generate_wave(T, vol->type, mode, s);
    if (e == hipSuccess && T.part_log2 > 0) e = lp::launch_combine_parts(T, s);
    if (e != hipSuccess) return hip_fail(e, "lf_generate");
    return LF_OK;
}

int lf_render_views(const lf_volume* vol, const lf_medium* medium, const lf_light* light,
                    const lf_gen_params* params, const lf_camera* cams, int32_t n_views, int32_t W, int32_t H,
                    float* img, void* ws, size_t* ws_bytes, void* stream) {
    g_err.clear();
    int r;
    if ((r = check_volume(vol)) || (r = check_medium(medium, "")) || (r = check_light(light))) return r;
    if (!params) return fail(LF_E_ARG, "params is NULL");
    if (params->spp < 1) return fail(LF_E_ARG, "spp must be >= 1");
    if (params->max_bounces < 1 || params->max_bounces > 65535)
        return fail(LF_E_ARG, "max_bounces must be in [1, 65535]");
    if (!(std::fabs(params->hg_g) < 1.0f)) return fail(LF_E_ARG, "|hg_g| must be < 1");
    if (!std::isfinite(params->majorant)) return fail(LF_E_ARG, "majorant must be finite");
    if (params->majorant_grid < 0 || params->majorant_grid > 16)
        return fail(LF_E_ARG, "majorant_grid must be in [0, 16] (got %d)", params->majorant_grid);
    if (params->surface != 0 && params->surface != 1) return fail(LF_E_ARG, "surface must be 0 or 1");
    if (!std::isfinite(params->iso)) return fail(LF_E_ARG, "iso must be finite");
    if (!cams) return fail(LF_E_ARG, "cams is NULL");
    if (n_views < 1 || W < 1 || H < 1) return fail(LF_E_ARG, "n_views, W and H must be >= 1");
    if ((unsigned long long)n_views * (unsigned long long)W * (unsigned long long)H >= (1ull << 32))
        return fail(LF_E_RANGE, "n_views * W * H must be < 2^32");
    if (!img) return fail(LF_E_ARG, "img is NULL");
    std::vector<lp::ViewCam> vc((size_t)n_views);
    for (int v = 0; v < n_views; ++v) {
        const lf_camera& c = cams[v];
        double f[3], u[3], rt[3], up[3];
        for (int a = 0; a < 3; ++a) {
            f[a] = (double)c.target[a] - c.eye[a];
            u[a] = c.up[a];
        }
        const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (!(c.vfov > 0.0f && c.vfov < 3.14159f) || !(fl > 0.0) || !finite3(c.eye))
            return fail(LF_E_ARG, "camera %d: bad eye, field of view or target", v);
        for (int a = 0; a < 3; ++a) f[a] /= fl;
        rt[0] = f[1] * u[2] - f[2] * u[1];
        rt[1] = f[2] * u[0] - f[0] * u[2];
        rt[2] = f[0] * u[1] - f[1] * u[0];
        const double rl = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
        if (!(rl > 1e-9)) return fail(LF_E_ARG, "camera %d: up is parallel to the view direction", v);
        for (int a = 0; a < 3; ++a) rt[a] /= rl;
        up[0] = rt[1] * f[2] - rt[2] * f[1];
        up[1] = rt[2] * f[0] - rt[0] * f[2];
        up[2] = rt[0] * f[1] - rt[1] * f[0];
        const double th = std::tan(0.5 * c.vfov);
        lp::ViewCam& g = vc[v];
        for (int a = 0; a < 3; ++a) {
            g.eye[a] = c.eye[a];
            g.fwd[a] = (float)f[a];
            g.right[a] = (float)rt[a];
            g.up[a] = (float)up[a];
        }
        g.sx = (float)(th * (double)W / (double)H);
        g.sy = (float)th;
    }
    // the tracer set-up of lf_generate with a one-point ray set, then the views
    lf_gen_params p1 = *params;
    p1.M = p1.N = 1;
    p1.sample_radiance = nullptr;
    p1.origin_rows = 0;
    p1.row_begin = 0;
    p1.row_end = 1;
    p1.jitter = 0;
    const size_t views_bytes = align256(sizeof(lp::ViewCam) * (size_t)n_views);
    const unsigned long long pixels = (unsigned long long)n_views * (unsigned long long)W * (unsigned long long)H;
    const int vpl = p1.surface ? 0 : view_part_log2(p1.spp, pixels);
    const size_t psum_bytes = vpl ? align256((size_t)(12 * pixels) << vpl) : 0;
    const size_t need =
        gen_order_bytes(&p1) + views_bytes + brick_copy_bytes(vol) + surface_range_bytes(&p1) + psum_bytes;
    r = check_workspace(ws, ws_bytes, need);
    if (r == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (r) return r;
    lp::TraceParams T;
    pack_trace(T, vol, medium, nullptr, light, &p1);
    T.out = img;
    T.dtype = LF_F32;
    char* w = (char*)ws;
    lp::ViewCam* dv = (lp::ViewCam*)(w + gen_order_bytes(&p1));
    T.vol = w + gen_order_bytes(&p1) + views_bytes;
    T.views = dv;
    T.nviews = n_views;
    T.W = W;
    T.H = H;
    T.vtx = (W + 7) / 8;
    T.vtiles = T.vtx * ((H + 7) / 8);
    hipStream_t s = (hipStream_t)stream;
    // the views travel as kernel arguments into the workspace (stream-ordered;
    // no host buffer has to outlive the call)
    hipError_t e = hipSuccess;
    for (int v0 = 0; v0 < n_views && e == hipSuccess; v0 += lp::kViewBatch) {
        lp::ViewBatch vb;
        vb.first = v0;
        vb.count = std::min(lp::kViewBatch, n_views - v0);
        for (int v = 0; v < vb.count; ++v) vb.v[v] = vc[v0 + v];
        e = lp::launch_fill_views(vb, dv, s);
    }
    if (e == hipSuccess)
        e = lp::launch_halo_bricks(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, (void*)T.vol, s);
    if (p1.surface) {
        if (e == hipSuccess)
            e = run_surface(T, vol, medium, &p1, w,
                            (float*)(w + gen_order_bytes(&p1) + views_bytes + brick_copy_bytes(vol)), s);
    } else {
        if (e == hipSuccess) e = setup_tracking(T, vol, medium, &p1, w, s);
        T.part_log2 = vpl;
        T.part_sums = (float*)(w + gen_order_bytes(&p1) + views_bytes + brick_copy_bytes(vol) + surface_range_bytes(&p1));
        if (e == hipSuccess) e = lp::launch_generate_wave(T, vol->type, lp::kFwd, s);
        if (e == hipSuccess && vpl > 0) e = lp::launch_combine_parts(T, s);
    }
    if (e != hipSuccess) return hip_fail(e, "lf_render_views");
    return LF_OK;
}

int lf_ssim(const float* a, const float* b, int32_t n_images, int32_t W, int32_t H, float data_range, double* out,
            void* ws, size_t* ws_bytes, void* stream) {
    g_err.clear();
    if (!a || !b || !out) return fail(LF_E_ARG, "a, b and out must be non-NULL");
    if (n_images < 1 || n_images > 21845) return fail(LF_E_ARG, "n_images must be in [1, 21845]");
    if (W < 11 || H < 11) return fail(LF_E_ARG, "images must be at least 11 x 11 (the window)");
    if ((long long)W * H > (1ll << 30)) return fail(LF_E_RANGE, "image too large");
    if (!(data_range > 0.0f) || !std::isfinite(data_range)) return fail(LF_E_ARG, "data_range must be > 0");
    const size_t need = align256(sizeof(double) * lp::ssim_partial_count(n_images, W, H));
    int r = check_workspace(ws, ws_bytes, need);
    if (r == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (r) return r;
    lp::SsimParams P;
    P.a = a;
    P.b = b;
    P.W = W;
    P.H = H;
    double g[11], sum = 0.0;
    for (int t = 0; t < 11; ++t) {
        g[t] = std::exp(-(double)((t - 5) * (t - 5)) / (2.0 * 1.5 * 1.5));
        sum += g[t];
    }
    for (int t = 0; t < 11; ++t) P.w[t] = (float)(g[t] / sum);
    P.c1 = (float)((0.01 * data_range) * (0.01 * data_range));
    P.c2 = (float)((0.03 * data_range) * (0.03 * data_range));
    P.partial = (double*)ws;
    P.out = out;
    hipError_t e = lp::launch_ssim(P, n_images, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lf_ssim");
    return LF_OK;
}

int lf_cw_ssim(const float* a, const float* b, int32_t n_images, int32_t W, int32_t H, float data_range,
               double* out, void* ws, size_t* ws_bytes, void* stream) {
    g_err.clear();
    if (!a || !b || !out) return fail(LF_E_ARG, "a, b and out must be non-NULL");
    if (n_images < 1) return fail(LF_E_ARG, "n_images must be >= 1");
    if (W < 7 || H < 7) return fail(LF_E_ARG, "images must be at least 7 x 7 (the window)");
    if (W > 4096 || H > 4096) return fail(LF_E_RANGE, "W and H must be <= 4096");
    if (!(data_range >= 0.0f) || !std::isfinite(data_range)) return fail(LF_E_ARG, "data_range must be >= 0");
    const size_t plane = align256(sizeof(float2) * (size_t)W * (size_t)H * 6);
    const size_t tw_w = align256(sizeof(float2) * (size_t)W), tw_h = align256(sizeof(float2) * (size_t)H);
    const size_t need = tw_w + tw_h + 3 * plane + align256(sizeof(double) * lp::cw_ssim_slots(W, H));
    int r = check_workspace(ws, ws_bytes, need);
    if (r == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (r) return r;
    char* w = (char*)ws;
    lp::CwParams P;
    P.a = a;
    P.b = b;
    P.W = W;
    P.H = H;
    P.K = (float)(49.0 * (0.01 * data_range) * (0.01 * data_range));
    P.tw_w = (float2*)w;
    P.tw_h = (float2*)(w + tw_w);
    P.spec = (float2*)(w + tw_w + tw_h);
    P.t1 = (float2*)(w + tw_w + tw_h + plane);
    P.t2 = (float2*)(w + tw_w + tw_h + 2 * plane);
    P.slots = (double*)(w + tw_w + tw_h + 3 * plane);
    P.out = out;
    hipError_t e = lp::launch_cw_ssim(P, n_images, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lf_cw_ssim");
    return LF_OK;
}

int lf_majorant_grid(const lf_volume* vol, const lf_medium* sample, const lf_gen_params* params, float* out,
                     void* stream) {
    g_err.clear();
    int r;
    if ((r = check_volume(vol)) || (r = check_medium(sample, "sample")) || (r = check_params(params, true))) return r;
    if (!out) return fail(LF_E_ARG, "out is NULL");
    const int G = params->majorant_grid;
    if (G < 1) return fail(LF_E_ARG, "majorant_grid must be >= 1 for lf_majorant_grid");
    hipError_t e = lp::launch_majorant_grid(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, G,
                                            sample->lut, sample->lut_size, sample->density_scale, vol->vmin,
                                            vol->vmax, out, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lf_majorant_grid");
    return LF_OK;
}

int lf_generate_backward(const lf_volume* vol, const lf_medium* medium, const lf_light* light,
                         const lf_gen_params* params, const float* d_lf, float* d_lut, float* d_scale, void* ws,
                         size_t* ws_bytes, void* stream) {
    g_err.clear();
    int r;
    if ((r = check_volume(vol)) || (r = check_medium(medium, "")) || (r = check_light(light)) ||
        (r = check_params(params, true)))
        return r;
    if (!d_lf || !d_lut || !d_scale) return fail(LF_E_ARG, "d_lf, d_lut and d_scale must be non-NULL");
    if (params->surface) return fail(LF_E_UNSUPPORTED, "the adjoint does not apply to the isosurface variant");
    // majorant, counters, spatial orders, list of rays with a nonzero adjoint,
    // then the brick copy of the volume
    const long long re = params->row_end <= 0 ? stored_rows(params) : params->row_end;
    const size_t list_bytes = align256(4 * (size_t)(re - params->row_begin) * (size_t)params->N);
    const size_t need = gen_order_bytes(params) + list_bytes + brick_copy_bytes(vol);
    r = check_workspace(ws, ws_bytes, need);
    if (r == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (r) return r;
    lp::TraceParams T;
    pack_trace(T, vol, medium, nullptr, light, params);
    T.d_lf = d_lf;
    T.d_lut = d_lut;
    T.d_scale = d_scale;
    T.part_log2 = part_log2(params, false);
    T.stats = nullptr;
    char* w = (char*)ws;
    T.ray_count = (unsigned int*)(w + 64) + 8;
    T.ray_list = (uint32_t*)(w + gen_order_bytes(params));
    T.vol = w + gen_order_bytes(params) + list_bytes;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = lp::launch_halo_bricks(vol->data, vol->type, vol->brick, vol->nx, vol->ny, vol->nz, (void*)T.vol, s);
    if (e == hipSuccess) e = lp::launch_zero(d_lut, 4ll * medium->lut_size, s);
    if (e == hipSuccess) e = lp::launch_zero(d_scale, 1, s);
    if (e == hipSuccess) e = setup_tracking(T, vol, medium, params, w, s);
    if (e == hipSuccess) e = lp::launch_active_rays(T, s);
    if (e == hipSuccess) e = lp::launch_generate_wave(T, vol->type, lp::kGrad, s);
    if (e != hipSuccess) return hip_fail(e, "lf_generate_backward");
    return LF_OK;
}

// lf_lookup and lf_lookup_l2: mode 0 forward, 1 adjoint, 2 fused L2 (views,
// their loss gradient against `target`, and its adjoint).
static int run_lookup(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams,
                      int32_t n_views, int32_t W, int32_t H, int32_t K, int32_t mode, float* img, const float* target,
                      float* d_lf, int32_t* nn_out, void* ws, size_t* ws_bytes, void* stream) {
    int r;
    if ((r = check_params(params, false))) return r;
    if (!cams) return fail(LF_E_ARG, "cams is NULL");
    if (n_views < 1 || W < 1 || H < 1) return fail(LF_E_ARG, "n_views, W and H must be >= 1");
    if ((long long)W * H > (1ll << 30) || (long long)n_views * W * H > (1ll << 40))
        return fail(LF_E_RANGE, "image too large");
    if (K < 1 || K > 9) return fail(LF_E_ARG, "K must be in [1, 9] (got %d)", K);
    if (dtype < LF_F32 || dtype > LF_BF16) return fail(LF_E_ARG, "unknown light-field dtype %d", dtype);
    if (!img) return fail(LF_E_ARG, "img is NULL");
    if (mode != LF_LOOKUP_ADJOINT && !lf) return fail(LF_E_ARG, "lf is NULL");
    if (mode != LF_LOOKUP_FORWARD && !d_lf) return fail(LF_E_ARG, "d_lf is NULL");
    if (mode == 2 && !target) return fail(LF_E_ARG, "target is NULL");
    // workspace: the point tables of both SF sets, then their zone bases
    const size_t tab_o_bytes = align256(16 * (size_t)params->M);
    const size_t tab_d_bytes = align256(16 * (size_t)params->N);
    const size_t need = tab_o_bytes + tab_d_bytes + 2 * lp::kZoneTableBytes;
    int rw = check_workspace(ws, ws_bytes, need);
    if (rw == 1) {
        *ws_bytes = need;
        return LF_OK;
    }
    if (rw) return rw;
    const double R = params->radius;
    lp::LookupParams L;
    std::memset(&L, 0, sizeof(L));
    L.M = params->M;
    L.N = params->N;
    L.invM = (float)(1.0 / params->M);
    L.invN = (float)(1.0 / params->N);
    L.inv_rM = (float)(1.0 / std::sqrt(4.0 * M_PI / params->M));
    L.inv_rN = (float)(1.0 / std::sqrt(4.0 * M_PI / params->N));
    L.W = W;
    L.H = H;
    L.K = K;
    L.dtype = dtype;
    L.degenerate = params->M == params->N;
    L.orows = (int32_t)stored_rows(params);
    L.thr = (float)(1e-6 * R * R);
    L.lf = lf;
    L.img = img;
    L.d_lf = d_lf;
    L.target = target;
    L.nn = mode == LF_LOOKUP_FORWARD ? nn_out : nullptr;
    L.tab_o = (const float4*)ws;
    L.tab_d = (const float4*)((char*)ws + tab_o_bytes);
    L.zone_o = (const lp::SfZone*)((char*)ws + tab_o_bytes + tab_d_bytes);
    L.zone_d = (const lp::SfZone*)((char*)ws + tab_o_bytes + tab_d_bytes + lp::kZoneTableBytes);
    // per-view geometry in double, rounded once to float
    std::vector<lp::ViewGeom> geo((size_t)n_views);
    for (int v = 0; v < n_views; ++v) {
        const lf_camera& c = cams[v];
        double oc[3], f[3], u[3], rt[3], up[3];
        for (int a = 0; a < 3; ++a) {
            oc[a] = (double)c.eye[a] - params->center[a];
            f[a] = (double)c.target[a] - c.eye[a];
            u[a] = c.up[a];
        }
        const double occ = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2];
        const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (!(occ > R * R)) {
            return fail(LF_E_ARG, "camera %d: eye is inside the bounding sphere", v);
        }
        if (!(c.vfov > 0.0f && c.vfov < 3.14159f) || !(fl > 0.0)) {
            return fail(LF_E_ARG, "camera %d: bad field of view or target", v);
        }
        for (int a = 0; a < 3; ++a) f[a] /= fl;
        rt[0] = f[1] * u[2] - f[2] * u[1];
        rt[1] = f[2] * u[0] - f[0] * u[2];
        rt[2] = f[0] * u[1] - f[1] * u[0];
        const double rl = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
        if (!(rl > 1e-9)) {
            return fail(LF_E_ARG, "camera %d: up is parallel to the view direction", v);
        }
        for (int a = 0; a < 3; ++a) rt[a] /= rl;
        up[0] = rt[1] * f[2] - rt[2] * f[1];
        up[1] = rt[2] * f[0] - rt[0] * f[2];
        up[2] = rt[0] * f[1] - rt[1] * f[0];
        const double th = std::tan(0.5 * c.vfov);
        lp::ViewGeom& g = geo[v];
        for (int a = 0; a < 3; ++a) {
            g.oc[a] = (float)oc[a];
            g.fwd[a] = (float)f[a];
            g.right[a] = (float)rt[a];
            g.up[a] = (float)up[a];
        }
        g.c = (float)(occ - R * R);
        g.sx = (float)(th * (double)W / (double)H);
        g.sy = (float)th;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t et = lp::launch_sf_tables(L, s);
    if (et != hipSuccess) return hip_fail(et, "lf_lookup (point tables)");
    for (int v0 = 0; v0 < n_views; v0 += lp::kMaxViewsPerLaunch) {
        const int nv = std::min(lp::kMaxViewsPerLaunch, n_views - v0);
        L.view0 = v0;
        L.nviews = nv;
        for (int v = 0; v < nv; ++v) L.v[v] = geo[v0 + v];
        hipError_t e = lp::launch_lookup(L, mode, s);
        if (e != hipSuccess) return hip_fail(e, "lf_lookup");
    }
    return LF_OK;
}

int lf_lookup(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams, int32_t n_views,
              int32_t W, int32_t H, int32_t K, int32_t mode, float* img, float* d_lf, int32_t* nn_out, void* ws,
              size_t* ws_bytes, void* stream) {
    g_err.clear();
    if (mode != LF_LOOKUP_FORWARD && mode != LF_LOOKUP_ADJOINT) return fail(LF_E_ARG, "unknown mode %d", mode);
    return run_lookup(lf, dtype, params, cams, n_views, W, H, K, mode, img, nullptr, d_lf, nn_out, ws, ws_bytes,
                      stream);
}

int lf_lookup_static(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams,
                     int32_t n_views, int32_t W, int32_t H, int32_t K, int32_t mode, float* img, float* d_lf,
                     int32_t* nn_out, void* stream) {
    g_err.clear();
    if (mode != LF_LOOKUP_FORWARD && mode != LF_LOOKUP_ADJOINT) return fail(LF_E_ARG, "unknown mode %d", mode);
    int r;
    if ((r = check_params(params, false))) return r;
    const size_t need = align256(16 * (size_t)params->M) + align256(16 * (size_t)params->N) + 2 * lp::kZoneTableBytes;
    if (need > lp::kLookupScratchBytes)
        return fail(LF_E_RANGE, "lf_lookup_static: the point tables need %zu bytes, above its fixed scratch of %zu",
                    need, lp::kLookupScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "lf_lookup_static (current device)");
    if (stream) {
        hipDevice_t sdev = 0;
        e = hipStreamGetDevice((hipStream_t)stream, &sdev);
        if (e != hipSuccess) return hip_fail(e, "lf_lookup_static (stream device)");
        if ((int)sdev != dev)
            return fail(LF_E_ARG, "lf_lookup_static: the stream belongs to device %d, device %d is current",
                        (int)sdev, dev);
    }
    void* ws = nullptr;
    e = lp::lookup_scratch(dev, &ws);
    if (e != hipSuccess) return hip_fail(e, "lf_lookup_static (scratch address)");
    size_t ws_bytes = lp::kLookupScratchBytes;
    return run_lookup(lf, dtype, params, cams, n_views, W, H, K, mode, img, nullptr, d_lf, nn_out, ws, &ws_bytes,
                      stream);
}

int lf_lookup_l2(const void* lf, int32_t dtype, const lf_gen_params* params, const lf_camera* cams, int32_t n_views,
                 int32_t W, int32_t H, int32_t K, const float* target, float* img, float* d_lf, void* ws,
                 size_t* ws_bytes, void* stream) {
    g_err.clear();
    return run_lookup(lf, dtype, params, cams, n_views, W, H, K, 2, img, target, d_lf, nullptr, ws, ws_bytes, stream);
}

}  // extern "C"
