// Host side of the C ABI declared in include/perf_gn.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "perf_internal.h"

using namespace perf;

struct perf_scene {
    perf_scene_desc desc;
    int n_cams;
    Geo geo;
    Layout lay;
    char* ws;
    const float* targets;
    hipStream_t stream;
    int64_t n_rays, units, P;
    int n_ray_blocks;
    DevCam* cams;
    double* partials;
    double* scalars;
    double* hist;
    int* iflags;
    float *vr, *vz, *vp, *vAp, *vdelta, *vxt, *blocks, *minv, *feat;
    uint16_t *xb16, *mlpw;
    float* mlpnorm;
    float q_fallback;
    bool mlp_ready;
    double host_scalars[S_COUNT];
    double host_hist[4 * PERF_MAX_PCG];
    int host_flags[I_COUNT];
};

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define CK(expr)                                                                                   \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(PERF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool finite_f(float v) { return isfinite(v); }

int32_t validate(const perf_scene_desc* d, int n_cams) {
    if (!d) return fail(PERF_EINVAL, "null descriptor");
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return fail(PERF_EINVAL, "grid dims must be >= 2");
    if (d->n_layers < 0 || d->n_layers > PERF_MAX_LAYERS) return fail(PERF_EINVAL, "n_layers must be in 0..8");
    if (d->n_layers > 0 && (d->env_w < 2 || d->env_h < 2)) return fail(PERF_EINVAL, "env_w and env_h must be >= 2");
    if (!(d->step_vox > 0.0f && d->step_vox <= 1.0f)) return fail(PERF_EINVAL, "step_vox must be in (0, 1]");
    if (d->param_dtype != PERF_F32 && d->param_dtype != PERF_BF16) return fail(PERF_EINVAL, "bad param_dtype");
    if (d->width < 1 || d->height < 1) return fail(PERF_EINVAL, "image size must be positive");
    if (!finite_f(d->aux_lambda) || d->aux_lambda < 0.0f) return fail(PERF_EINVAL, "aux_lambda must be >= 0");
    if (!(d->render_threshold >= 0.0f && d->render_threshold <= 1.0f))
        return fail(PERF_EINVAL, "render_threshold must be in [0, 1]");
    if (n_cams < 1) return fail(PERF_EINVAL, "need at least one camera");
    double corner = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!finite_f(d->bbox_min[a]) || !finite_f(d->bbox_max[a]) || !(d->bbox_max[a] > d->bbox_min[a]))
            return fail(PERF_EINVAL, "bad bounding box");
        const double m = fmax(fabs(d->bbox_min[a]), fabs(d->bbox_max[a]));
        corner += m * m;
    }
    corner = sqrt(corner);
    float prev = 0.0f;
    for (int l = 0; l < d->n_layers; ++l) {
        const float R = d->layer_radius[l];
        if (!finite_f(R) || !(R > corner)) return fail(PERF_EINVAL, "layer %d radius must exceed the box corner distance", l);
        if (l > 0 && !(R > prev)) return fail(PERF_EINVAL, "layer radii must increase");
        prev = R;
    }
    const int64_t units = (int64_t)d->nx * d->ny * d->nz + (int64_t)d->n_layers * d->env_w * d->env_h;
    if (units * 10 >= (int64_t)1 << 31) return fail(PERF_EUNSUPPORTED, "too many parameters for 32-bit indexing");
    return PERF_OK;
}

}  // namespace

namespace perf {

Geo make_geo(const perf_scene_desc& d, int n_cams) {
    Geo g{};
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.n_layers = d.n_layers;
    g.env_w = d.env_w;
    g.env_h = d.env_h;
    g.width = d.width;
    g.height = d.height;
    g.n_cams = n_cams;
    g.tiles_x = (d.width + kTileX - 1) / kTileX;
    g.tiles_y = (d.height + kTileY - 1) / kTileY;
    g.n_tiles = g.tiles_x * g.tiles_y;
    const int n[3] = {d.nx, d.ny, d.nz};
    float h = INFINITY;
    for (int a = 0; a < 3; ++a) {
        g.bmin[a] = d.bbox_min[a];
        g.bmax[a] = d.bbox_max[a];
        const float hv = (d.bbox_max[a] - d.bbox_min[a]) / (float)n[a];
        g.inv_hv[a] = (float)n[a] / (d.bbox_max[a] - d.bbox_min[a]);
        h = fminf(h, hv);
        g.bg[a] = d.background[a];
    }
    g.h = h;
    g.step = d.step_vox;
    for (int l = 0; l < kMaxLayers; ++l) g.radius[l] = l < d.n_layers ? d.layer_radius[l] : 0.0f;
    g.nvox = d.nx * d.ny * d.nz;
    return g;
}

Layout make_layout(const perf_scene_desc& d, int n_cams) {
    Layout L{};
    const int64_t units = (int64_t)d.nx * d.ny * d.nz + (int64_t)d.n_layers * d.env_w * d.env_h;
    const int64_t P = 4 * units;
    const Geo g = make_geo(d, n_cams);
    const int64_t ray_blocks = (int64_t)n_cams * g.n_tiles;
    L.n_partials = ray_blocks > 2 * kVecGrid ? ray_blocks : 2 * kVecGrid;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.cams = take(sizeof(DevCam) * (size_t)n_cams);
    L.partials = take(sizeof(double) * (size_t)L.n_partials);
    L.scalars = take(sizeof(double) * S_COUNT);
    L.hist = take(sizeof(double) * 4 * PERF_MAX_PCG);
    L.iflags = take(sizeof(int) * I_COUNT);
    L.vr = take(sizeof(float) * (size_t)P);
    L.vz = take(sizeof(float) * (size_t)P);
    L.vp = take(sizeof(float) * (size_t)P);
    L.vAp = take(sizeof(float) * (size_t)P);
    L.vdelta = take(sizeof(float) * (size_t)P);
    L.vxt = take(sizeof(float) * (size_t)P);
    L.blocks = take(sizeof(float) * 5 * (size_t)units);
    L.minv = take(sizeof(float) * 12 * (size_t)units);  // the largest scaled form (learned: 12 per unit)
    L.xb16 = d.param_dtype == PERF_BF16 ? take(sizeof(uint16_t) * (size_t)P) : 0;
    if (d.learned) {
        // feature rows; also holds the gradient for a fallback solve, so at least P floats
        L.feat = take(sizeof(float) * (size_t)std::max(PERF_MLP_NFEAT, 4) * (size_t)units);
        L.mlpw = take(sizeof(uint16_t) * PERF_MLP_NW);
        L.mlpnorm = take(sizeof(float) * PERF_MLP_NNORM);
    }
    L.total = o;
    return L;
}

}  // namespace perf

extern "C" {

const char* perf_last_error(void) { return g_err.c_str(); }

size_t perf_workspace_bytes(const perf_scene_desc* desc, int32_t n_cams) {
    if (validate(desc, n_cams) != PERF_OK) return 0;
    return make_layout(*desc, n_cams).total;
}

int32_t perf_init_scene(const perf_scene_desc* desc, const perf_camera* cams, int32_t n_cams, const float* d_targets,
                        void* d_workspace, size_t ws_bytes, void* stream, perf_scene** out) {
    if (!out) return fail(PERF_EINVAL, "null output handle");
    *out = nullptr;
    int32_t rc = validate(desc, n_cams);
    if (rc != PERF_OK) return rc;
    if (!cams || !d_workspace) return fail(PERF_EINVAL, "null cameras or workspace");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(PERF_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = make_layout(*desc, n_cams);
    if (ws_bytes < L.total) return fail(PERF_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    DevCam* hc = new DevCam[n_cams];
    for (int c = 0; c < n_cams; ++c) {
        bool ok = finite_f(cams[c].fx) && finite_f(cams[c].fy) && cams[c].fx != 0.0f && cams[c].fy != 0.0f &&
                  finite_f(cams[c].cx) && finite_f(cams[c].cy);
        for (int i = 0; i < 3; ++i) ok = ok && finite_f(cams[c].origin[i]);
        for (int i = 0; i < 9; ++i) ok = ok && finite_f(cams[c].rot[i]);
        if (!ok) {
            delete[] hc;
            return fail(PERF_EINVAL, "camera %d is not finite", c);
        }
        memcpy(hc[c].o, cams[c].origin, sizeof(float) * 3);
        memcpy(hc[c].R, cams[c].rot, sizeof(float) * 9);
        hc[c].fx = cams[c].fx;
        hc[c].fy = cams[c].fy;
        hc[c].cx = cams[c].cx;
        hc[c].cy = cams[c].cy;
    }
    perf_scene* s = new perf_scene();
    s->desc = *desc;
    s->n_cams = n_cams;
    s->geo = make_geo(*desc, n_cams);
    s->lay = L;
    s->ws = (char*)d_workspace;
    s->targets = d_targets;
    s->stream = (hipStream_t)stream;
    s->units = (int64_t)desc->nx * desc->ny * desc->nz + (int64_t)desc->n_layers * desc->env_w * desc->env_h;
    s->P = 4 * s->units;
    s->n_rays = (int64_t)n_cams * desc->width * desc->height;
    s->n_ray_blocks = n_cams * s->geo.n_tiles;
    s->cams = (DevCam*)(s->ws + L.cams);
    s->partials = (double*)(s->ws + L.partials);
    s->scalars = (double*)(s->ws + L.scalars);
    s->hist = (double*)(s->ws + L.hist);
    s->iflags = (int*)(s->ws + L.iflags);
    s->vr = (float*)(s->ws + L.vr);
    s->vz = (float*)(s->ws + L.vz);
    s->vp = (float*)(s->ws + L.vp);
    s->vAp = (float*)(s->ws + L.vAp);
    s->vdelta = (float*)(s->ws + L.vdelta);
    s->vxt = (float*)(s->ws + L.vxt);
    s->blocks = (float*)(s->ws + L.blocks);
    s->minv = (float*)(s->ws + L.minv);
    s->xb16 = desc->param_dtype == PERF_BF16 ? (uint16_t*)(s->ws + L.xb16) : nullptr;
    s->feat = desc->learned ? (float*)(s->ws + L.feat) : nullptr;
    s->mlpw = desc->learned ? (uint16_t*)(s->ws + L.mlpw) : nullptr;
    s->mlpnorm = desc->learned ? (float*)(s->ws + L.mlpnorm) : nullptr;
    s->q_fallback = INFINITY;
    s->mlp_ready = false;
    hipError_t e = hipMemcpyAsync(s->cams, hc, sizeof(DevCam) * n_cams, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    delete[] hc;
    if (e != hipSuccess) {
        delete s;
        return fail(PERF_EDEVICE, "copying cameras: %s", hipGetErrorString(e));
    }
    *out = s;
    return PERF_OK;
}

int32_t perf_set_targets(perf_scene* s, const float* d_targets) {
    if (!s) return fail(PERF_EINVAL, "null scene");
    s->targets = d_targets;
    return PERF_OK;
}

int32_t perf_set_jitter(perf_scene* s, uint32_t seed) {
    if (!s) return fail(PERF_EINVAL, "null scene");
    s->geo.jseed = seed;
    return PERF_OK;
}

int32_t perf_set_stream(perf_scene* s, void* stream) {
    if (!s) return fail(PERF_EINVAL, "null scene");
    s->stream = (hipStream_t)stream;
    return PERF_OK;
}

int32_t perf_scene_sizes(const perf_scene* s, int64_t* n_rays, int64_t* n_units, int64_t* n_params) {
    if (!s) return fail(PERF_EINVAL, "null scene");
    if (n_rays) *n_rays = s->n_rays;
    if (n_units) *n_units = s->units;
    if (n_params) *n_params = s->P;
    return PERF_OK;
}

int32_t perf_destroy_scene(perf_scene* s) {
    delete s;
    return PERF_OK;
}

// Kernel arguments every ray launch of a scene shares: cameras and the auxiliary residual.
static RayArgs base_args(const perf_scene* s) {
    RayArgs a{};
    a.cams = s->cams;
    a.aux = s->desc.aux_lambda;
    a.nres = s->desc.aux_lambda > 0.0f ? 4 : 3;
    return a;
}

int32_t perf_render_residuals(perf_scene* s, const void* d_x, float* d_r, double* d_F) {
    if (!s || !d_x) return fail(PERF_EINVAL, "null scene or parameters");
    RayArgs a = base_args(s);
    a.x = d_x;
    a.targets = s->targets;
    a.rout = d_r;
    a.partials = d_F ? s->partials : nullptr;
    a.thresh = s->desc.render_threshold;
    CK(launch_ray(M_RENDER, s->desc.param_dtype, s->geo, a, s->stream));
    if (d_F) CK(launch_sum_partials(s->partials, s->n_ray_blocks, 0.5, d_F, s->stream));
    return PERF_OK;
}

int32_t perf_apply_J(perf_scene* s, const void* d_x, const float* d_v, float* d_u) {
    if (!s || !d_x || !d_v || !d_u) return fail(PERF_EINVAL, "null argument");
    RayArgs a = base_args(s);
    a.x = d_x;
    a.v = d_v;
    a.rout = d_u;
    CK(launch_ray(M_JVP, s->desc.param_dtype, s->geo, a, s->stream));
    return PERF_OK;
}

int32_t perf_apply_Jt(perf_scene* s, const void* d_x, const float* d_u, float* d_y) {
    if (!s || !d_x || !d_u || !d_y) return fail(PERF_EINVAL, "null argument");
    CK(launch_zero(d_y, s->P, s->stream));
    RayArgs a = base_args(s);
    a.x = d_x;
    a.uin = d_u;
    a.y = d_y;
    CK(launch_ray(M_VJP, s->desc.param_dtype, s->geo, a, s->stream));
    return PERF_OK;
}

int32_t perf_apply_JtJ(perf_scene* s, const void* d_x, const float* d_v, float* d_y) {
    if (!s || !d_x || !d_v || !d_y) return fail(PERF_EINVAL, "null argument");
    CK(launch_zero(d_y, s->P, s->stream));
    RayArgs a = base_args(s);
    a.x = d_x;
    a.v = d_v;
    a.y = d_y;
    CK(launch_ray(M_JTJ, s->desc.param_dtype, s->geo, a, s->stream));
    return PERF_OK;
}

static int32_t grad_pass(perf_scene* s, const void* xg, float* grad, float* blocks, bool want_F) {
    if (grad) CK(launch_zero(grad, s->P, s->stream));
    if (blocks) CK(launch_zero(blocks, 5 * s->units, s->stream));
    RayArgs a = base_args(s);
    a.x = xg;
    a.targets = s->targets;
    a.y = grad;
    a.blocks = blocks;
    a.partials = s->partials;
    CK(launch_ray(M_GRAD, s->desc.param_dtype, s->geo, a, s->stream));
    if (want_F) CK(launch_sum_partials(s->partials, s->n_ray_blocks, 0.5, s->scalars + S_F, s->stream));
    return PERF_OK;
}

int32_t perf_build_precond(perf_scene* s, const void* d_x, int32_t kind, float* d_grad, float* d_blocks, float* d_out,
                           double* d_F) {
    if (!s || !d_x) return fail(PERF_EINVAL, "null argument");
    if (!s->targets) return fail(PERF_EINVAL, "scene has no targets");
    if (kind != PERF_PRECOND_NONE && kind != PERF_PRECOND_JACOBI && kind != PERF_PRECOND_BLOCK4)
        return fail(PERF_EINVAL, "kind must be NONE, JACOBI or BLOCK4");
    if (kind != PERF_PRECOND_NONE && !d_out) return fail(PERF_EINVAL, "null output");
    float* blocks = d_blocks ? d_blocks : s->blocks;
    int32_t rc = grad_pass(s, d_x, d_grad, blocks, d_F != nullptr);
    if (rc != PERF_OK) return rc;
    if (d_F) CK(hipMemcpyAsync(d_F, s->scalars + S_F, sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    if (kind != PERF_PRECOND_NONE) CK(launch_precond_invert(kind, blocks, s->units, d_out, s->stream));
    return PERF_OK;
}

int32_t perf_footprint(perf_scene* s, int32_t* d_per_ray, uint64_t* d_totals) {
    if (!s) return fail(PERF_EINVAL, "null scene");
    if (d_totals) CK(launch_zero_u64((unsigned long long*)d_totals, 3, s->stream));
    CK(launch_footprint(s->geo, s->cams, d_per_ray, (unsigned long long*)d_totals, s->stream));
    return PERF_OK;
}

int32_t perf_upsample(const perf_scene_desc* from, const float* d_from, const perf_scene_desc* to, float* d_to,
                      void* stream) {
    if (!from || !to) return fail(PERF_EINVAL, "null descriptor");
    if (!d_from || !d_to) return fail(PERF_EINVAL, "null parameter vector");
    for (const perf_scene_desc* d : {from, to}) {
        if (d->nx < 2 || d->ny < 2 || d->nz < 2) return fail(PERF_EINVAL, "grid dims must be >= 2");
        if (d->n_layers < 0 || d->n_layers > PERF_MAX_LAYERS) return fail(PERF_EINVAL, "n_layers must be in 0..8");
        if (d->n_layers > 0 && (d->env_w < 2 || d->env_h < 2)) return fail(PERF_EINVAL, "env_w and env_h must be >= 2");
        const int64_t units = (int64_t)d->nx * d->ny * d->nz + (int64_t)d->n_layers * d->env_w * d->env_h;
        if (units * 10 >= (int64_t)1 << 31) return fail(PERF_EUNSUPPORTED, "too many parameters for 32-bit indexing");
    }
    if (from->n_layers != to->n_layers) return fail(PERF_EINVAL, "levels must have the same environment layers");
    for (int a = 0; a < 3; ++a) {
        if (from->bbox_min[a] != to->bbox_min[a] || from->bbox_max[a] != to->bbox_max[a])
            return fail(PERF_EINVAL, "levels must share the bounding box");
        if (!(from->bbox_max[a] > from->bbox_min[a])) return fail(PERF_EINVAL, "bad bounding box");
    }
    for (int l = 0; l < from->n_layers; ++l)
        if (from->layer_radius[l] != to->layer_radius[l]) return fail(PERF_EINVAL, "levels must share the layer radii");
    // sigma is an optical depth per shortest voxel side: scale by the ratio of the sides
    auto side = [](const perf_scene_desc* d) {
        const float h[3] = {(d->bbox_max[0] - d->bbox_min[0]) / (float)d->nx, (d->bbox_max[1] - d->bbox_min[1]) / (float)d->ny,
                            (d->bbox_max[2] - d->bbox_min[2]) / (float)d->nz};
        return fminf(h[0], fminf(h[1], h[2]));
    };
    const float scale = side(to) / side(from);
    CK(launch_upsample(d_from, from->nx, from->ny, from->nz, from->env_w, from->env_h, d_to, to->nx, to->ny, to->nz,
                       to->env_w, to->env_h, to->n_layers, scale, (hipStream_t)stream));
    return PERF_OK;
}

int32_t perf_invert_blocks(const float* d_blocks, int64_t units, int32_t kind, float* d_out, void* stream) {
    if (units < 0) return fail(PERF_EINVAL, "negative unit count");
    if ((!d_blocks || !d_out) && units > 0) return fail(PERF_EINVAL, "null argument");
    if (kind != PERF_PRECOND_JACOBI && kind != PERF_PRECOND_BLOCK4) return fail(PERF_EINVAL, "kind must be JACOBI or BLOCK4");
    if (units == 0) return PERF_OK;
    CK(launch_precond_invert(kind, d_blocks, units, d_out, (hipStream_t)stream));
    return PERF_OK;
}

int32_t perf_pack_bf16(const float* d_in, uint16_t* d_out, int64_t n, void* stream) {
    if ((!d_in || !d_out) && n > 0) return fail(PERF_EINVAL, "null argument");
    if (n < 0) return fail(PERF_EINVAL, "negative size");
    CK(launch_pack_bf16(d_in, d_out, n, (hipStream_t)stream));
    return PERF_OK;
}

// F(proj(x + gamma delta)) on the device into scalars[S_TMP]; the trial point is left in
// vxt (FP32) and, for BF16 storage, in xb16.
static int32_t trial_objective(perf_scene* s, const float* d_x, const float* d_delta, float gamma) {
    CK(launch_trial(d_x, d_delta, gamma, s->units, s->geo.nvox, s->vxt, s->xb16, s->stream));
    RayArgs a = base_args(s);
    a.x = s->xb16 ? (const void*)s->xb16 : (const void*)s->vxt;
    a.targets = s->targets;
    a.partials = s->partials;
    CK(launch_ray(M_RENDER, s->desc.param_dtype, s->geo, a, s->stream));
    CK(launch_sum_partials(s->partials, s->n_ray_blocks, 0.5, s->scalars + S_TMP, s->stream));
    return PERF_OK;
}

static int32_t read_scalar(perf_scene* s, int idx, double* out) {
    CK(hipMemcpyAsync(out, s->scalars + idx, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    CK(hipStreamSynchronize(s->stream));
    return PERF_OK;
}

int32_t perf_objective(perf_scene* s, const float* d_x, const float* d_delta, float gamma, double* F_host) {
    if (!s || !d_x || !F_host) return fail(PERF_EINVAL, "null argument");
    if (!s->targets) return fail(PERF_EINVAL, "scene has no targets");
    int32_t rc = trial_objective(s, d_x, d_delta, gamma);
    if (rc != PERF_OK) return rc;
    return read_scalar(s, S_TMP, F_host);
}


// ---------------------------------------------------------------- learned block preconditioner
int32_t perf_precond_features(perf_scene* s, const void* d_x, float* d_feat, float* d_blocks) {
    if (!s || !d_x || !d_feat) return fail(PERF_EINVAL, "null argument");
    if (!s->feat) return fail(PERF_EUNSUPPORTED, "the scene was created without learned = 1");
    float* blocks = d_blocks ? d_blocks : s->blocks;
    int32_t rc = grad_pass(s, d_x, nullptr, blocks, false);
    if (rc != PERF_OK) return rc;
    CK(launch_unit_features(d_x, s->desc.param_dtype, blocks, s->units, d_feat, s->stream));
    return PERF_OK;
}

int32_t perf_mlp_set_weights(perf_scene* s, const uint16_t* d_w, int32_t n_w, const float* d_norm, float q_fallback) {
    if (!s || !d_w || !d_norm) return fail(PERF_EINVAL, "null argument");
    if (!s->mlpw) return fail(PERF_EUNSUPPORTED, "the scene was created without learned = 1");
    if (n_w != PERF_MLP_NW) return fail(PERF_EINVAL, "expected %d weights, got %d", PERF_MLP_NW, n_w);
    if (isnan(q_fallback) || q_fallback < 0.0f) return fail(PERF_EINVAL, "q_fallback must be >= 0 (INFINITY: never)");
    CK(hipMemcpyAsync(s->mlpw, d_w, sizeof(uint16_t) * PERF_MLP_NW, hipMemcpyDeviceToDevice, s->stream));
    CK(hipMemcpyAsync(s->mlpnorm, d_norm, sizeof(float) * PERF_MLP_NNORM, hipMemcpyDeviceToDevice, s->stream));
    s->q_fallback = q_fallback;
    s->mlp_ready = true;
    return PERF_OK;
}

int32_t perf_mlp_infer(perf_scene* s, const float* d_feat, const float* d_blocks, float* d_minv) {
    if (!s || !d_feat || !d_blocks || !d_minv) return fail(PERF_EINVAL, "null argument");
    if (!s->mlp_ready) return fail(PERF_EINVAL, "no weights (perf_mlp_set_weights)");
    CK(launch_mlp_infer(s->mlpw, s->mlpnorm, s->q_fallback, d_feat, d_blocks, s->units, d_minv, s->stream));
    return PERF_OK;
}

int32_t perf_mlp_train_step(float* d_w32, uint16_t* d_wbf16, float* d_m, float* d_v, int32_t t, float lr,
                            float damp, const float* d_norm, const float* d_feat, const float* d_blocks, int32_t n,
                            float* d_loss, float* d_grad_scratch, void* stream) {
    if (!d_w32 || !d_wbf16 || !d_m || !d_v || !d_loss || !d_grad_scratch || !d_norm)
        return fail(PERF_EINVAL, "null argument");
    if (n < 0 || (n > 0 && (!d_feat || !d_blocks))) return fail(PERF_EINVAL, "bad batch");
    if (t < 1 || !(lr > 0.0f)) return fail(PERF_EINVAL, "need t >= 1 and lr > 0");
    if (!(damp >= 0.0f && damp <= 1e6f)) return fail(PERF_EINVAL, "damp must be in [0, 1e6]");
    CK(launch_mlp_train(d_w32, d_wbf16, d_m, d_v, t, lr, damp, d_norm, d_feat, d_blocks, n, d_loss, d_grad_scratch,
                        (hipStream_t)stream));
    return PERF_OK;
}

int32_t perf_mlp_train_step_noalloc(float* d_w32, uint16_t* d_wbf16, float* d_m, float* d_v, int32_t t, float lr,
                                    float damp, const float* d_norm, const float* d_feat, const float* d_blocks,
                                    int32_t n, float* d_loss, void* stream) {
    if (!d_w32 || !d_wbf16 || !d_m || !d_v || !d_loss || !d_norm) return fail(PERF_EINVAL, "null argument");
    if (n < 0 || (n > 0 && (!d_feat || !d_blocks))) return fail(PERF_EINVAL, "bad batch");
    if (t < 1 || !(lr > 0.0f)) return fail(PERF_EINVAL, "need t >= 1 and lr > 0");
    if (!(damp >= 0.0f && damp <= 1e6f)) return fail(PERF_EINVAL, "damp must be in [0, 1e6]");
    CK(launch_mlp_train_static(d_w32, d_wbf16, d_m, d_v, t, lr, damp, d_norm, d_feat, d_blocks, n, d_loss,
                               (hipStream_t)stream));
    return PERF_OK;
}

int32_t perf_mlp_feature_stats(const float* d_feat, int64_t n, float* d_norm, void* stream) {
    if (!d_norm || (n > 0 && !d_feat)) return fail(PERF_EINVAL, "null argument");
    if (n < 0) return fail(PERF_EINVAL, "negative row count");
    CK(launch_feature_stats(d_feat, n, d_norm, (hipStream_t)stream));
    return PERF_OK;
}

int32_t perf_mlp_training_rows(perf_scene* s, const float* d_feat, const float* d_blocks, uint32_t seed, float keep,
                               float* d_feat_out, float* d_blocks_out, int64_t cap, int64_t* n_kept) {
    if (!s || !d_feat || !d_blocks || !n_kept) return fail(PERF_EINVAL, "null argument");
    if (cap < 0 || (cap > 0 && (!d_feat_out || !d_blocks_out))) return fail(PERF_EINVAL, "bad output capacity");
    if (!(keep >= 0.0f && keep <= 1.0f)) return fail(PERF_EINVAL, "keep must be in [0, 1]");
    long long* counts = reinterpret_cast<long long*>(s->partials);  // kVecGrid + 1 entries
    CK(launch_training_rows(d_feat, d_blocks, s->units, seed, keep, d_feat_out, d_blocks_out, cap, counts, s->stream));
    long long total = 0;
    CK(hipMemcpyAsync(&total, counts + kVecGrid, sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    CK(hipStreamSynchronize(s->stream));
    *n_kept = total;
    return PERF_OK;
}

// features from the parameters the gradient pass gathered (xg: the bfloat16 copy with bf16
// storage, as perf_precond_features sees them) and its blocks (in s->blocks), then the predicted
// inverses: no further traversal
static int32_t learned_minv(perf_scene* s, const void* xg) {
    CK(launch_unit_features(xg, s->desc.param_dtype, s->blocks, s->units, s->feat, s->stream));
    CK(launch_mlp_infer(s->mlpw, s->mlpnorm, s->q_fallback, s->feat, s->blocks, s->units, s->minv, s->stream));
    return PERF_OK;
}

// PCG (Alg. 2) from Delta_0 = 0 on the gradient in s->vr, then the line search (Alg. 3).
// Records ev[0] after the solve and ev[1] after the search; the J^T J v launches are bracketed
// by jev[2k], jev[2k+1].
struct SolveOut {
    int flags = 0, iters = 0, trials = 0, n_jtj = 0;
    double F0 = 0.0, gamma = 0.0, mu_acc = 0.0;
};

static int32_t solve_and_search(perf_scene* s, const void* xg, float* d_x, const perf_pcg_opts* opts,
                                int apply_kind, hipEvent_t* ev, hipEvent_t* jev, SolveOut* out) {
    hipStream_t st = s->stream;
    s->host_scalars[S_MAXITERS] = opts->max_iters;
    s->host_scalars[S_RELTOL] = opts->rel_tol;
    s->host_scalars[S_ABSEPS] = opts->abs_eps;
    s->host_scalars[S_STALL] = opts->stall_ratio;
    CK(hipMemcpyAsync(s->scalars + S_MAXITERS, s->host_scalars + S_MAXITERS, 4 * sizeof(double),
                      hipMemcpyHostToDevice, st));
    CK(launch_zero(reinterpret_cast<float*>(s->hist), 8 * PERF_MAX_PCG, st));
    CK(launch_pcg_init(apply_kind, s->vr, s->minv, s->vr, s->vz, s->vp, s->vdelta, s->units, s->partials, s->scalars,
                       s->iflags, st));
    const bool poll = opts->rel_tol > 0.0 || opts->abs_eps > 0.0 || opts->stall_ratio > 0.0;
    int n_jtj = 0;
    for (int it = 0; it < opts->max_iters; ++it) {
        CK(launch_zero(s->vAp, s->P, st, s->iflags + I_DONE));
        RayArgs a = base_args(s);
        a.x = xg;
        a.v = s->vp;
        a.y = s->vAp;
        a.done = s->iflags + I_DONE;
        CK(hipEventRecord(jev[2 * it], st));
        CK(launch_ray(M_JTJ, s->desc.param_dtype, s->geo, a, st));
        CK(hipEventRecord(jev[2 * it + 1], st));
        ++n_jtj;
        CK(launch_pcg_alpha(s->vp, s->vAp, s->units, s->partials, s->scalars, s->hist, s->iflags, st));
        CK(launch_pcg_update(apply_kind, s->minv, s->vdelta, s->vr, s->vz, s->vp, s->vAp, s->units, s->partials,
                             s->scalars, s->hist, s->iflags, st));
        CK(launch_pcg_direction(s->vz, s->vp, s->units, s->scalars, s->iflags, st));
        if (poll) {
            int done = 0;
            CK(hipMemcpyAsync(&done, s->iflags + I_DONE, sizeof(int), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            if (done) break;
        }
    }
    CK(hipMemcpyAsync(s->host_scalars, s->scalars, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(s->host_hist, s->hist, sizeof(double) * 4 * PERF_MAX_PCG, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(s->host_flags, s->iflags, sizeof(int) * I_COUNT, hipMemcpyDeviceToHost, st));
    CK(hipEventRecord(ev[0], st));
    CK(hipStreamSynchronize(st));
    const double F0 = s->host_scalars[S_F];
    int flags = s->host_flags[I_FLAGS];
    const int iters = s->host_flags[I_ITERS];
    // line search (Alg. 3) on F(proj(x + gamma Delta)), capped at ls_max trials
    double gamma = 1.0, mu_acc = F0;
    int trials = 0;
    int32_t rc;
    if (opts->line_search) {
        const double fac = opts->ls_factor;
        double g = 1.0, mu_prev = INFINITY, best_mu = INFINITY, best_g = 0.0;
        bool decided = false;
        while (trials < opts->ls_max) {
            rc = trial_objective(s, d_x, s->vdelta, (float)g);
            if (rc != PERF_OK) return rc;
            double mu = 0.0;
            rc = read_scalar(s, S_TMP, &mu);
            if (rc != PERF_OK) return rc;
            ++trials;
            if (mu < best_mu) {
                best_mu = mu;
                best_g = g;
            }
            if (mu > mu_prev) {
                if (mu_prev < F0) {
                    gamma = g / fac;
                    mu_acc = mu_prev;
                } else {
                    gamma = 0.0;
                    mu_acc = F0;
                }
                decided = true;
                break;
            }
            g *= fac;
            mu_prev = mu;
        }
        if (!decided) {
            flags |= PERF_FLAG_LS_CAPPED;
            if (best_mu < F0) {
                gamma = best_g;
                mu_acc = best_mu;
            } else {
                gamma = 0.0;
                mu_acc = F0;
            }
        }
    } else {
        rc = trial_objective(s, d_x, s->vdelta, 1.0f);
        if (rc != PERF_OK) return rc;
        rc = read_scalar(s, S_TMP, &mu_acc);
        if (rc != PERF_OK) return rc;
        trials = 1;
        gamma = 1.0;
    }
    if (gamma == 0.0) flags |= PERF_FLAG_NO_DESCENT;
    CK(hipEventRecord(ev[1], st));
    out->flags = flags;
    out->iters = iters;
    out->trials = trials;
    out->n_jtj = n_jtj;
    out->F0 = F0;
    out->gamma = gamma;
    out->mu_acc = mu_acc;
    return PERF_OK;
}

int32_t perf_gn_step(perf_scene* s, float* d_x, const perf_pcg_opts* opts, perf_gn_stats* stats) {
    if (!s || !d_x || !opts) return fail(PERF_EINVAL, "null argument");
    if (!s->targets) return fail(PERF_EINVAL, "scene has no targets");
    if (opts->max_iters < 1 || opts->max_iters > PERF_MAX_PCG) return fail(PERF_EINVAL, "max_iters must be 1..256");
    if (opts->precond < PERF_PRECOND_NONE || opts->precond > PERF_PRECOND_LEARNED)
        return fail(PERF_EINVAL, "bad preconditioner kind");
    if (opts->line_search && (!(opts->ls_factor > 0.0f && opts->ls_factor < 1.0f) || opts->ls_max < 1))
        return fail(PERF_EINVAL, "line search needs 0 < ls_factor < 1 and ls_max >= 1");
    if (opts->precond == PERF_PRECOND_LEARNED && !s->mlp_ready)
        return fail(PERF_EINVAL, "learned preconditioner has no weights (perf_mlp_set_weights)");
    hipStream_t st = s->stream;
    // phase events, plus a pair around every J^T J v launch (its kernel time, for the roofline)
    constexpr int kPh = 6;
    hipEvent_t ev[kPh + 2 * PERF_MAX_PCG];
    const int n_ev = kPh + 2 * opts->max_iters;
    for (int i = 0; i < n_ev; ++i) CK(hipEventCreate(&ev[i]));
    struct EvGuard {
        hipEvent_t* e;
        int n;
        ~EvGuard() {
            for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
        }
    } guard{ev, n_ev};
    CK(hipEventRecord(ev[0], st));
    if (s->desc.checks) {
        CK(hipMemsetAsync(s->iflags + I_NONFINITE, 0, sizeof(int), st));
        CK(launch_check_finite(d_x, s->P, s->iflags + I_NONFINITE, st));
        CK(launch_check_finite(s->targets, 3 * s->n_rays, s->iflags + I_NONFINITE, st));
        int bad = 0;
        CK(hipMemcpyAsync(&bad, s->iflags + I_NONFINITE, sizeof(int), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        if (bad) return fail(PERF_ENUMERIC, "non-finite parameters or targets");
    }
    const void* xg = d_x;
    if (s->xb16) {
        CK(launch_pack_bf16(d_x, s->xb16, s->P, st));
        xg = s->xb16;
    }
    // 1. gradient b = -J^T r (into vr) and the exact 4x4 blocks, F(x)
    const int kind = opts->precond;
    int32_t rc = grad_pass(s, xg, s->vr, s->blocks, true);
    if (rc != PERF_OK) return rc;
    CK(hipEventRecord(ev[1], st));
    // 2. preconditioner
    if (kind == PERF_PRECOND_JACOBI || kind == PERF_PRECOND_BLOCK4) {
        CK(launch_precond_invert(kind, s->blocks, s->units, s->minv, st));
    } else if (kind == PERF_PRECOND_LEARNED) {
        rc = learned_minv(s, xg);
        if (rc != PERF_OK) return rc;
        // keep b for a fallback solve: the feature rows (at least P floats) are free now
        CK(hipMemcpyAsync(s->feat, s->vr, sizeof(float) * s->P, hipMemcpyDeviceToDevice, st));
    }
    CK(hipEventRecord(ev[2], st));
    // 3-4. PCG and the line search
    SolveOut so;
    rc = solve_and_search(s, xg, d_x, opts, kind, ev + 3, ev + kPh, &so);
    if (rc != PERF_OK) return rc;
    int fallback_iters = 0;
    if (kind == PERF_PRECOND_LEARNED &&
        (so.flags & (PERF_FLAG_BREAKDOWN | PERF_FLAG_STALL | PERF_FLAG_NO_DESCENT))) {
        // the learned solve failed: solve again from Delta_0 = 0 with the exact block inverse
        fallback_iters = so.iters;
        CK(hipMemcpyAsync(s->vr, s->feat, sizeof(float) * s->P, hipMemcpyDeviceToDevice, st));
        CK(launch_precond_invert(PERF_PRECOND_BLOCK4, s->blocks, s->units, s->minv, st));
        rc = solve_and_search(s, xg, d_x, opts, PERF_PRECOND_BLOCK4, ev + 3, ev + kPh, &so);
        if (rc != PERF_OK) return rc;
        so.flags |= PERF_FLAG_FALLBACK;
    }
    // 5. x <- proj(x + gamma Delta), in place
    if (so.gamma != 0.0) CK(launch_trial(d_x, s->vdelta, (float)so.gamma, s->units, s->geo.nvox, d_x, nullptr, st));
    CK(hipEventRecord(ev[5], st));
    CK(hipEventSynchronize(ev[5]));
    if (stats) {
        const int iters = so.iters, flags = so.flags;
        memset(stats, 0, sizeof(*stats));
        stats->F_before = so.F0;
        stats->F_after = so.mu_acc;
        stats->gamma = so.gamma;
        stats->pcg_iters = iters;
        stats->ls_trials = so.trials;
        stats->flags = flags;
        stats->fallback_iters = fallback_iters;
        stats->R0 = s->host_scalars[S_R0];
        for (int k = 0; k < iters && k < PERF_MAX_PCG; ++k) {
            stats->alpha[k] = s->host_hist[4 * k + 0];
            stats->beta[k] = s->host_hist[4 * k + 1];
            stats->R[k] = s->host_hist[4 * k + 2];
            stats->pAp[k] = s->host_hist[4 * k + 3];
        }
        if (iters < PERF_MAX_PCG && (flags & PERF_FLAG_BREAKDOWN)) stats->pAp[iters] = s->host_hist[4 * iters + 3];
        float ms = 0.0f;
        for (int i = 0; i < 5; ++i) {
            CK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            stats->ms_phase[i] = ms;
        }
        CK(hipEventElapsedTime(&ms, ev[0], ev[5]));
        stats->ms_phase[5] = ms;
        // J^T J v kernel time summed over the launches of the final solve that did work (the
        // solve's stop flag turns later launches into immediate exits)
        float jtj = 0.0f;
        const int worked = iters + ((flags & PERF_FLAG_BREAKDOWN) ? 1 : 0);
        for (int k = 0; k < so.n_jtj && k < worked; ++k) {
            CK(hipEventElapsedTime(&ms, ev[kPh + 2 * k], ev[kPh + 2 * k + 1]));
            jtj += ms;
        }
        stats->ms_phase[6] = jtj;
        stats->ms_phase[7] = (float)worked;
    }
    return PERF_OK;
}

}  // extern "C"
