// Internal declarations of the gfx950 Gauss-Newton library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perf_gn.h"

namespace perf {

constexpr int kMaxLayers = PERF_MAX_LAYERS;
constexpr int kWaves = 2;       // wave64s per ray workgroup
constexpr int kBlock = 64 * kWaves;
constexpr int kTileX = 16;      // ray workgroup tile: 16 x 8 pixels, each wave an 8x8 half
constexpr int kTileY = 8;
constexpr int kVecBlock = 256;  // threads per vector workgroup
constexpr int kVecGrid = 2048;  // workgroups of the grid-stride vector kernels (FP64 partials)

// Camera as the kernels read it: 16 floats, 64 bytes.
struct DevCam {
    float o[3];
    float R[9];
    float fx, fy, cx, cy;
};

// Scene geometry passed by value to every ray kernel.
struct Geo {
    int nx, ny, nz, n_layers;
    int env_w, env_h, width, height;
    int n_cams, tiles_x, tiles_y, n_tiles;
    float bmin[3], bmax[3];
    float inv_hv[3];  // 1 / voxel side per axis
    float h;          // shortest voxel side (the unit of delta)
    float step;       // march step in units of h
    float radius[kMaxLayers];
    float bg[3];
    int nvox;         // voxel units; texel units follow
    unsigned jseed;   // jittering seed (Sec. IV), 0 = pixel centres and step midpoints
};

// Device scalars of a Gauss-Newton step (FP64), indices into the scalar array.
enum Scalar {
    S_RZ = 0,      // r_k^T z_k
    S_PAP = 1,     // p_k^T A p_k
    S_ALPHA = 2,
    S_BETA = 3,
    S_R = 4,       // r_{k+1}^T r_{k+1}
    S_RPREV = 5,
    S_R0 = 6,
    S_F = 7,       // objective of the last render / grad pass
    S_RZNEW = 8,
    S_MAXITERS = 9,
    S_RELTOL = 10,
    S_ABSEPS = 11,
    S_STALL = 12,
    S_TMP = 16,    // scratch for perf_objective etc.
    S_COUNT = 32
};
// Device int flags.
enum IFlag { I_DONE = 0, I_ITERS = 1, I_FLAGS = 2, I_NONFINITE = 3, I_COUNT = 16 };

// Workspace layout (offsets in bytes from the workspace base).
struct Layout {
    size_t cams, partials, scalars, hist, iflags;
    size_t vr, vz, vp, vAp, vdelta, vxt, blocks, minv, xb16, feat, mlpw, mlpnorm;
    size_t total;
    int64_t n_partials;
};

Layout make_layout(const perf_scene_desc& d, int n_cams);
Geo make_geo(const perf_scene_desc& d, int n_cams);

// ---------------------------------------------------------------- launchers (raymarch.hip)
enum RayMode { M_RENDER = 0, M_JVP = 1, M_VJP = 2, M_JTJ = 3, M_GRAD = 4, M_COUNT = 5 };

struct RayArgs {
    const DevCam* cams;
    const void* x;           // params (FP32 float4 or BF16 ushort4 per unit)
    const float* v;          // tangent [P] (JVP / JTJ)
    const float* targets;    // [rays][3] (RENDER residuals / GRAD)
    const float* uin;        // [rays][nres] (VJP)
    float* rout;             // [rays][nres] residuals (RENDER with targets) or u (JVP); [rays][3] H otherwise
    float* y;                // [P] scatter target (VJP / JTJ), gradient (GRAD)
    float* blocks;           // [units][5] (GRAD)
    double* partials;        // [n_tiles] FP64 sums of r^2
    const int* done;         // skip the launch's work when *done != 0 (PCG stop on device)
    float aux;               // weight lambda of the auxiliary opacity residual (Sec. III-I), 0 = off
    int nres;                // residuals per ray: 4 with the auxiliary residual, else 3
    float thresh;            // RENDER: volume counts as transparent when 1 - T_exit < thresh (0 = off)
};

hipError_t launch_ray(int mode, int param_dtype, const Geo& g, const RayArgs& a, hipStream_t st);
hipError_t launch_footprint(const Geo& g, const DevCam* cams, int32_t* per_ray, unsigned long long* totals,
                            hipStream_t st);

// ---------------------------------------------------------------- launchers (vector.hip)
hipError_t launch_zero(float* p, int64_t n, hipStream_t st, const int* done = nullptr);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_sum_partials(const double* partials, int64_t n, double scale, double* out, hipStream_t st);
hipError_t launch_precond_invert(int kind, const float* blocks, int64_t units, float* out, hipStream_t st);
hipError_t launch_pcg_init(int kind, const float* b, const float* minv, float* r, float* z, float* p, float* delta,
                           int64_t units, double* partials, double* scalars, int* iflags, hipStream_t st);
hipError_t launch_pcg_alpha(const float* p, const float* Ap, int64_t units, double* partials, double* scalars,
                            double* hist, int* iflags, hipStream_t st);
hipError_t launch_pcg_update(int kind, const float* minv, float* delta, float* r, float* z, const float* p,
                             const float* Ap, int64_t units, double* partials, double* scalars, double* hist,
                             int* iflags, hipStream_t st);
hipError_t launch_pcg_direction(const float* z, float* p, int64_t units, const double* scalars, const int* iflags,
                                hipStream_t st);
hipError_t launch_trial(const float* x, const float* delta, float gamma, int64_t units, int nvox, float* xt,
                        uint16_t* xb16, hipStream_t st);
hipError_t launch_pack_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t st);
hipError_t launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t st);
hipError_t launch_unit_features(const void* x, int x_dtype, const float* blocks, int64_t units, float* feat,
                                hipStream_t st);
// counts: kVecGrid + 1 int64 of scratch; counts[kVecGrid] receives the number of kept rows
hipError_t launch_training_rows(const float* feat, const float* blocks, int64_t units, unsigned seed, float keep,
                                float* feat_out, float* blocks_out, int64_t cap, long long* counts, hipStream_t st);

// ---------------------------------------------------------------- launchers (mlp.hip)
hipError_t launch_mlp_infer(const uint16_t* w, const float* norm, float q_fallback, const float* feat,
                            const float* blocks, int64_t units, float* minv, hipStream_t st);
hipError_t launch_mlp_train(float* w32, uint16_t* wbf, float* m, float* v, int t, float lr, float damp,
                            const float* norm, const float* feat, const float* blocks, int n, float* loss, float* grad,
                            hipStream_t st);
hipError_t launch_mlp_train_static(float* w32, uint16_t* wbf, float* m, float* v, int t, float lr, float damp,
                                   const float* norm, const float* feat, const float* blocks, int n, float* loss,
                                   hipStream_t st);
hipError_t launch_feature_stats(const float* feat, int64_t n, float* norm, hipStream_t st);

hipError_t launch_upsample(const float* src, int sx, int sy, int sz, int sw, int sh, float* dst, int dx, int dy,
                           int dz, int dw, int dh, int layers, float sigma_scale, hipStream_t st);

}  // namespace perf
