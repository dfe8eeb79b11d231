// Resampling of the parameters between hierarchical levels (Sec. IV, hierarchical
// formulation): the next level's grid and environment layers are filled from the current
// ones by linear interpolation at the new cell and texel centres.  One thread per
// destination unit; reads are gathers of 8 (voxel) or 4 (texel) float4 from the source.
#include "perf_internal.h"

namespace perf {
namespace {

// Source coordinate of destination cell j along an axis (cell-centred): clamped to the
// source's first and last centres, lower index at most n_src - 2.
__device__ __forceinline__ void lerp_clamped(int j, int n_src, int n_dst, int& i0, float& f) {
    float g = ((float)j + 0.5f) * (float)n_src / (float)n_dst - 0.5f;
    g = fminf(fmaxf(g, 0.0f), (float)(n_src - 1));
    i0 = min((int)g, n_src - 2);
    f = g - (float)i0;
}

// Periodic axis (azimuth): the lower index wraps.
__device__ __forceinline__ void lerp_periodic(int j, int n_src, int n_dst, int& i0, int& i1, float& f) {
    const float g = ((float)j + 0.5f) * (float)n_src / (float)n_dst - 0.5f;
    const float fl = floorf(g);
    f = g - fl;
    i0 = (int)fl;
    i0 = ((i0 % n_src) + n_src) % n_src;
    i1 = (i0 + 1 == n_src) ? 0 : i0 + 1;
}

__global__ __launch_bounds__(256) void k_upsample_grid(const float4* __restrict__ src, int sx, int sy, int sz,
                                                      float4* __restrict__ dst, int dx, int dy, int dz,
                                                      float sigma_scale) {
    const int64_t n = (int64_t)dx * dy * dz;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(u % dx);
        const int y = (int)((u / dx) % dy);
        const int z = (int)(u / ((int64_t)dx * dy));
        int ix, iy, iz;
        float fx, fy, fz;
        lerp_clamped(x, sx, dx, ix, fx);
        lerp_clamped(y, sy, dy, iy, fy);
        lerp_clamped(z, sz, dz, iz, fz);
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int ox = b & 1, oy = (b >> 1) & 1, oz = b >> 2;
            const float w = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy) * (oz ? fz : 1.0f - fz);
            const float4 q = src[((int64_t)(iz + oz) * sy + (iy + oy)) * sx + (ix + ox)];
            acc.x += w * q.x;
            acc.y += w * q.y;
            acc.z += w * q.z;
            acc.w += w * q.w;
        }
        acc.w *= sigma_scale;
        dst[u] = acc;
    }
}

__global__ __launch_bounds__(256) void k_upsample_env(const float4* __restrict__ src, int sw, int sh,
                                                     float4* __restrict__ dst, int dw, int dh, int layers) {
    const int64_t n = (int64_t)layers * dw * dh;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(u % dw);
        const int j = (int)((u / dw) % dh);
        const int l = (int)(u / ((int64_t)dw * dh));
        int i0, i1, j0;
        float fu, fv;
        lerp_periodic(i, sw, dw, i0, i1, fu);
        lerp_clamped(j, sh, dh, j0, fv);
        const float4* s = src + (int64_t)l * sw * sh;
        const float4 a = s[(int64_t)j0 * sw + i0], b = s[(int64_t)j0 * sw + i1];
        const float4 c = s[(int64_t)(j0 + 1) * sw + i0], d = s[(int64_t)(j0 + 1) * sw + i1];
        const float wa = (1.0f - fu) * (1.0f - fv), wb = fu * (1.0f - fv), wc = (1.0f - fu) * fv, wd = fu * fv;
        dst[u] = make_float4(wa * a.x + wb * b.x + wc * c.x + wd * d.x, wa * a.y + wb * b.y + wc * c.y + wd * d.y,
                             wa * a.z + wb * b.z + wc * c.z + wd * d.z, wa * a.w + wb * b.w + wc * c.w + wd * d.w);
    }
}

unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65535) g = 65535;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_upsample(const float* src, int sx, int sy, int sz, int sw, int sh, float* dst, int dx, int dy,
                           int dz, int dw, int dh, int layers, float sigma_scale, hipStream_t st) {
    const int64_t nv_dst = (int64_t)dx * dy * dz;
    hipLaunchKernelGGL(k_upsample_grid, dim3(grid_for(nv_dst)), dim3(256), 0, st, (const float4*)src, sx, sy, sz,
                       (float4*)dst, dx, dy, dz, sigma_scale);
    if (layers > 0) {
        const int64_t nv_src = (int64_t)sx * sy * sz;
        const int64_t nt = (int64_t)layers * dw * dh;
        hipLaunchKernelGGL(k_upsample_env, dim3(grid_for(nt)), dim3(256), 0, st, (const float4*)src + nv_src, sw, sh,
                           (float4*)dst + nv_dst, dw, dh, layers);
    }
    return hipGetLastError();
}

}  // namespace perf
