// Per-ray kernels of the Gauss-Newton step on gfx950.
//
// One lane marches one pixel ray; a 256-thread workgroup owns a 16x16 pixel tile of one
// camera and each wave64 an 8x8 quarter of it, so the lanes of a wave sample neighbouring
// rays at the same step index and their trilinear gathers hit the same cache lines.
//
// Per ray (Sec. III-A, Eq. 3-4): slab test against the grid box, K = ceil(L / step)
// samples at the midpoints of equal steps of `step` voxel lengths (the last one shortened
// so the steps add up to the chord L), cell-centred trilinear sampling of (c, sigma),
// alpha = 1 - exp(-sigma delta) with delta in voxel lengths, exclusive transmittance,
// then the environment layers (sphere far roots, equirectangular bilinear lookups,
// opacity used as alpha) and the background.
//
// Derivatives (Sec. III-E): the forward-mode pass carries the tangent of T and H; the
// adjoint pass re-marches the ray back to front, as Alg. 1 does, and forms per sample
//   dH/dc_k = T_k alpha_k,   dH/dsigma_k = delta_k (T_{k+1} c_k - G_k),
// with G_k (everything composited behind sample k) accumulated from the back and started
// at the environment and background seen from the grid exit (the term Alg. 1 needs for
// the derivative to be exact when layers are visible).  T_k = exp(-V_k) uses the optical
// depth V summed with compensation in the forward pass and stepped back in the adjoint
// pass, so front samples keep T to ~eps*V_total and deep samples keep G to full relative
// precision (forming G as H minus a prefix would lose it behind opaque matter).
//
// Clamp-to-edge trilinear sampling is evaluated with the coordinate clamped to
// [0, n-1] and the lower corner to n-2: identical values and derivatives, and the eight
// corners are always distinct voxels, which the per-ray window of the gradient pass needs.
#include "perf_internal.h"

#include <math.h>

namespace perf {
namespace {

__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

template <int PD>
struct XL;
template <>
struct XL<PERF_F32> {
    const float4* __restrict__ p;
    __device__ __forceinline__ float4 operator()(int i) const { return p[i]; }
};
template <>
struct XL<PERF_BF16> {
    const ushort4* __restrict__ p;
    __device__ __forceinline__ float4 operator()(int i) const {
        ushort4 q = p[i];
        return make_float4(bf16_to_f32(q.x), bf16_to_f32(q.y), bf16_to_f32(q.z), bf16_to_f32(q.w));
    }
};

struct Ray {
    float o[3], d[3];
    float tn, tf, L;
    int K;
    bool hit;
    float g0[3], gd[3];
};

__device__ __forceinline__ void make_ray(const Geo& G, const DevCam& c, int px, int py, Ray& r) {
    const float dcx = ((float)px + 0.5f - c.cx) / c.fx;
    const float dcy = ((float)py + 0.5f - c.cy) / c.fy;
    float d0 = c.R[0] * dcx + c.R[1] * dcy + c.R[2];
    float d1 = c.R[3] * dcx + c.R[4] * dcy + c.R[5];
    float d2 = c.R[6] * dcx + c.R[7] * dcy + c.R[8];
    const float inv = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    r.d[0] = d0 * inv;
    r.d[1] = d1 * inv;
    r.d[2] = d2 * inv;
    r.o[0] = c.o[0];
    r.o[1] = c.o[1];
    r.o[2] = c.o[2];
    float t0 = -INFINITY, t1 = INFINITY;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] == 0.0f) {
            if (r.o[a] < G.bmin[a] || r.o[a] > G.bmax[a]) ok = false;
        } else {
            const float ta = (G.bmin[a] - r.o[a]) / r.d[a];
            const float tb = (G.bmax[a] - r.o[a]) / r.d[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        }
    }
    t0 = fmaxf(t0, 0.0f);
    r.hit = ok && (t1 > t0);
    r.tn = t0;
    r.tf = t1;
    if (r.hit) {
        r.L = (t1 - t0) / G.h;
        r.K = (int)ceilf(r.L / G.step);
    } else {
        r.L = 0.0f;
        r.K = 0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.g0[a] = (r.o[a] + t0 * r.d[a] - G.bmin[a]) * G.inv_hv[a] - 0.5f;
        r.gd[a] = G.h * r.d[a] * G.inv_hv[a];
    }
}

// Sample k of a ray: step length delta and position in grid coordinates.
__device__ __forceinline__ float sample_at(const Geo& G, const Ray& r, int k, float g[3]) {
    const float dk = fmaxf(fminf(G.step, r.L - (float)k * G.step), 0.0f);
    const float s = (float)k * G.step + 0.5f * dk;
    g[0] = r.g0[0] + r.gd[0] * s;
    g[1] = r.g0[1] + r.gd[1] * s;
    g[2] = r.g0[2] + r.gd[2] * s;
    return dk;
}

struct Corners {
    int v;          // lower corner voxel
    int i[3];       // lower corner coordinates
    float w[8];     // weights, corner j = (j&1, j>>1&1, j>>2) offsets
};

__device__ __forceinline__ void corners(const Geo& G, const float g[3], Corners& c) {
    const int n[3] = {G.nx, G.ny, G.nz};
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float gc = fminf(fmaxf(g[a], 0.0f), (float)(n[a] - 1));
        const int i0 = min((int)gc, n[a] - 2);
        c.i[a] = i0;
        f[a] = gc - (float)i0;
    }
    c.v = (c.i[2] * G.ny + c.i[1]) * G.nx + c.i[0];
    const float wx0 = 1.0f - f[0], wx1 = f[0];
    const float wy0 = 1.0f - f[1], wy1 = f[1];
    const float wz0 = 1.0f - f[2], wz1 = f[2];
    const float a00 = wy0 * wz0, a10 = wy1 * wz0, a01 = wy0 * wz1, a11 = wy1 * wz1;
    c.w[0] = wx0 * a00;
    c.w[1] = wx1 * a00;
    c.w[2] = wx0 * a10;
    c.w[3] = wx1 * a10;
    c.w[4] = wx0 * a01;
    c.w[5] = wx1 * a01;
    c.w[6] = wx0 * a11;
    c.w[7] = wx1 * a11;
}

__device__ __forceinline__ int corner_off(int j, int nx, int nxy) { return (j & 1) + ((j >> 1) & 1) * nx + (j >> 2) * nxy; }

struct Tex {
    int t[4];
    float w[4];
};

// Far intersection with layer l beyond tmin and its bilinear equirectangular texels.
__device__ __forceinline__ bool env_hit(const Geo& G, const Ray& r, int l, float tmin, Tex& tx) {
    const float R = G.radius[l];
    const float b = r.o[0] * r.d[0] + r.o[1] * r.d[1] + r.o[2] * r.d[2];
    const float cc = r.o[0] * r.o[0] + r.o[1] * r.o[1] + r.o[2] * r.o[2] - R * R;
    const float disc = b * b - cc;
    if (disc < 0.0f) return false;
    const float t = -b + sqrtf(disc);
    if (!(t > tmin)) return false;
    const float px = r.o[0] + t * r.d[0], py = r.o[1] + t * r.d[1], pz = r.o[2] + t * r.d[2];
    const float kInv2Pi = 0.15915494309189535f, kInvPi = 0.3183098861837907f;
    const int W = G.env_w, Hh = G.env_h;
    const float u = (atan2f(py, px) * kInv2Pi + 0.5f) * (float)W - 0.5f;
    const float v = atan2f(sqrtf(px * px + py * py), pz) * kInvPi * (float)Hh - 0.5f;
    const float fu0 = floorf(u);
    const float fu = u - fu0;
    int i0 = (int)fu0;
    i0 = ((i0 % W) + W) % W;
    const int i1 = (i0 + 1 == W) ? 0 : i0 + 1;
    const float vc = fminf(fmaxf(v, 0.0f), (float)(Hh - 1));
    const int j0 = min((int)vc, Hh - 2);
    const float fv = vc - (float)j0;
    const int base = G.nvox + l * W * Hh + j0 * W;
    tx.t[0] = base + i0;
    tx.t[1] = base + i1;
    tx.t[2] = base + W + i0;
    tx.t[3] = base + W + i1;
    tx.w[0] = (1.0f - fu) * (1.0f - fv);
    tx.w[1] = fu * (1.0f - fv);
    tx.w[2] = (1.0f - fu) * fv;
    tx.w[3] = fu * fv;
    return true;
}

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// ------------------------------------------------------------------ forward pass (+ tangent)
// Optical depth in front of a sample, summed with compensation (Kahan) so that the
// adjoint pass can step it back sample by sample with an error of order eps * V_total.
struct Depth {
    float s, c;  // value ~ s - c
    __device__ __forceinline__ void add(float v) {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ float value() const { return s - c; }
};

template <int PD, bool TAN>
__device__ __forceinline__ void forward(const Geo& G, const Ray& r, XL<PD> X, const float4* __restrict__ V, float H[3],
                                        float& Texit, float Hd[3], Depth& depth) {
    float T = 1.0f, Td = 0.0f;
    depth.s = 0.0f;
    depth.c = 0.0f;
    H[0] = H[1] = H[2] = 0.0f;
    Hd[0] = Hd[1] = Hd[2] = 0.0f;
    const int nx = G.nx, nxy = G.nx * G.ny;
    for (int k = 0; k < r.K; ++k) {
        float g[3];
        const float dk = sample_at(G, r, k, g);
        Corners c;
        corners(G, g, c);
        float sg = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        float sgd = 0.0f, cd0 = 0.0f, cd1 = 0.0f, cd2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int vi = c.v + corner_off(j, nx, nxy);
            const float4 q = X(vi);
            c0 += c.w[j] * q.x;
            c1 += c.w[j] * q.y;
            c2 += c.w[j] * q.z;
            sg += c.w[j] * q.w;
            if constexpr (TAN) {
                const float4 t = V[vi];
                cd0 += c.w[j] * t.x;
                cd1 += c.w[j] * t.y;
                cd2 += c.w[j] * t.z;
                sgd += c.w[j] * t.w;
            }
        }
        const float tau = sg * dk;
        depth.add(tau);
        const float e = expf(-tau);
        const float al = -expm1f(-tau);
        const float Ta = T * al;
        H[0] += Ta * c0;
        H[1] += Ta * c1;
        H[2] += Ta * c2;
        if constexpr (TAN) {
            const float ald = dk * e * sgd;  // d alpha
            const float k1 = Td * al + T * ald;
            Hd[0] += k1 * c0 + Ta * cd0;
            Hd[1] += k1 * c1 + Ta * cd1;
            Hd[2] += k1 * c2 + Ta * cd2;
            Td = Td * e - T * ald;
        }
        T *= e;
    }
    Texit = T;
    const float tmin = r.hit ? r.tf : 0.0f;
    for (int l = 0; l < G.n_layers; ++l) {
        Tex tx;
        if (!env_hit(G, r, l, tmin, tx)) continue;
        float al = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        float ald = 0.0f, cd0 = 0.0f, cd1 = 0.0f, cd2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 q = X(tx.t[j]);
            c0 += tx.w[j] * q.x;
            c1 += tx.w[j] * q.y;
            c2 += tx.w[j] * q.z;
            al += tx.w[j] * q.w;
            if constexpr (TAN) {
                const float4 t = V[tx.t[j]];
                cd0 += tx.w[j] * t.x;
                cd1 += tx.w[j] * t.y;
                cd2 += tx.w[j] * t.z;
                ald += tx.w[j] * t.w;
            }
        }
        const float Ta = T * al;
        H[0] += Ta * c0;
        H[1] += Ta * c1;
        H[2] += Ta * c2;
        if constexpr (TAN) {
            const float k1 = Td * al + T * ald;
            Hd[0] += k1 * c0 + Ta * cd0;
            Hd[1] += k1 * c1 + Ta * cd1;
            Hd[2] += k1 * c2 + Ta * cd2;
            Td = Td * (1.0f - al) - T * ald;
        }
        T *= (1.0f - al);
    }
    H[0] += T * G.bg[0];
    H[1] += T * G.bg[1];
    H[2] += T * G.bg[2];
    if constexpr (TAN) {
        Hd[0] += Td * G.bg[0];
        Hd[1] += Td * G.bg[1];
        Hd[2] += Td * G.bg[2];
    }
}

// ------------------------------------------------------------------ adjoint pass: y += J_ray^T u
// Environment layers first (S, the radiance behind a layer, by the over-recurrence from
// the background), then the voxel samples from the last to the first as in Alg. 1: the
// colour behind sample k, G_k, is accumulated from the back (a sum of T-scaled terms, so
// it keeps its relative precision deep behind opaque matter), and T_k = exp(-V_k) with
// V_k the compensated optical depth stepped back from the total.
template <int PD>
__device__ __forceinline__ float env_adjoint(const Geo& G, const Ray& r, XL<PD> X, const float u[3], float Tx,
                                             float* __restrict__ y) {
    float Tl[kMaxLayers];
    unsigned used = 0;
    float T = Tx;
    const float tmin = r.hit ? r.tf : 0.0f;
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) {
        Tl[l] = 0.0f;
        if (l < G.n_layers) {
            Tex tx;
            if (env_hit(G, r, l, tmin, tx)) {
                float al = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) al += tx.w[j] * X(tx.t[j]).w;
                Tl[l] = T;
                used |= 1u << l;
                T *= (1.0f - al);
            }
        }
    }
    float uS = u[0] * G.bg[0] + u[1] * G.bg[1] + u[2] * G.bg[2];
#pragma unroll
    for (int l = kMaxLayers - 1; l >= 0; --l) {
        if (used & (1u << l)) {
            Tex tx;
            env_hit(G, r, l, tmin, tx);
            float al = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 q = X(tx.t[j]);
                c0 += tx.w[j] * q.x;
                c1 += tx.w[j] * q.y;
                c2 += tx.w[j] * q.z;
                al += tx.w[j] * q.w;
            }
            const float uc = u[0] * c0 + u[1] * c1 + u[2] * c2;
            const float A = Tl[l] * al;              // dH/dc_l
            const float dA = Tl[l] * (uc - uS);      // u . dH/dalpha_l
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float* yy = y + 4 * (size_t)tx.t[j];
                const float wA = tx.w[j] * A;
                atomic_add(yy + 0, wA * u[0]);
                atomic_add(yy + 1, wA * u[1]);
                atomic_add(yy + 2, wA * u[2]);
                atomic_add(yy + 3, tx.w[j] * dA);
            }
            uS = al * uc + (1.0f - al) * uS;
        }
    }
    return uS;  // u . (environment radiance seen from the grid exit)
}

template <int PD>
__device__ __forceinline__ void adjoint_scatter(const Geo& G, const Ray& r, XL<PD> X, const float u[3], Depth depth,
                                                float* __restrict__ y) {
    const float Tx = expf(-depth.value());
    const float uE = env_adjoint<PD>(G, r, X, u, Tx, y);
    float uG = Tx * uE;   // u . G_k, the colour composited behind sample k
    float Tn = Tx;        // T_{k+1}
    const int nx = G.nx, nxy = G.nx * G.ny;
    for (int k = r.K - 1; k >= 0; --k) {
        float g[3];
        const float dk = sample_at(G, r, k, g);
        Corners c;
        corners(G, g, c);
        float sg = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float4 q = X(c.v + corner_off(j, nx, nxy));
            c0 += c.w[j] * q.x;
            c1 += c.w[j] * q.y;
            c2 += c.w[j] * q.z;
            sg += c.w[j] * q.w;
        }
        const float tau = sg * dk;
        depth.add(-tau);
        const float T = (k == 0) ? 1.0f : expf(-depth.value());
        const float al = -expm1f(-tau);
        const float A = T * al;
        const float uc = u[0] * c0 + u[1] * c1 + u[2] * c2;
        const float ds = dk * (Tn * uc - uG);
        uG += A * uc;
        Tn = T;
        const float Au0 = A * u[0], Au1 = A * u[1], Au2 = A * u[2];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float* yy = y + 4 * (size_t)(c.v + corner_off(j, nx, nxy));
            const float w = c.w[j];
            atomic_add(yy + 0, w * Au0);
            atomic_add(yy + 1, w * Au1);
            atomic_add(yy + 2, w * Au2);
            atomic_add(yy + 3, w * ds);
        }
    }
}

// ------------------------------------------------------------------ gradient + exact blocks
// Per-ray window over the current 8 corners.  A voxel is a corner of a contiguous run of
// a ray's samples (its corner region is a box and the ray is a line), so a voxel that
// leaves the window never returns: flushing on leave aggregates the ray's partials per
// voxel exactly before they are squared into the block.
struct Win {
    int i[3];
    float a[8], s0[8], s1[8], s2[8];
};

__device__ __forceinline__ void flush_unit(int unit, float a, float s0, float s1, float s2, const float rr[3],
                                           float* __restrict__ grad, float* __restrict__ blocks) {
    if (a == 0.0f && s0 == 0.0f && s1 == 0.0f && s2 == 0.0f) return;
    if (grad) {
        float* g = grad + 4 * (size_t)unit;
        atomic_add(g + 0, -a * rr[0]);
        atomic_add(g + 1, -a * rr[1]);
        atomic_add(g + 2, -a * rr[2]);
        atomic_add(g + 3, -(s0 * rr[0] + s1 * rr[1] + s2 * rr[2]));
    }
    if (blocks) {
        float* b = blocks + 5 * (size_t)unit;
        atomic_add(b + 0, a * a);
        atomic_add(b + 1, a * s0);
        atomic_add(b + 2, a * s1);
        atomic_add(b + 3, a * s2);
        atomic_add(b + 4, s0 * s0 + s1 * s1 + s2 * s2);
    }
}

__device__ __forceinline__ void win_flush_slot(const Geo& G, Win& w, int b, const float rr[3], float* grad,
                                               float* blocks) {
    const int unit = ((w.i[2] + ((b >> 2) & 1)) * G.ny + (w.i[1] + ((b >> 1) & 1))) * G.nx + (w.i[0] + (b & 1));
    flush_unit(unit, w.a[b], w.s0[b], w.s1[b], w.s2[b], rr, grad, blocks);
}

template <int AX>
__device__ __forceinline__ void win_shift(const Geo& G, Win& w, int target, const float rr[3], float* grad,
                                          float* blocks) {
    constexpr int bit = 1 << AX;
    const int delta = target - w.i[AX];
    if (delta == 0) return;
    if (delta == 1) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            if (!(b & bit)) {
                win_flush_slot(G, w, b, rr, grad, blocks);
                w.a[b] = w.a[b | bit]; w.s0[b] = w.s0[b | bit]; w.s1[b] = w.s1[b | bit]; w.s2[b] = w.s2[b | bit];
                w.a[b | bit] = 0.0f; w.s0[b | bit] = 0.0f; w.s1[b | bit] = 0.0f; w.s2[b | bit] = 0.0f;
            }
        }
    } else if (delta == -1) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            if (b & bit) {
                win_flush_slot(G, w, b, rr, grad, blocks);
                w.a[b] = w.a[b ^ bit]; w.s0[b] = w.s0[b ^ bit]; w.s1[b] = w.s1[b ^ bit]; w.s2[b] = w.s2[b ^ bit];
                w.a[b ^ bit] = 0.0f; w.s0[b ^ bit] = 0.0f; w.s1[b ^ bit] = 0.0f; w.s2[b ^ bit] = 0.0f;
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            win_flush_slot(G, w, b, rr, grad, blocks);
            w.a[b] = 0.0f; w.s0[b] = 0.0f; w.s1[b] = 0.0f; w.s2[b] = 0.0f;
        }
    }
    w.i[AX] = target;
}

template <int PD>
__device__ __forceinline__ void grad_scatter(const Geo& G, const Ray& r, XL<PD> X, const float rr[3], Depth depth,
                                             float* __restrict__ grad, float* __restrict__ blocks) {
    const float Tx = expf(-depth.value());
    float S0 = G.bg[0], S1 = G.bg[1], S2 = G.bg[2];
    // environment layers (the four texels of one lookup are distinct units)
    {
        float Tl[kMaxLayers];
        unsigned used = 0;
        float T = Tx;
        const float tmin = r.hit ? r.tf : 0.0f;
#pragma unroll
        for (int l = 0; l < kMaxLayers; ++l) {
            Tl[l] = 0.0f;
            if (l < G.n_layers) {
                Tex tx;
                if (env_hit(G, r, l, tmin, tx)) {
                    float al = 0.0f;
#pragma unroll
                    for (int j = 0; j < 4; ++j) al += tx.w[j] * X(tx.t[j]).w;
                    Tl[l] = T;
                    used |= 1u << l;
                    T *= (1.0f - al);
                }
            }
        }
#pragma unroll
        for (int l = kMaxLayers - 1; l >= 0; --l) {
            if (used & (1u << l)) {
                Tex tx;
                env_hit(G, r, l, tmin, tx);
                float al = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 q = X(tx.t[j]);
                    c0 += tx.w[j] * q.x;
                    c1 += tx.w[j] * q.y;
                    c2 += tx.w[j] * q.z;
                    al += tx.w[j] * q.w;
                }
                const float A = Tl[l] * al;
                const float d0 = Tl[l] * (c0 - S0), d1 = Tl[l] * (c1 - S1), d2 = Tl[l] * (c2 - S2);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float w = tx.w[j];
                    flush_unit(tx.t[j], w * A, w * d0, w * d1, w * d2, rr, grad, blocks);
                }
                S0 = al * c0 + (1.0f - al) * S0;
                S1 = al * c1 + (1.0f - al) * S1;
                S2 = al * c2 + (1.0f - al) * S2;
            }
        }
    }
    if (r.K <= 0) return;
    Win w;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        w.a[b] = 0.0f; w.s0[b] = 0.0f; w.s1[b] = 0.0f; w.s2[b] = 0.0f;
    }
    // G_k from the back, starting with the environment seen from the grid exit
    float G0 = Tx * S0, G1 = Tx * S1, G2 = Tx * S2;
    float Tn = Tx;
    const int nx = G.nx, nxy = G.nx * G.ny;
    for (int k = r.K - 1; k >= 0; --k) {
        float g[3];
        const float dk = sample_at(G, r, k, g);
        Corners c;
        corners(G, g, c);
        if (k == r.K - 1) {
            w.i[0] = c.i[0]; w.i[1] = c.i[1]; w.i[2] = c.i[2];
        } else {
            win_shift<0>(G, w, c.i[0], rr, grad, blocks);
            win_shift<1>(G, w, c.i[1], rr, grad, blocks);
            win_shift<2>(G, w, c.i[2], rr, grad, blocks);
        }
        float sg = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float4 q = X(c.v + corner_off(j, nx, nxy));
            c0 += c.w[j] * q.x;
            c1 += c.w[j] * q.y;
            c2 += c.w[j] * q.z;
            sg += c.w[j] * q.w;
        }
        const float tau = sg * dk;
        depth.add(-tau);
        const float T = (k == 0) ? 1.0f : expf(-depth.value());
        const float al = -expm1f(-tau);
        const float A = T * al;
        const float ds0 = dk * (Tn * c0 - G0);
        const float ds1 = dk * (Tn * c1 - G1);
        const float ds2 = dk * (Tn * c2 - G2);
        G0 += A * c0;
        G1 += A * c1;
        G2 += A * c2;
        Tn = T;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            w.a[j] += c.w[j] * A;
            w.s0[j] += c.w[j] * ds0;
            w.s1[j] += c.w[j] * ds1;
            w.s2[j] += c.w[j] * ds2;
        }
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) win_flush_slot(G, w, b, rr, grad, blocks);
}

// ------------------------------------------------------------------ features for the learned preconditioner
// Per sample and corner (weight w): sums[unit] += (w, w T, w G (3), w alpha), G = colour behind.
template <int PD>
__device__ __forceinline__ void feature_scatter(const Geo& G, const Ray& r, XL<PD> X, const float H[3], float Texit,
                                                float* __restrict__ sums) {
    {
        float T = Texit;
        float Tl[kMaxLayers], Al[kMaxLayers];
        unsigned used = 0;
        const float tmin = r.hit ? r.tf : 0.0f;
#pragma unroll
        for (int l = 0; l < kMaxLayers; ++l) {
            Tl[l] = 0.0f;
            Al[l] = 0.0f;
            if (l < G.n_layers) {
                Tex tx;
                if (env_hit(G, r, l, tmin, tx)) {
                    float al = 0.0f;
#pragma unroll
                    for (int j = 0; j < 4; ++j) al += tx.w[j] * X(tx.t[j]).w;
                    Tl[l] = T;
                    Al[l] = al;
                    used |= 1u << l;
                    T *= (1.0f - al);
                }
            }
        }
        float S0 = G.bg[0], S1 = G.bg[1], S2 = G.bg[2];
#pragma unroll
        for (int l = kMaxLayers - 1; l >= 0; --l) {
            if (used & (1u << l)) {
                Tex tx;
                env_hit(G, r, l, tmin, tx);
                float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 q = X(tx.t[j]);
                    c0 += tx.w[j] * q.x;
                    c1 += tx.w[j] * q.y;
                    c2 += tx.w[j] * q.z;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float* s = sums + 6 * (size_t)tx.t[j];
                    const float w = tx.w[j];
                    atomic_add(s + 0, w);
                    atomic_add(s + 1, w * Tl[l]);
                    atomic_add(s + 2, w * S0);
                    atomic_add(s + 3, w * S1);
                    atomic_add(s + 4, w * S2);
                    atomic_add(s + 5, w * Al[l]);
                }
                const float al = Al[l];
                S0 = al * c0 + (1.0f - al) * S0;
                S1 = al * c1 + (1.0f - al) * S1;
                S2 = al * c2 + (1.0f - al) * S2;
            }
        }
    }
    float T = 1.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
    const int nx = G.nx, nxy = G.nx * G.ny;
    for (int k = 0; k < r.K; ++k) {
        float g[3];
        const float dk = sample_at(G, r, k, g);
        Corners c;
        corners(G, g, c);
        float sg = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float4 q = X(c.v + corner_off(j, nx, nxy));
            c0 += c.w[j] * q.x;
            c1 += c.w[j] * q.y;
            c2 += c.w[j] * q.z;
            sg += c.w[j] * q.w;
        }
        const float tau = sg * dk;
        const float e = expf(-tau);
        const float al = -expm1f(-tau);
        const float A = T * al;
        const float G0 = H[0] - P0 - A * c0, G1 = H[1] - P1 - A * c1, G2 = H[2] - P2 - A * c2;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float* s = sums + 6 * (size_t)(c.v + corner_off(j, nx, nxy));
            const float w = c.w[j];
            atomic_add(s + 0, w);
            atomic_add(s + 1, w * T);
            atomic_add(s + 2, w * G0);
            atomic_add(s + 3, w * G1);
            atomic_add(s + 4, w * G2);
            atomic_add(s + 5, w * al);
        }
        P0 += A * c0;
        P1 += A * c1;
        P2 += A * c2;
        T *= e;
    }
}

// ------------------------------------------------------------------ workgroup FP64 sum
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void block_sum_store(double v, double* out) {
    __shared__ double red[kBlock / 64];
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
        *out = s;
    }
}

struct Pix {
    int cam, px, py;
    bool active;
    long long ray;
};

__device__ __forceinline__ Pix pixel_of(const Geo& G) {
    Pix p;
    const int b = blockIdx.x;
    p.cam = b / G.n_tiles;
    const int tile = b - p.cam * G.n_tiles;
    const int ty = tile / G.tiles_x, tx = tile - ty * G.tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    p.px = tx * kTile + (wave & 1) * 8 + (lane & 7);
    p.py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
    p.active = p.px < G.width && p.py < G.height;
    p.ray = ((long long)p.cam * G.height + p.py) * G.width + p.px;
    return p;
}

template <int MODE, int PD>
__global__ __launch_bounds__(kBlock) void k_ray(Geo G, RayArgs A) {
    if (A.done && *A.done) return;
    const Pix p = pixel_of(G);
    XL<PD> X;
    X.p = reinterpret_cast<decltype(X.p)>(A.x);
    double rr_sum = 0.0;
    if (p.active) {
        Ray r;
        make_ray(G, A.cams[p.cam], p.px, p.py, r);
        float H[3], Hd[3], Texit;
        Depth depth;
        if constexpr (MODE == M_JVP || MODE == M_JTJ) {
            forward<PD, true>(G, r, X, reinterpret_cast<const float4*>(A.v), H, Texit, Hd, depth);
        } else {
            forward<PD, false>(G, r, X, nullptr, H, Texit, Hd, depth);
        }
        if constexpr (MODE == M_RENDER) {
            if (A.targets) {
                float res[3];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    res[ch] = H[ch] - A.targets[3 * p.ray + ch];
                    rr_sum += (double)res[ch] * (double)res[ch];
                }
                if (A.rout) {
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) A.rout[3 * p.ray + ch] = res[ch];
                }
            } else if (A.rout) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) A.rout[3 * p.ray + ch] = H[ch];
            }
        } else if constexpr (MODE == M_JVP) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) A.rout[3 * p.ray + ch] = Hd[ch];
        } else if constexpr (MODE == M_VJP) {
            const float u[3] = {A.uin[3 * p.ray], A.uin[3 * p.ray + 1], A.uin[3 * p.ray + 2]};
            adjoint_scatter<PD>(G, r, X, u, depth, A.y);
        } else if constexpr (MODE == M_JTJ) {
            adjoint_scatter<PD>(G, r, X, Hd, depth, A.y);
        } else if constexpr (MODE == M_GRAD) {
            float res[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                res[ch] = H[ch] - A.targets[3 * p.ray + ch];
                rr_sum += (double)res[ch] * (double)res[ch];
            }
            grad_scatter<PD>(G, r, X, res, depth, A.y, A.blocks);
        } else if constexpr (MODE == M_FEAT) {
            feature_scatter<PD>(G, r, X, H, Texit, A.y);
        }
    }
    if constexpr (MODE == M_RENDER || MODE == M_GRAD) {
        if (A.partials) block_sum_store(rr_sum, A.partials + blockIdx.x);
    }
}

// ------------------------------------------------------------------ footprint counts
// Distinct clamp-to-edge corner voxels of all samples of a ray: a voxel's membership is a
// contiguous run of samples, so the count is the sum over samples of the corners not
// already corners of the previous sample (per-axis sets of one or two indices).
__global__ __launch_bounds__(kBlock) void k_footprint(Geo G, const DevCam* cams, int32_t* per_ray,
                                                      unsigned long long* totals) {
    const Pix p = pixel_of(G);
    unsigned long long U = 0, nl = 0, hit = 0;
    if (p.active) {
        Ray r;
        make_ray(G, cams[p.cam], p.px, p.py, r);
        const int n[3] = {G.nx, G.ny, G.nz};
        int prev_lo[3] = {0, 0, 0}, prev_hi[3] = {-1, -1, -1};
        for (int k = 0; k < r.K; ++k) {
            float g[3];
            sample_at(G, r, k, g);
            int lo[3], hi[3], cnt = 1, inter = 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int i0 = (int)floorf(g[a]);
                lo[a] = min(max(i0, 0), n[a] - 1);
                hi[a] = min(max(i0 + 1, 0), n[a] - 1);
                cnt *= (hi[a] - lo[a] + 1);
                const int ilo = max(lo[a], prev_lo[a]), ihi = min(hi[a], prev_hi[a]);
                inter *= max(ihi - ilo + 1, 0);
            }
            U += (unsigned long long)(cnt - inter);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                prev_lo[a] = lo[a];
                prev_hi[a] = hi[a];
            }
        }
        const float tmin = r.hit ? r.tf : 0.0f;
        for (int l = 0; l < G.n_layers; ++l) {
            Tex tx;
            if (env_hit(G, r, l, tmin, tx)) ++nl;
        }
        hit = r.K > 0 ? 1 : 0;
        if (per_ray) {
            per_ray[2 * p.ray] = (int32_t)U;
            per_ray[2 * p.ray + 1] = (int32_t)nl;
        }
    }
    if (totals) {
        __shared__ unsigned long long red[3];
        if (threadIdx.x < 3) red[threadIdx.x] = 0;
        __syncthreads();
        if (U) atomicAdd(&red[0], U);
        if (nl) atomicAdd(&red[1], nl);
        if (hit) atomicAdd(&red[2], hit);
        __syncthreads();
        if (threadIdx.x < 3 && red[threadIdx.x]) atomicAdd(&totals[threadIdx.x], red[threadIdx.x]);
    }
}

template <int MODE, int PD>
hipError_t launch_one(const Geo& g, const RayArgs& a, hipStream_t st) {
    const unsigned grid = (unsigned)((long long)g.n_cams * g.n_tiles);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_ray<MODE, PD>), dim3(grid), dim3(kBlock), 0, st, g, a);
    return hipGetLastError();
}

template <int PD>
hipError_t launch_mode(int mode, const Geo& g, const RayArgs& a, hipStream_t st) {
    switch (mode) {
        case M_RENDER: return launch_one<M_RENDER, PD>(g, a, st);
        case M_JVP: return launch_one<M_JVP, PD>(g, a, st);
        case M_VJP: return launch_one<M_VJP, PD>(g, a, st);
        case M_JTJ: return launch_one<M_JTJ, PD>(g, a, st);
        case M_GRAD: return launch_one<M_GRAD, PD>(g, a, st);
        case M_FEAT: return launch_one<M_FEAT, PD>(g, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_ray(int mode, int param_dtype, const Geo& g, const RayArgs& a, hipStream_t st) {
    if (param_dtype == PERF_BF16) return launch_mode<PERF_BF16>(mode, g, a, st);
    return launch_mode<PERF_F32>(mode, g, a, st);
}

hipError_t launch_footprint(const Geo& g, const DevCam* cams, int32_t* per_ray, unsigned long long* totals,
                            hipStream_t st) {
    const unsigned grid = (unsigned)((long long)g.n_cams * g.n_tiles);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_footprint, dim3(grid), dim3(kBlock), 0, st, g, cams, per_ray, totals);
    return hipGetLastError();
}

hipError_t launch_features(int param_dtype, const Geo& g, const DevCam* cams, const void* x, float* sums,
                           hipStream_t st) {
    RayArgs a{};
    a.cams = cams;
    a.x = x;
    a.y = sums;
    return launch_ray(M_FEAT, param_dtype, g, a, st);
}

}  // namespace perf
