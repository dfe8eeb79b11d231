// Per-ray kernels of the Gauss-Newton step on gfx950.
//
// One lane marches one pixel ray; a 128-thread workgroup owns a 16x8 pixel tile of one
// camera and each wave64 an 8x8 half of it.  The lanes of a wave march their rays in step
// at matched depths, so their trilinear gathers hit the same cache lines and their
// scatter lands in one small voxel window that the wave combines in LDS before HBM.
//
// Per ray (Sec. III-A, Eq. 3-4): slab test against the grid box, K = ceil(L / step)
// samples at the midpoints of equal steps of `step` voxel lengths (the last one shortened
// so the steps add up to the chord L), cell-centred trilinear sampling of (c, sigma),
// alpha = 1 - exp(-sigma delta) with delta in voxel lengths, exclusive transmittance,
// then the environment layers (sphere far roots, equirectangular bilinear lookups,
// opacity used as alpha) and the background.  With jittering (Sec. IV) the ray starts at
// a pseudo-random point of its pixel and each sample sits at a pseudo-random point of its
// step.  The optional auxiliary residual (Sec. III-I, Eq. 10) is a fourth residual per ray
// that depends on the transmittance through the volume only.
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

// Loads of parameter and tangent vectors go through buffer resources: the voxel's byte offset is
// one 32-bit VGPR and the trilinear corner's offset (a multiple of the row and slice pitch, the
// same for every lane) an SGPR, so a corner costs one load and no 64-bit address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

struct VecF4 {  // FP32 float4 per unit
    __amdgpu_buffer_rsrc_t r;
    static constexpr int kBytes = 16;
    __device__ __forceinline__ float4 load(int voff, int soff) const {
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        return make_float4(__int_as_float((int)q[0]), __int_as_float((int)q[1]), __int_as_float((int)q[2]),
                           __int_as_float((int)q[3]));
    }
    __device__ __forceinline__ float4 operator()(int i) const { return load(i * kBytes, 0); }
};

template <int PD>
struct XL;
template <>
struct XL<PERF_F32> : VecF4 {};
template <>
struct XL<PERF_BF16> {  // bfloat16 x 4 per unit
    __amdgpu_buffer_rsrc_t r;
    static constexpr int kBytes = 8;
    __device__ __forceinline__ float4 load(int voff, int soff) const {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        const unsigned a = (unsigned)q[0], b = (unsigned)q[1];
        return make_float4(__uint_as_float(a << 16), __uint_as_float(a & 0xffff0000u), __uint_as_float(b << 16),
                           __uint_as_float(b & 0xffff0000u));
    }
    __device__ __forceinline__ float4 operator()(int i) const { return load(i * kBytes, 0); }
};

struct Ray {
    float o[3], d[3];
    float tn, tf, L;
    int K;
    bool hit;
    unsigned jkey;  // the ray's jittering key (when jittering is on)
    float g0[3], gd[3];
    const DevCam* cam;  // the camera (uniform over a workgroup)
    int px, py;         // the pixel
    float ox, oy;       // the ray's point inside the pixel (0.5, 0.5 at the centre)
};

// Jittering (Sec. IV): uniform numbers in [0, 1) from a counter-based generator, the 32-bit
// finaliser of MurmurHash3 (Appleby), keyed by (seed, ray, stream): streams 0 and 1 are the
// sub-pixel offsets, stream 2 + k the position of sample k inside its step.  (h >> 8) 2^-24
// is exact in single precision.
__device__ __forceinline__ unsigned fmix32(unsigned h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
__device__ __forceinline__ float jitter_u(unsigned key, unsigned stream) {
    return (float)(fmix32(key + stream * 0x9e3779b9u) >> 8) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ void make_ray(const Geo& G, const DevCam& c, int px, int py, long long ray, Ray& r) {
    float ox = 0.5f, oy = 0.5f;
    r.jkey = 0u;
    if (G.jseed) {
        r.jkey = fmix32(fmix32(G.jseed) ^ (unsigned)ray);
        ox = jitter_u(r.jkey, 0u);
        oy = jitter_u(r.jkey, 1u);
    }
    r.cam = &c;
    r.px = px;
    r.py = py;
    r.ox = ox;
    r.oy = oy;
    const float dcx = ((float)px + ox - c.cx) / c.fx;
    const float dcy = ((float)py + oy - c.cy) / c.fy;
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
    // the step's midpoint, or with jittering a uniform point of the step itself
    const float u = G.jseed ? jitter_u(r.jkey, 2u + (unsigned)k) : 0.5f;
    const float s = (float)k * G.step + u * dk;
    g[0] = r.g0[0] + r.gd[0] * s;
    g[1] = r.g0[1] + r.gd[1] * s;
    g[2] = r.g0[2] + r.gd[2] * s;
    return dk;
}

struct Corners {
    int v;          // lower corner voxel
    int i[3];       // lower corner coordinates
    float f[3];     // fractional position inside the cell
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
        c.f[a] = f[a];
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

// the lower-corner voxel corners() would give for the grid coordinates g
__device__ __forceinline__ int cell_key(const Geo& G, const float g[3]) {
    const int n[3] = {G.nx, G.ny, G.nz};
    int i[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) i[a] = min((int)fminf(fmaxf(g[a], 0.0f), (float)(n[a] - 1)), n[a] - 2);
    return (i[2] * G.ny + i[1]) * G.nx + i[0];
}

__device__ __forceinline__ int corner_off(int j, int nx, int nxy) { return (j & 1) + ((j >> 1) & 1) * nx + (j >> 2) * nxy; }

struct Tex {
    int t[4];
    float w[4];
};

// Far intersection with layer l beyond tmin and its bilinear equirectangular texels.  In double
// precision from the camera and the pixel: a texel coordinate is an angle times W / 2 pi texels
// per radian, so single precision (a rounded ray direction, then u near W) would move the
// bilinear weights by about W * 1e-7.  A few of these per ray cost little beside the march.
__device__ __forceinline__ bool env_hit(const Geo& G, const Ray& r, int l, float tmin, Tex& tx) {
    // the layer's radius by selects: a computed index into the kernel-argument struct would
    // move the whole struct to scratch memory
    float Rf = G.radius[0];
#pragma unroll
    for (int q = 1; q < kMaxLayers; ++q) Rf = (l == q) ? G.radius[q] : Rf;
    const DevCam& c = *r.cam;
    const double dcx = ((double)r.px + (double)r.ox - (double)c.cx) / (double)c.fx;
    const double dcy = ((double)r.py + (double)r.oy - (double)c.cy) / (double)c.fy;
    const double D0 = (double)c.R[0] * dcx + (double)c.R[1] * dcy + (double)c.R[2];
    const double D1 = (double)c.R[3] * dcx + (double)c.R[4] * dcy + (double)c.R[5];
    const double D2 = (double)c.R[6] * dcx + (double)c.R[7] * dcy + (double)c.R[8];
    const double o0 = c.o[0], o1 = c.o[1], o2 = c.o[2], R = Rf;
    // |o + s D| = R with D unnormalised: a s^2 + 2 b s + cc = 0, far root; t = s |D|
    const double a = D0 * D0 + D1 * D1 + D2 * D2;
    const double b = o0 * D0 + o1 * D1 + o2 * D2;
    const double cc = o0 * o0 + o1 * o1 + o2 * o2 - R * R;
    const double disc = b * b - a * cc;
    if (disc < 0.0) return false;
    const double sroot = (-b + sqrt(disc)) / a;
    if (!(sroot * sqrt(a) > (double)tmin)) return false;
    const double px = o0 + sroot * D0, py = o1 + sroot * D1, pz = o2 + sroot * D2;
    const double kInv2Pi = 0.15915494309189535, kInvPi = 0.3183098861837907;
    const int W = G.env_w, Hh = G.env_h;
    const double u = (atan2(py, px) * kInv2Pi + 0.5) * (double)W - 0.5;
    const double v = atan2(sqrt(px * px + py * py), pz) * kInvPi * (double)Hh - 0.5;
    const double fu0 = floor(u);
    const float fu = (float)(u - fu0);
    int i0 = (int)fu0;
    i0 = ((i0 % W) + W) % W;
    const int i1 = (i0 + 1 == W) ? 0 : i0 + 1;
    const double vc = fmin(fmax(v, 0.0), (double)(Hh - 1));
    const int j0 = min((int)vc, Hh - 2);
    const float fv = (float)(vc - (double)j0);
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

// exp(-t) from the hardware base-2 exponential, 2^(-t log2 e): v_exp_f32 is accurate to
// about an ulp of its result, and rounding t log2 e moves the exponent by at most t ulp,
// so the relative error stays near (1 + t) * 6e-8.
__device__ __forceinline__ float exp_neg(float t) { return __builtin_amdgcn_exp2f(-t * 1.4426950408889634f); }

// alpha = 1 - exp(-t) given e = exp(-t).  For |t| < 1/4 the difference 1 - e cancels, so
// the truncated series t (1 - t/2 + t^2/6 - t^3/24 + t^4/120 - t^5/720) is used instead
// (truncation error below t^6/5040 relative, 5e-8 at t = 1/4); above it 1 - e loses at most
// a factor e/(1-e) < 3.6 on the relative error of e.
__device__ __forceinline__ float one_minus_exp_neg(float t, float e) {
    const float series =
        t * (1.0f - t * (0.5f - t * (0.16666667f - t * (0.041666668f - t * (0.008333334f - t * 0.0013888889f)))));
    return fabsf(t) < 0.25f ? series : 1.0f - e;
}

// ------------------------------------------------------------------ lane swaps (DPP)
// Value of lane ^ 1 (quad permutation 1,0,3,2), of lane ^ 2 (quad permutation 2,3,0,1) and of
// lane ^ 8 (rotation by 8 inside each row of 16 lanes).  Called with every lane of the wave active.
__device__ __forceinline__ int dpp_xor1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_xor2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_row_xor8(int v) { return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true); }
__device__ __forceinline__ float dpp_xor1(float v) { return __int_as_float(dpp_xor1(__float_as_int(v))); }
__device__ __forceinline__ float dpp_row_xor8(float v) { return __int_as_float(dpp_row_xor8(__float_as_int(v))); }

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ bool wave_any(bool b) { return __ballot(b) != 0ull; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ void lds_add(__attribute__((address_space(3))) float* p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ float lds_take(__attribute__((address_space(3))) float* p) {
    return __hip_atomic_exchange(p, 0.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// ------------------------------------------------------------------ per-wave scatter combining
// An 8x8x8 voxel window held in LDS as a ring buffer (voxel (x,y,z) lives in slot
// (x&7, y&7, z&7)), one window per wave.  The lanes of a wave march neighbouring rays at
// matched depths, so every step's trilinear corners fall inside the window and are added
// there; when the wave moves on, the voxels that leave the window are flushed to HBM with
// one global atomic per channel (non-zero voxels only) and their slots cleared.  Each voxel
// a wave touches then costs one flush instead of one global atomic per sample, corner and
// ray.  Lanes whose corners do not fit go straight to global atomics.
constexpr int kB = 8;
constexpr int kB3 = kB * kB * kB;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f4 dpp_xor1(f4 v) { return f4{dpp_xor1(v.x), dpp_xor1(v.y), dpp_xor1(v.z), dpp_xor1(v.w)}; }
__device__ __forceinline__ f4 dpp_row_xor8(f4 v) {
    return f4{dpp_row_xor8(v.x), dpp_row_xor8(v.y), dpp_row_xor8(v.z), dpp_row_xor8(v.w)};
}

// Folding of a 2x2 lane quad before an election: a lane hands its value to its x neighbour
// (lane ^ 1), then to its y neighbour (lane ^ 8), then across the quad's diagonal (lane ^ 9),
// each time when both are still in the election and sit in the same cell (same key); the
// higher lane of a pair gives.  Every lane of the wave must run it (DPP swaps).
struct QuadFolds {
    bool give_x, give_y, give_d, keep;
};
__device__ __forceinline__ QuadFolds quad_folds(bool mine, int cell) {
    const int lane = lane_id();
    const int key = mine ? cell : -1;
    QuadFolds q;
    q.give_x = mine & (dpp_xor1(key) == key) & ((lane & 1) != 0);
    const bool keep_x = mine & !q.give_x;
    const int k2 = keep_x ? key : -1;
    q.give_y = keep_x & (dpp_row_xor8(k2) == k2) & ((lane & 8) != 0);
    const bool keep_y = keep_x & !q.give_y;
    const int k3 = keep_y ? key : -1;
    q.give_d = keep_y & (dpp_row_xor8(dpp_xor1(k3)) == k3) & ((lane & 8) != 0);
    q.keep = keep_y & !q.give_d;
    return q;
}
// explicit LDS pointers, so accesses compile to ds_* instructions rather than flat ones
#define LDS __attribute__((address_space(3)))
typedef LDS f4 lds_f4;
typedef LDS f2 lds_f2;
typedef LDS float lds_float;
typedef LDS int lds_int;
typedef LDS unsigned char lds_u8;

__device__ __forceinline__ int ring_slot(int x, int y, int z) {
    return ((z & (kB - 1)) * kB + (y & (kB - 1))) * kB + (x & (kB - 1));
}

// Corner order of the elected scatters.  The 2x2 lane quad to the right of another visits corner
// k + 2 in the round where that one visits corner k, the quad below it corner k + 1.  Two
// face-adjacent cells then never update one voxel in the same round, except when the right-hand
// quad's cell lies at -y or the lower quad's at -x; mirroring the corners' y offset when the
// camera's right vector points to -y, and their x offset when its down vector points to -x,
// removes those cases.  This mask holds the mirrored axes.
__device__ __forceinline__ int corner_mask(const DevCam& c) { return (c.R[1] < 0.0f ? 1 : 0) | (c.R[3] < 0.0f ? 2 : 0); }

// Window bookkeeping shared by the accumulator kinds: origin, fit and slab iteration.
struct Window {
    int o[3];  // window origin (voxel coordinates), wave-uniform
    __device__ __forceinline__ bool inside(const int lo[3], const int hi[3]) const {
        return lo[0] >= o[0] && hi[0] < o[0] + kB && lo[1] >= o[1] && hi[1] < o[1] + kB && lo[2] >= o[2] &&
               hi[2] < o[2] + kB;
    }
    // coordinate of the window along axis a that sits in ring slot sa
    __device__ __forceinline__ int coord(int a, int sa) const { return o[a] + ((sa - o[a]) & (kB - 1)); }
    // flush(x, y, z) for every window voxel, one per lane per round
    template <class Flush>
    __device__ __forceinline__ void each_voxel(Flush& flush) const {
        for (int i = lane_id(); i < kB3; i += 64) {
            const int sx = i & (kB - 1), sy = (i >> 3) & (kB - 1), sz = i >> 6;
            flush(coord(0, sx), coord(1, sy), coord(2, sz));
        }
    }
    template <class Flush>
    __device__ __forceinline__ void move_axis(int a, int no, Flush& flush) {
        const int d = no - o[a];
        if (d == 0) return;
        if (d >= kB || d <= -kB) {
            each_voxel(flush);
        } else {
            const int first = d > 0 ? o[a] : o[a] + kB + d;
            const int cnt = d > 0 ? d : -d;
            const int p = lane_id() & (kB - 1), q = lane_id() >> 3;
            const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
            const int v1 = coord(b1, p), v2 = coord(b2, q);
            for (int t = 0; t < cnt; ++t) {
                int c[3];
                c[a] = first + t;
                c[b1] = v1;
                c[b2] = v2;
                flush(c[0], c[1], c[2]);
            }
        }
        o[a] = no;
    }
    // Make the window cover the corner boxes [lo, hi] of every lane that is on.
    template <class Flush>
    __device__ __forceinline__ void fit(bool on, const int lo[3], const int hi[3], Flush& flush) {
        const bool fits = !on || inside(lo, hi);
        if (!wave_any(!fits)) return;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int mn = wave_min_i(on ? lo[a] : (1 << 30));
            const int mx = wave_max_i(on ? hi[a] : -(1 << 30));
            if (mn > mx) continue;  // no lane on
            int no = o[a];
            if (mx - mn < kB) {
                if (mn < no) no = mn;
                else if (mx > no + kB - 1) no = mx - kB + 1;
            } else if (mn < no || mn > no + kB - 1) {
                no = mn;  // cannot cover every lane: keep the low end, the rest go to HBM
            }
            move_axis(a, no, flush);
        }
    }
};

// The J^T accumulator: float4 (three colour channels and sigma) per window voxel.  LDS
// float atomics are slow on this hardware even without address conflicts, so updates are
// plain read-modify-writes by one elected lane per slot: every pending lane writes its lane
// id into the slot's tag and reads the tag and the slot back in one batch; the lanes that
// read their own id own a distinct slot this round and write the sum, the others retry.
// Lanes of one cell are folded into one (quad_folds); lanes of neighbouring cells visit
// the corners in orders chosen so that they target different voxels in the same round.
struct Brick4 {
    Window win;
    int cmask;            // corner-order mirror of the camera (corner_mask)
    volatile lds_f4* s;   // [kB3]
    volatile lds_u8* tag; // [kB3] lane ids

    __device__ __forceinline__ void init(f4* sb, unsigned char* tb) {
        s = (volatile lds_f4*)sb;
        tag = (volatile lds_u8*)tb;
        win.o[0] = win.o[1] = win.o[2] = -(1 << 24);
        for (int i = lane_id(); i < kB3; i += 64) s[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // Flush one leaving voxel per lane (a uniform call: every lane holds one).  Where most voxels
    // of the pass carry all four channels (a medium with some density everywhere), the adds go
    // out four lanes per voxel, one channel each, so a voxel's four adds form one 16-byte run and
    // the L2 sees about a quarter of the atomic requests; where most carry only the sigma channel
    // (empty space: alpha = 0 zeroes the colour channels), each lane sends its own nonzero channels.
    template <class Sink>
    __device__ __forceinline__ void flush_voxel(const Geo& G, int x, int y, int z, Sink& out) {
        const int sl = ring_slot(x, y, z);
        const f4 v = s[sl];
        const bool in = x >= 0 && y >= 0 && z >= 0 && x < G.nx && y < G.ny && z < G.nz;
        const int u = (z * G.ny + y) * G.nx + x;
        const bool full = in && v.x != 0.0f && v.y != 0.0f && v.z != 0.0f && v.w != 0.0f;
        if (__popcll(__ballot(full)) >= 32) {
            const int ch = lane_id() & 3;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int j = g * 16 + (lane_id() >> 2);
                const int uj = __shfl(u, j, 64);
                const int slj = __shfl(sl, j, 64);
                const int inj = __shfl(in ? 1 : 0, j, 64);
                const float f = ((volatile lds_float*)s)[4 * slj + ch];
                if (inj && f != 0.0f) out.one(uj, ch, f);
            }
        } else if (in && (v.x != 0.0f || v.y != 0.0f || v.z != 0.0f || v.w != 0.0f)) {
            const float vv[4] = {v.x, v.y, v.z, v.w};
            out(u, vv);
        }
        s[sl] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    __device__ __forceinline__ void clear_head(int n) {
        for (int i = lane_id(); i < n; i += 64) s[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    template <class Sink>
    __device__ __forceinline__ void fit(const Geo& G, bool on, const int lo[3], const int hi[3], Sink& out) {
        auto fl = [&](int x, int y, int z) { flush_voxel(G, x, y, z, out); };
        win.fit(on, lo, hi, fl);
    }
    template <class Sink>
    __device__ __forceinline__ void flush_all(const Geo& G, Sink& out) {
        auto fl = [&](int x, int y, int z) { flush_voxel(G, x, y, z, out); };
        win.each_voxel(fl);
    }
    // add val * weight(corner) to the 8 corners of every lane that is on (uniform call).
    // Lanes of one grid cell share all eight corners.  Before the election, the lanes of a
    // 2x2 quad that sit in one cell fold their contributions into one lane (quad_folds, DPP
    // lane swaps), so one lane per group enters the election.  Lanes of different cells
    // never target one voxel with the same corner index, so every lane of a 2x2 lane quad
    // visits the corners in the same order, rotated per quad (and mirrored per camera,
    // corner_mask) so that neighbouring quads update different voxels in the same round.
    template <class Sink>
    __device__ __forceinline__ void scatter8(const Geo& G, bool on, bool inb, const Corners& c, f4 val, bool two,
                                             f4 val2, const float f2[3], Sink& out) {
        // two: a second sample of the same cell (fractional position f2) is added with this one
        const float v2x0 = 1.0f - f2[0], v2y0 = 1.0f - f2[1], v2z0 = 1.0f - f2[2];
        auto w2_of = [&](int i) {
            return two ? ((i & 1) ? f2[0] : v2x0) * ((i & 2) ? f2[1] : v2y0) * ((i & 4) ? f2[2] : v2z0) : 0.0f;
        };
        if (wave_any(on && !inb)) {  // corners outside the window: straight to HBM
            if (on && !inb) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = c.i[0] + (i & 1), y = c.i[1] + ((i >> 1) & 1), z = c.i[2] + (i >> 2);
                    const f4 add = val * c.w[i] + val2 * w2_of(i);
                    const float vv[4] = {add.x, add.y, add.z, add.w};
                    out((z * G.ny + y) * G.nx + x, vv);
                }
            }
        }
        const bool mine = on && inb;
        if (!wave_any(mine)) return;
        const int lane = lane_id();
        const unsigned char tag_id = (unsigned char)lane;
        // The swaps run in straight-line code with every lane active: a lane swap executed
        // under a partial mask would read the other lane's register as it was last written.
        const QuadFolds q = quad_folds(mine, c.v);
        const int phi = ((((lane & 7) >> 1) << 1) + (lane >> 4)) & 7;
        const int sx0 = c.i[0] & 7, sx1 = (c.i[0] + 1) & 7;
        const int sy0 = (c.i[1] & 7) << 3, sy1 = ((c.i[1] + 1) & 7) << 3;
        const int sz0 = (c.i[2] & 7) << 6, sz1 = ((c.i[2] + 1) & 7) << 6;
        const float wx0 = 1.0f - c.f[0], wy0 = 1.0f - c.f[1], wz0 = 1.0f - c.f[2];
        // the next corner's slot and value are formed while this corner's first round waits on LDS
        auto corner = [&](int r, int& sl, f4& add) {
            const int i = ((r + phi) & 7) ^ cmask;
            const bool bx = i & 1, by = i & 2, bz = i & 4;
            sl = (bz ? sz1 : sz0) + (by ? sy1 : sy0) + (bx ? sx1 : sx0);
            const float w = mine ? (bx ? c.f[0] : wx0) * (by ? c.f[1] : wy0) * (bz ? c.f[2] : wz0) : 0.0f;
            const float w2 = mine ? w2_of(i) : 0.0f;
            const f4 a0 = val * w + val2 * w2;
            {
#pragma clang fp contract(off)
                add = a0;
                // a donor hands its value over; every other lane hands over zero
                const f4 zero = f4{0.0f, 0.0f, 0.0f, 0.0f};
                add += dpp_xor1(q.give_x ? add : zero);
                add += dpp_row_xor8(q.give_y ? add : zero);
                add += dpp_row_xor8(dpp_xor1(q.give_d ? add : zero));
            }
        };
        int sl;
        f4 add;
        corner(0, sl, add);
#pragma unroll 1
        for (int r = 0; r < 8; ++r) {
            bool pend = q.keep;
            unsigned char t = 0;
            f4 cur = f4{0.0f, 0.0f, 0.0f, 0.0f};
            if (pend) {
                tag[sl] = tag_id;
                t = tag[sl];
                cur = s[sl];
            }
            int sl_n = 0;
            f4 add_n = f4{0.0f, 0.0f, 0.0f, 0.0f};
            if (r < 7) corner(r + 1, sl_n, add_n);
            if (pend && t == tag_id) {
                s[sl] = cur + add;
                pend = false;
            }
            while (wave_any(pend)) {
                if (pend) {
                    tag[sl] = tag_id;
                    // read the slot with the tag, so a round waits on LDS once
                    const unsigned char t2 = tag[sl];
                    const f4 c2 = s[sl];
                    if (t2 == tag_id) {
                        s[sl] = c2 + add;
                        pend = false;
                    }
                }
            }
            sl = sl_n;
            add = add_n;
        }
    }
};

// Accumulator with NCH scalar channels updated by LDS atomics: the gradient pass flushes
// per-ray window sums that many lanes of a wave hand over for one voxel at the same step,
// where atomics serialise more cheaply than elections.
template <int NCH>
struct BrickAtomic {
    Window win;
    lds_float* s;  // [NCH][kB3]

    __device__ __forceinline__ void init(float* base) {
        s = (lds_float*)base;
        win.o[0] = win.o[1] = win.o[2] = -(1 << 24);
        for (int i = lane_id(); i < NCH * kB3; i += 64) s[i] = 0.0f;
    }
    __device__ __forceinline__ bool inside(const int lo[3], const int hi[3]) const { return win.inside(lo, hi); }
    // zero the first n floats (the texel table's keys after its flush)
    __device__ __forceinline__ void clear_head(int n) {
        for (int i = lane_id(); i < n; i += 64) s[i] = 0.0f;
    }
    __device__ __forceinline__ void add(int x, int y, int z, const float v[NCH]) {
        const int sl = ring_slot(x, y, z);
#pragma unroll
        for (int c = 0; c < NCH; ++c) lds_add(s + c * kB3 + sl, v[c]);
    }
    template <class F>
    __device__ __forceinline__ void flush_voxel(const Geo& G, int x, int y, int z, F& out) {
        const int sl = ring_slot(x, y, z);
        float v[NCH];
        bool nz = false;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            v[c] = lds_take(s + c * kB3 + sl);
            nz |= v[c] != 0.0f;
        }
        if (nz && x >= 0 && y >= 0 && z >= 0 && x < G.nx && y < G.ny && z < G.nz) out((z * G.ny + y) * G.nx + x, v);
    }
    template <class F>
    __device__ __forceinline__ void flush_all(const Geo& G, F& out) {
        auto fl = [&](int x, int y, int z) { flush_voxel(G, x, y, z, out); };
        win.each_voxel(fl);
    }
    template <class F>
    __device__ __forceinline__ void fit(const Geo& G, bool on, const int lo[3], const int hi[3], F& out) {
        auto fl = [&](int x, int y, int z) { flush_voxel(G, x, y, z, out); };
        win.fit(on, lo, hi, fl);
    }
};

__device__ __forceinline__ int __hip_atomic_compare_exchange_strong_ret(lds_int* p, int expected, int desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WAVEFRONT);
    return expected;  // the value found: equals the old expected value on success
}

// Per-wave LDS hash table for the environment texels a wave's rays hit (64 slots, linear
// probing; a texel that finds no slot goes straight to a global atomic).
template <int NCH>
struct TexTable {
    lds_int* keys;  // [64]
    lds_float* s;   // [NCH][64]
    __device__ __forceinline__ void init(int* kbase, float* sbase) {
        keys = (lds_int*)kbase;
        s = (lds_float*)sbase;
        keys[lane_id()] = -1;
#pragma unroll
        for (int c = 0; c < NCH; ++c) s[c * 64 + lane_id()] = 0.0f;
    }
    template <class F>
    __device__ __forceinline__ void insert(int t, const float v[NCH], F& out) {
        int sl = (int)(((unsigned)t * 2654435761u) >> 26);
#pragma unroll
        for (int probe = 0; probe < 4; ++probe) {
            const int prev = __hip_atomic_compare_exchange_strong_ret(keys + sl, -1, t);
            if (prev == -1 || prev == t) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) lds_add(s + c * 64 + sl, v[c]);
                return;
            }
            sl = (sl + 1) & 63;
        }
        out(t, v);
    }
    template <class F>
    __device__ __forceinline__ void flush(F& out) {
        const int l = lane_id();
        const int t = __hip_atomic_exchange(keys + l, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        float v[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) v[c] = lds_take(s + c * 64 + l);
        if (t >= 0) out(t, v);
    }
};

// Global sinks: add a unit's channels to HBM.
struct SinkY {  // y[4u + c], c < 4
    float* y;
    __device__ __forceinline__ void operator()(int u, const float* v) const {
        float* p = y + 4 * (size_t)u;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (v[c] != 0.0f) atomic_add(p + c, v[c]);
    }
    __device__ __forceinline__ void one(int u, int c, float v) const { atomic_add(y + 4 * (size_t)u + c, v); }
};
struct SinkGrad {  // grad[4u + c] (c < 4) and blocks[5u + c] (channels 4..8)
    float* grad;
    float* blocks;
    __device__ __forceinline__ void operator()(int u, const float* v) const {
        if (grad) {
            float* g = grad + 4 * (size_t)u;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (v[c] != 0.0f) atomic_add(g + c, v[c]);
        }
        if (blocks) {
            float* b = blocks + 5 * (size_t)u;
#pragma unroll
            for (int c = 0; c < 5; ++c)
                if (v[4 + c] != 0.0f) atomic_add(b + c, v[4 + c]);
        }
    }
};
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

// Byte offsets of the 8 trilinear corners from the lower corner (wave-uniform).
struct CornerOffs {
    int o[8];
};
template <int BYTES>
__device__ __forceinline__ CornerOffs corner_offs(int nx, int nxy) {
    CornerOffs k;
#pragma unroll
    for (int j = 0; j < 8; ++j) k.o[j] = corner_off(j, nx, nxy) * BYTES;
    return k;
}

// Gather the trilinear sample of a float4-per-unit vector at corners c.
template <class L>
__device__ __forceinline__ float4 gather4(const L& X, const Corners& c, const CornerOffs& k) {
    const int base = c.v * L::kBytes;
    float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float4 q = X.load(base, k.o[j]);
        s.x += c.w[j] * q.x;
        s.y += c.w[j] * q.y;
        s.z += c.w[j] * q.z;
        s.w += c.w[j] * q.w;
    }
    return s;
}

// Gather the trilinear sample of (c, sigma) at corners c.
template <int PD>
__device__ __forceinline__ void gather(XL<PD> X, const Corners& c, int nx, int nxy, float& sg, float& c0, float& c1,
                                       float& c2) {
    const float4 s = gather4(X, c, corner_offs<XL<PD>::kBytes>(nx, nxy));
    c0 = s.x;
    c1 = s.y;
    c2 = s.z;
    sg = s.w;
}

// The march of a wave is aligned in depth: lane i starts its first sample at wave step
// off_i = (t_n,i - min t_n) / (h step), so at every step the lanes sample their rays at
// about the same distance from the camera (the rays of an 8x8 tile are nearly parallel).
// Every lane still takes its own samples in its own order; only their timing changes.
template <int PD, bool TAN>
__device__ __forceinline__ void forward(const Geo& G, const Ray& r, bool live, XL<PD> X, VecF4 V,
                                        float H[3], float& Texit, float& Tdexit, float Hd[3], Depth& depth,
                                        float thresh = 0.0f) {
    float T = 1.0f, Td = 0.0f;
    depth.s = 0.0f;
    depth.c = 0.0f;
    H[0] = H[1] = H[2] = 0.0f;
    Hd[0] = Hd[1] = Hd[2] = 0.0f;
    const int nx = G.nx, nxy = G.nx * G.ny;
    const float unit = G.h * G.step;
    const float t_min = wave_min_f(r.K > 0 ? r.tn : INFINITY);
    const int off = r.K > 0 ? (int)((r.tn - t_min) / unit + 0.5f) : 0;
    const int J = wave_max_i(r.K > 0 ? off + r.K : 0);
    for (int j = 0; j < J; ++j) {
        const int k = j - off;
        if (k < 0 || k >= r.K) continue;
        float g[3];
        const float dk = sample_at(G, r, k, g);
        Corners c;
        corners(G, g, c);
        float sg, c0, c1, c2;
        gather<PD>(X, c, nx, nxy, sg, c0, c1, c2);
        float sgd = 0.0f, cd0 = 0.0f, cd1 = 0.0f, cd2 = 0.0f;
        if constexpr (TAN) {
            const float4 t = gather4(V, c, corner_offs<VecF4::kBytes>(nx, nxy));
            cd0 = t.x;
            cd1 = t.y;
            cd2 = t.z;
            sgd = t.w;
        }
        const float tau = sg * dk;
        depth.add(tau);
        const float e = exp_neg(tau);
        const float al = one_minus_exp_neg(tau, e);
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
    Tdexit = Td;
    if (thresh > 0.0f && 1.0f - T < thresh) {
        // rendering rule (Sec. IV): a volume this transparent counts as empty
        H[0] = H[1] = H[2] = 0.0f;
        T = 1.0f;
    }
    if (!live) return;
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
                const float4 t = V(tx.t[j]);
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

// ------------------------------------------------------------------ environment part of the adjoint
// T_l in front of every layer the ray hits (front to back from the grid exit), then the
// layers back to front with S, the radiance behind a layer (over-recurrence from the
// background).  emit(l, tx, c, alpha, T_l, S) hands each layer's data to the mode; returns
// S seen from the grid exit (unattenuated).
template <int PD, class Emit>
__device__ __forceinline__ void env_back(const Geo& G, const Ray& r, XL<PD> X, float Tx, float S[3], Emit& emit) {
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
    S[0] = G.bg[0];
    S[1] = G.bg[1];
    S[2] = G.bg[2];
#pragma unroll
    for (int l = kMaxLayers - 1; l >= 0; --l) {
        if (used & (1u << l)) {
            Tex tx;
            env_hit(G, r, l, tmin, tx);
            float al = 0.0f, c[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 q = X(tx.t[j]);
                c[0] += tx.w[j] * q.x;
                c[1] += tx.w[j] * q.y;
                c[2] += tx.w[j] * q.z;
                al += tx.w[j] * q.w;
            }
            emit(tx, c, al, Tl[l], S);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) S[ch] = al * c[ch] + (1.0f - al) * S[ch];
        }
    }
}

// ------------------------------------------------------------------ J^T u (and J^T J v) scatter
// Voxel samples from the last to the first, as in Alg. 1: G_k (colour composited behind
// sample k) is accumulated from the back starting at the environment seen from the exit,
// and T_k = exp(-V_k) with V_k the compensated optical depth stepped back.
template <int PD>
__device__ __forceinline__ void adjoint_scatter(const Geo& G, const Ray& r, bool live, XL<PD> X, const float u[3],
                                                float q4, Depth depth, Brick4& B, TexTable<4>& TT,
                                                float* __restrict__ y) {
    SinkY sink{y};
    const float Tx = exp_neg(depth.value());
    float uE = 0.0f;
    if (live) {
        float S[3];
        auto emit = [&](const Tex& tx, const float c[3], float al, float Tl, const float Sb[3]) {
            const float uc = u[0] * c[0] + u[1] * c[1] + u[2] * c[2];
            const float uS = u[0] * Sb[0] + u[1] * Sb[1] + u[2] * Sb[2];
            const float A = Tl * al;          // dH/dc_l
            const float dA = Tl * (uc - uS);  // u . dH/dalpha_l
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float wA = tx.w[j] * A;
                const float v[4] = {wA * u[0], wA * u[1], wA * u[2], tx.w[j] * dA};
                TT.insert(tx.t[j], v, sink);
            }
        };
        env_back<PD>(G, r, X, Tx, S, emit);
        uE = u[0] * S[0] + u[1] * S[1] + u[2] * S[2];
    }
    TT.flush(sink);
    B.clear_head(16);  // the table's keys (the table's sums are left at zero by the flush)
    float uG = Tx * uE;  // u . G_k
    float Tn = Tx;       // T_{k+1}
    const int nx = G.nx, nxy = G.nx * G.ny;
    const float unit = G.h * G.step;
    const float t_max = wave_max_f(r.K > 0 ? r.tf : -INFINITY);
    const int off = r.K > 0 ? (int)((t_max - r.tf) / unit + 0.5f) : 0;
    const int J = wave_max_i(r.K > 0 ? off + r.K : 0);
    // A lane whose next sample lies in the same cell hands this sample's value to the next
    // step, which scatters both together (one deferred sample at most): fewer updates enter
    // the elections.
    bool dpend = false;
    f4 dval = f4{0.0f, 0.0f, 0.0f, 0.0f};
    float df[3] = {0.0f, 0.0f, 0.0f};
    for (int j = 0; j < J; ++j) {
        const int m = j - off;
        const bool on = m >= 0 && m < r.K;
        const int k = r.K - 1 - m;
        Corners c{};
        float dk = 0.0f;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        if (on) {
            float g[3];
            dk = sample_at(G, r, k, g);
            corners(G, g, c);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = c.i[a];
                hi[a] = c.i[a] + 1;
            }
        }
        B.fit(G, on, lo, hi, sink);
        f4 val = {0.0f, 0.0f, 0.0f, 0.0f};
        if (on) {
            float sg, c0, c1, c2;
            gather<PD>(X, c, nx, nxy, sg, c0, c1, c2);
            const float tau = sg * dk;
            depth.add(-tau);
            const float T = (k == 0) ? 1.0f : exp_neg(depth.value());
            const float al = one_minus_exp_neg(tau, exp_neg(tau));
            const float A = T * al;
            const float uc = u[0] * c0 + u[1] * c1 + u[2] * c2;
            const float ds = dk * (Tn * uc - uG + q4);
            uG += A * uc;
            Tn = T;
            val = f4{A * u[0], A * u[1], A * u[2], ds};
        }
        bool defer = false;
        if (on && !dpend && k > 0) {
            float gn[3];
            (void)sample_at(G, r, k - 1, gn);
            defer = cell_key(G, gn) == c.v;
        }
        const bool two = on && dpend;
        B.scatter8(G, on && !defer, on && !defer && B.win.inside(lo, hi), c, val, two, dval, df, sink);
        if (defer) {
            dval = val;
            df[0] = c.f[0];
            df[1] = c.f[1];
            df[2] = c.f[2];
        }
        dpend = defer;
    }
    B.flush_all(G, sink);
}

// ------------------------------------------------------------------ gradient + exact blocks
// Per-ray window over the current 8 corners.  A voxel is a corner of a contiguous run of
// a ray's samples (its corner region is a box and the ray is a line), so a voxel that
// leaves the window never returns: flushing on leave aggregates the ray's partials per
// voxel exactly before they are squared into the block.  Register slot b holds the window
// voxel whose coordinate parities are the bits of b, so a voxel entering the window takes
// the slot of the one that left and nothing moves.  The flushed per-ray products
// (gradient and block entries, linear in the rays) are combined per wave in LDS.
struct GradWin {
    int i[3];                                 // low corner of the window
    float a[8], s0[8], s1[8], s2[8], s3[8];   // per slot: sum w A, sum w d_sigma (3 colours), sum w delta
};

// slots whose voxel leaves when the window's low corner moves from w to c (at most one cell
// per axis per sample; a larger jump empties the whole window)
__device__ __forceinline__ unsigned leaving_slots(const int w[3], const int c[3]) {
    constexpr unsigned kBit0[3] = {0x55u, 0x33u, 0x0Fu};  // slots with bit a = 0
    unsigned m = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int d = c[a] - w[a];
        if (d != 0) {
            const int gone = d > 0 ? w[a] : w[a] + 1;  // coordinate left behind
            m |= (d > 1 || d < -1) ? 0xFFu : ((gone & 1) ? (~kBit0[a] & 0xFFu) : kBit0[a]);
        }
    }
    return m;
}

template <int SLOT>
__device__ __forceinline__ void grad_flush_slot(const Geo& G, unsigned pend, const GradWin& w, const float rr[3],
                                                float r4, float g4, BrickAtomic<9>& B, const SinkGrad& sink) {
    const bool mine = (pend >> SLOT) & 1u;
    if (!wave_any(mine)) return;
    const int x = w.i[0] + (((SLOT >> 0) ^ w.i[0]) & 1);
    const int y = w.i[1] + (((SLOT >> 1) ^ w.i[1]) & 1);
    const int z = w.i[2] + (((SLOT >> 2) ^ w.i[2]) & 1);
    const float a = w.a[SLOT], s0 = w.s0[SLOT], s1 = w.s1[SLOT], s2 = w.s2[SLOT];
    const float q = g4 * w.s3[SLOT];  // the auxiliary residual's sigma partial (0 when off)
    float v[9] = {-a * rr[0], -a * rr[1], -a * rr[2], -(s0 * rr[0] + s1 * rr[1] + s2 * rr[2] + q * r4),
                  a * a,      a * s0,     a * s1,     a * s2,
                  s0 * s0 + s1 * s1 + s2 * s2 + q * q};
    // Neighbouring rays hand over the same voxel at the same step, and their LDS atomics on one
    // address serialise.  Fold the x neighbour's (lane ^ 1), the y neighbour's (lane ^ 8) and
    // then lane ^ 2's product into this lane when the voxel is the same; the donor drops out.
    // Straight-line code with every lane active (the swaps read the partner's registers).
    const int lane = lane_id();
    const int key = mine ? (z * G.ny + y) * G.nx + x : -1;
    bool keep = mine;
    auto fold = [&](auto swap, int bit) {
        const int kc = keep ? key : -1;
        const bool g = keep & (swap(kc) == kc);
        const bool give = g & ((lane & bit) != 0);
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] += __int_as_float(swap(__float_as_int(give ? v[c] : 0.0f)));
        keep = keep & !give;
    };
    fold([](int u) { return dpp_xor1(u); }, 1);
    fold([](int u) { return dpp_row_xor8(u); }, 8);
    fold([](int u) { return dpp_xor2(u); }, 2);
    if (!keep) return;
    const int lo[3] = {x, y, z};
    if (B.inside(lo, lo)) B.add(x, y, z, v);
    else sink((z * G.ny + y) * G.nx + x, v);
}

__device__ __forceinline__ void grad_flush(const Geo& G, unsigned pend, GradWin& w, const float rr[3], float r4,
                                           float g4, BrickAtomic<9>& B, const SinkGrad& sink) {
    grad_flush_slot<0>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<1>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<2>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<3>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<4>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<5>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<6>(G, pend, w, rr, r4, g4, B, sink);
    grad_flush_slot<7>(G, pend, w, rr, r4, g4, B, sink);
}

__device__ __forceinline__ unsigned nonzero_slots(const GradWin& w) {
    unsigned m = 0u;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if (w.a[b] != 0.0f || w.s0[b] != 0.0f || w.s1[b] != 0.0f || w.s2[b] != 0.0f || w.s3[b] != 0.0f) m |= 1u << b;
    return m;
}

__device__ __forceinline__ void clear_slots(GradWin& w, unsigned m) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (m & (1u << b)) {
            w.a[b] = 0.0f; w.s0[b] = 0.0f; w.s1[b] = 0.0f; w.s2[b] = 0.0f; w.s3[b] = 0.0f;
        }
    }
}

template <int PD>
__device__ __forceinline__ void grad_scatter(const Geo& G, const Ray& r, bool live, XL<PD> X, const float rr[3],
                                             float r4, float g4, Depth depth, BrickAtomic<9>& B, TexTable<9>& TT,
                                             float* __restrict__ grad,
                                             float* __restrict__ blocks) {
    SinkGrad sink{grad, blocks};
    const float Tx = exp_neg(depth.value());
    float S[3] = {0.0f, 0.0f, 0.0f};
    if (live) {
        // environment layers (the four texels of one lookup are distinct units)
        auto emit = [&](const Tex& tx, const float c[3], float al, float Tl, const float Sb[3]) {
            const float A = Tl * al;
            const float d0 = Tl * (c[0] - Sb[0]), d1 = Tl * (c[1] - Sb[1]), d2 = Tl * (c[2] - Sb[2]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float w = tx.w[j];
                const float a = w * A, s0 = w * d0, s1 = w * d1, s2 = w * d2;
                if (a == 0.0f && s0 == 0.0f && s1 == 0.0f && s2 == 0.0f) continue;
                const float v[9] = {-a * rr[0], -a * rr[1], -a * rr[2], -(s0 * rr[0] + s1 * rr[1] + s2 * rr[2]),
                                    a * a,      a * s0,     a * s1,     a * s2,
                                    s0 * s0 + s1 * s1 + s2 * s2};
                TT.insert(tx.t[j], v, sink);
            }
        };
        env_back<PD>(G, r, X, Tx, S, emit);
    }
    TT.flush(sink);
    B.clear_head(64);  // the table's keys (its sums are left at zero by the flush)
    GradWin w;
    w.i[0] = w.i[1] = w.i[2] = 0;
    clear_slots(w, 0xFFu);
    bool started = false;  // the window holds this ray's sums
    bool ended = false;    // the ray's last sample is in the window, to be flushed whole
    // G_k from the back, starting with the environment seen from the grid exit
    float G0 = Tx * S[0], G1 = Tx * S[1], G2 = Tx * S[2];
    float Tn = Tx;
    const int nx = G.nx, nxy = G.nx * G.ny;
    const float unit = G.h * G.step;
    const float t_max = wave_max_f(r.K > 0 ? r.tf : -INFINITY);
    const int off = r.K > 0 ? (int)((t_max - r.tf) / unit + 0.5f) : 0;
    const int J = wave_max_i(r.K > 0 ? off + r.K : 0);
    for (int j = 0; j < J; ++j) {
        const int m = j - off;
        const bool on = m >= 0 && m < r.K;
        const int k = r.K - 1 - m;
        Corners c;
        float dk = 0.0f;
        int lo[3] = {w.i[0], w.i[1], w.i[2]}, hi[3] = {w.i[0] + 1, w.i[1] + 1, w.i[2] + 1};
        if (on) {
            float g[3];
            dk = sample_at(G, r, k, g);
            corners(G, g, c);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // cover the voxels about to leave the lane's window as well as the new ones
                const int prev = started ? w.i[a] : c.i[a];
                lo[a] = min(prev, c.i[a]);
                hi[a] = max(prev, c.i[a]) + 1;
            }
        }
        B.fit(G, on || ended, lo, hi, sink);
        unsigned pend = 0u;
        if (ended) pend = 0xFFu;
        else if (on && started) pend = leaving_slots(w.i, c.i);
        if (pend) pend &= nonzero_slots(w);
        grad_flush(G, pend, w, rr, r4, g4, B, sink);
        if (ended) {
            clear_slots(w, 0xFFu);
            ended = false;
            started = false;
        }
        if (!on) continue;
        if (started) clear_slots(w, leaving_slots(w.i, c.i));
        w.i[0] = c.i[0]; w.i[1] = c.i[1]; w.i[2] = c.i[2];
        started = true;
        float sg, c0, c1, c2;
        gather<PD>(X, c, nx, nxy, sg, c0, c1, c2);
        const float tau = sg * dk;
        depth.add(-tau);
        const float T = (k == 0) ? 1.0f : exp_neg(depth.value());
        const float al = one_minus_exp_neg(tau, exp_neg(tau));
        const float A = T * al;
        const float ds0 = dk * (Tn * c0 - G0);
        const float ds1 = dk * (Tn * c1 - G1);
        const float ds2 = dk * (Tn * c2 - G2);
        G0 += A * c0;
        G1 += A * c1;
        G2 += A * c2;
        Tn = T;
        // slot b holds the corner whose offset along axis a is bit a of b xor the parity of
        // c.i[a]: its weight is the product of the per-axis weights
        float gw[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool odd = c.i[a] & 1;
            gw[a][0] = odd ? c.f[a] : 1.0f - c.f[a];
            gw[a][1] = odd ? 1.0f - c.f[a] : c.f[a];
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const float wb = gw[0][b & 1] * gw[1][(b >> 1) & 1] * gw[2][b >> 2];
            w.a[b] += wb * A;
            w.s0[b] += wb * ds0;
            w.s1[b] += wb * ds1;
            w.s2[b] += wb * ds2;
            w.s3[b] += wb * dk;
        }
        if (k == 0) ended = true;
    }
    // rays whose last sample came in the final step
    {
        const int lo[3] = {w.i[0], w.i[1], w.i[2]}, hi[3] = {w.i[0] + 1, w.i[1] + 1, w.i[2] + 1};
        B.fit(G, ended, lo, hi, sink);
        unsigned pend = ended ? nonzero_slots(w) : 0u;
        grad_flush(G, pend, w, rr, r4, g4, B, sink);
    }
    B.flush_all(G, sink);
}

// ------------------------------------------------------------------ workgroup FP64 sum
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void block_sum_store(double v, double* out) {
    __shared__ double red[kWaves];
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) s += red[i];
        *out = s;
    }
}

struct Pix {
    int cam, px, py;
    bool active;
    long long ray;
};

// Workgroup b covers a 16x8 pixel tile of camera b / n_tiles; wave w its 8x8 half w.
__device__ __forceinline__ Pix pixel_of(const Geo& G) {
    Pix p;
    const int b = blockIdx.x;
    p.cam = b / G.n_tiles;
    const int tile = b - p.cam * G.n_tiles;
    const int ty = tile / G.tiles_x, tx = tile - ty * G.tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    p.px = tx * kTileX + wave * 8 + (lane & 7);
    p.py = ty * kTileY + (lane >> 3);
    p.active = p.px < G.width && p.py < G.height;
    p.ray = ((long long)p.cam * G.height + p.py) * G.width + p.px;
    return p;
}

template <int MODE>
struct Lds {
    static constexpr int NCH = MODE == M_GRAD ? 9 : 4;
    static constexpr bool SCATTER = MODE == M_VJP || MODE == M_JTJ || MODE == M_GRAD;
};

template <int MODE, int PD>
__global__ __launch_bounds__(kBlock) void k_ray(Geo G, RayArgs A) {
    constexpr int NCH = Lds<MODE>::NCH;
    constexpr bool SCATTER = Lds<MODE>::SCATTER;
    constexpr bool JT = MODE == M_VJP || MODE == M_JTJ;
    __shared__ f4 s_brick[(SCATTER && !JT) ? kWaves * NCH * kB3 / 4 : 1];
    __shared__ f4 s_brick4[JT ? kWaves * kB3 : 1];
    __shared__ unsigned char s_tag[(SCATTER && MODE != M_GRAD) ? kWaves * kB3 : 1];
    if (A.done && *A.done) return;
    const Pix p = pixel_of(G);
    const int wave = threadIdx.x >> 6;
    const int units = G.nvox + G.n_layers * G.env_w * G.env_h;
    XL<PD> X;
    X.r = make_rsrc(A.x, (unsigned)units * XL<PD>::kBytes);
    Ray r;
    make_ray(G, A.cams[p.cam], p.px, p.py, p.ray, r);
    if (!p.active) {
        r.K = 0;
        r.hit = false;
    }
    float H[3], Hd[3], Texit, Tdexit;
    Depth depth;
    if constexpr (MODE == M_JVP || MODE == M_JTJ) {
        VecF4 V;
        V.r = make_rsrc(A.v, (unsigned)units * VecF4::kBytes);
        forward<PD, true>(G, r, p.active, X, V, H, Texit, Tdexit, Hd, depth);
    } else {
        forward<PD, false>(G, r, p.active, X, VecF4{}, H, Texit, Tdexit, Hd, depth,
                           MODE == M_RENDER ? A.thresh : 0.0f);
    }
    // auxiliary opacity residual (Sec. III-I, Eq. 10): r4 = lambda (1 - 4 (T - 1/2)^2) =
    // 4 lambda T (1 - T) with T the transmittance through the volume; dr4/dT = 4 lambda (1 - 2T)
    const bool aux = A.aux > 0.0f;
    const float r4 = aux ? 4.0f * A.aux * Texit * (1.0f - Texit) : 0.0f;
    const float dr4 = aux ? 4.0f * A.aux * (1.0f - 2.0f * Texit) : 0.0f;
    const int nres = A.nres;
    double rr_sum = 0.0;
    if constexpr (MODE == M_RENDER) {
        if (p.active) {
            if (A.targets) {
                float res[3];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    res[ch] = H[ch] - A.targets[3 * p.ray + ch];
                    rr_sum += (double)res[ch] * (double)res[ch];
                }
                rr_sum += (double)r4 * (double)r4;
                if (A.rout) {
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) A.rout[nres * p.ray + ch] = res[ch];
                    if (aux) A.rout[nres * p.ray + 3] = r4;
                }
            } else if (A.rout) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) A.rout[3 * p.ray + ch] = H[ch];
            }
        }
    } else if constexpr (MODE == M_JVP) {
        if (p.active) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) A.rout[nres * p.ray + ch] = Hd[ch];
            if (aux) A.rout[nres * p.ray + 3] = dr4 * Tdexit;  // d r4 = dr4/dT * dT
        }
    } else if constexpr (SCATTER) {
        // the texel hash table of each pass borrows the head of its window's storage until it
        // is flushed (keys: 64 ints, then NCH x 64 sums)
        TexTable<NCH> TT;
        if constexpr (JT) {
            Brick4 B;
            B.init(s_brick4 + wave * kB3, s_tag + wave * kB3);
            B.cmask = corner_mask(A.cams[p.cam]);
            TT.init((int*)(s_brick4 + wave * kB3), (float*)(s_brick4 + wave * kB3 + 16));
            float u[3] = {0.0f, 0.0f, 0.0f};
            float u4 = 0.0f;
            if (p.active) {
                if constexpr (MODE == M_VJP) {
                    u[0] = A.uin[nres * p.ray];
                    u[1] = A.uin[nres * p.ray + 1];
                    u[2] = A.uin[nres * p.ray + 2];
                    if (aux) u4 = A.uin[nres * p.ray + 3];
                } else {
                    u[0] = Hd[0];
                    u[1] = Hd[1];
                    u[2] = Hd[2];
                    u4 = dr4 * Tdexit;
                }
            }
            // u4 d r4 / d sigma_k = u4 dr4/dT (-T delta_k): a per-ray constant times delta_k,
            // added to the sigma partial of every sample
            const float q4 = -u4 * dr4 * Texit;
            adjoint_scatter<PD>(G, r, p.active, X, u, q4, depth, B, TT, A.y);
        } else {
            BrickAtomic<NCH> B;
            B.init((float*)(s_brick + wave * NCH * kB3 / 4));
            TT.init((int*)(s_brick + wave * NCH * kB3 / 4), (float*)(s_brick + wave * NCH * kB3 / 4) + 64);
            float res[3] = {0.0f, 0.0f, 0.0f};
            if (p.active && A.targets) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    res[ch] = H[ch] - A.targets[3 * p.ray + ch];
                    rr_sum += (double)res[ch] * (double)res[ch];
                }
                rr_sum += (double)r4 * (double)r4;
            }
            // the auxiliary residual's row: d r4 / d sigma_k = g4 delta_k
            const float g4 = -dr4 * Texit;
            grad_scatter<PD>(G, r, p.active, X, res, p.active ? r4 : 0.0f, g4, depth, B, TT, A.y, A.blocks);
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
        make_ray(G, cams[p.cam], p.px, p.py, p.ray, r);
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

}  // namespace perf
