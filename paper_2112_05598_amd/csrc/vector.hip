// Parameter-vector kernels of the PCG solve (Alg. 2), the preconditioner (Sec. III-G) and
// the line search (Alg. 3).  One thread handles one unit (float4 = the 4 parameters of a
// voxel or texel) in a grid-stride loop over a fixed grid of kVecGrid workgroups, so every
// dot product is reduced the same way on every call: FP64 per-thread sums, FP64 wave and
// workgroup reduction, one partial per workgroup, then a single workgroup adds the
// partials in index order.  All PCG scalars (alpha, beta, R, r^T z) stay on the device;
// the stop rules of Alg. 2 are evaluated there and raise a flag that every later kernel
// of the solve checks, so the host can enqueue a whole solve without reading anything back.
#include "perf_internal.h"

#include <math.h>

namespace perf {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup sum of two doubles; thread 0 stores them.
__device__ __forceinline__ void block_sum2(double a, double b, double* oa, double* ob) {
    __shared__ double red[2][kVecBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int i = 0; i < kVecBlock / 64; ++i) {
            sa += red[0][i];
            sb += red[1][i];
        }
        if (oa) *oa = sa;
        if (ob) *ob = sb;
    }
}

// Sum n partials in a fixed order with one workgroup (deterministic).
__device__ __forceinline__ double fixed_order_sum(const double* p, int64_t n) {
    __shared__ double red[kVecBlock / 64];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kVecBlock) s += p[i];
    s = wave_sum(s);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kVecBlock / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double dot4(float4 a, float4 b) {
    return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
}

// z = M^-1 r for one unit, from the preconditioner in scaled form.  Every stored value stays in
// FP32 range whatever the scale of the block (t = D^-1/2 is at most the inverse square root of
// the smallest subnormal), and the unscaled inverse is never formed.
//   Jacobi   t per parameter: z = t (t r).
//   Block    (t_d, t_f, e~, 1/s): D^-1/2 = diag(t_d, t_d, t_d, t_f), the normalised block
//            [[I, e~], [e~^T, 1]] and its Schur complement s = 1 - |e~|^2; with y = D^-1/2 r the
//            block is solved by elimination, z_sigma = (y_sigma - e~ . y_c) / s,
//            z_c = y_c - e~ z_sigma, then z = D^-1/2 z.  Elimination keeps the FP32 rounding
//            error along the block's own near-null direction; multiplying by the explicit
//            inverse, whose entries reach 1/s, would spread it over every direction.
//   Learned  (t_d, t_f, L row by row): z = D^-1/2 L (L^T (D^-1/2 r)); a unit on the exact-block
//            fallback holds the block form (-t_d, t_f, e~, 1/s) instead, told apart by t_d < 0.
template <int KIND>
__device__ __forceinline__ float4 precond_apply(const float* __restrict__ minv, int64_t u, float4 r) {
    if constexpr (KIND == PERF_PRECOND_NONE) {
        return r;
    } else if constexpr (KIND == PERF_PRECOND_JACOBI) {
        const float4 t = reinterpret_cast<const float4*>(minv)[u];
        return make_float4(t.x * (t.x * r.x), t.y * (t.y * r.y), t.z * (t.z * r.z), t.w * (t.w * r.w));
    } else if constexpr (KIND == PERF_PRECOND_BLOCK4) {
        const float4* q = reinterpret_cast<const float4*>(minv) + 2 * u;
        const float4 q0 = q[0], q1 = q[1];
        const float td = q0.x, tf = q0.y, e0 = q0.z, e1 = q0.w, e2 = q1.x, is = q1.y;
        const float y0 = td * r.x, y1 = td * r.y, y2 = td * r.z, y3 = tf * r.w;
        const float zs = (y3 - (e0 * y0 + e1 * y1 + e2 * y2)) * is;
        return make_float4(td * (y0 - e0 * zs), td * (y1 - e1 * zs), td * (y2 - e2 * zs), tf * zs);
    } else {
        const float4* q = reinterpret_cast<const float4*>(minv) + 3 * u;
        const float4 q0 = q[0], q1 = q[1];
        if (q0.x < 0.0f) {
            // a unit on the exact-block fallback: the block form, with t_d stored negated
            const float td = -q0.x, tf = q0.y, e0 = q0.z, e1 = q0.w, e2 = q1.x, is = q1.y;
            const float y0 = td * r.x, y1 = td * r.y, y2 = td * r.z, y3 = tf * r.w;
            const float zs = (y3 - (e0 * y0 + e1 * y1 + e2 * y2)) * is;
            return make_float4(td * (y0 - e0 * zs), td * (y1 - e1 * zs), td * (y2 - e2 * zs), tf * zs);
        }
        const float4 q2 = q[2];
        const float td = q0.x, tf = q0.y;
        const float l00 = q0.z, l10 = q0.w, l11 = q1.x, l20 = q1.y, l21 = q1.z, l22 = q1.w, l30 = q2.x, l31 = q2.y,
                    l32 = q2.z, l33 = q2.w;
        const float y0 = td * r.x, y1 = td * r.y, y2 = td * r.z, y3 = tf * r.w;
        // w = L^T y, then v = L w
        const float w0 = l00 * y0 + l10 * y1 + l20 * y2 + l30 * y3;
        const float w1 = l11 * y1 + l21 * y2 + l31 * y3;
        const float w2 = l22 * y2 + l32 * y3;
        const float w3 = l33 * y3;
        return make_float4(td * (l00 * w0), td * (l10 * w0 + l11 * w1), td * (l20 * w0 + l21 * w1 + l22 * w2),
                           tf * (l30 * w0 + l31 * w1 + l32 * w2 + l33 * w3));
    }
}

__global__ void k_zero(float* __restrict__ p, int64_t n, const int* done) {
    if (done && *done) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_sum_partials(const double* p, int64_t n, double scale, double* out) {
    const double s = fixed_order_sum(p, n);
    if (threadIdx.x == 0) *out = scale * s;
}

// Scaled form of the preconditioner (Sec. III-G) from the blocks [[d I, e], [e^T, f]], FP64 inside.
// Jacobi: (t_d, t_d, t_d, t_f) with t = 1/sqrt(diagonal), 0 for a zero diagonal, so that
// M^-1 = t^2 = 1/diag(J^T J).  Block: after a ridge rho = 1e-6 max(d, f), t_d = (d + rho)^-1/2,
// t_f = (f + rho)^-1/2, the normalised coupling e~ = t_d t_f e and 1/s with s = 1 - |e~|^2, the
// Schur complement of the normalised block [[I, e~], [e~^T, 1]]: (t_d, t_f, e~, 1/s, 0, 0).
__global__ void k_invert(int kind, const float* __restrict__ blocks, int64_t units, float* __restrict__ out) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const float* b = blocks + 5 * u;
        const double d = b[0], e0 = b[1], e1 = b[2], e2 = b[3], f = b[4];
        if (kind == PERF_PRECOND_JACOBI) {
            const float td = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.0f;
            const float tf = f > 0.0 ? (float)(1.0 / sqrt(f)) : 0.0f;
            reinterpret_cast<float4*>(out)[u] = make_float4(td, td, td, tf);
        } else {
            float4* o = reinterpret_cast<float4*>(out) + 2 * u;
            const double m = fmax(d, f);
            if (!(m > 0.0) || !isfinite(d + e0 + e1 + e2 + f)) {  // no ray, or a non-finite block
                o[0] = o[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                continue;
            }
            const double rho = 1e-6 * m;
            const double td = 1.0 / sqrt(d + rho), tf = 1.0 / sqrt(f + rho);
            const double a0 = e0 * td * tf, a1 = e1 * td * tf, a2 = e2 * td * tf;
            const double is = 1.0 / (1.0 - (a0 * a0 + a1 * a1 + a2 * a2));
            o[0] = make_float4((float)td, (float)tf, (float)a0, (float)a1);
            o[1] = make_float4((float)a2, (float)is, 0.0f, 0.0f);
        }
    }
}

// r = b, z = M^-1 r, p = z, delta = 0; partials of r.r and r.z
template <int KIND>
__global__ void k_pcg_init(const float4* __restrict__ b, const float* __restrict__ minv, float4* __restrict__ r,
                           float4* __restrict__ z, float4* __restrict__ p, float4* __restrict__ delta, int64_t units,
                           double* partials) {
    double rr = 0.0, rz = 0.0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const float4 ru = b[u];
        const float4 zu = precond_apply<KIND>(minv, u, ru);
        r[u] = ru;
        z[u] = zu;
        p[u] = zu;
        delta[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        rr += dot4(ru, ru);
        rz += dot4(ru, zu);
    }
    block_sum2(rr, rz, partials + blockIdx.x, partials + gridDim.x + blockIdx.x);
}

__global__ void k_pcg_init_fin(const double* partials, int64_t nb, double* sc, int* fl) {
    const double rr = fixed_order_sum(partials, nb);
    const double rz = fixed_order_sum(partials + nb, nb);
    if (threadIdx.x == 0) {
        sc[S_R0] = rr;
        sc[S_RPREV] = rr;
        sc[S_R] = rr;
        sc[S_RZ] = rz;
        fl[I_ITERS] = 0;
        fl[I_FLAGS] = 0;
        const int max_iters = (int)sc[S_MAXITERS];
        if (rr == 0.0 || max_iters <= 0) {
            fl[I_DONE] = 1;
            if (rr == 0.0) fl[I_FLAGS] |= PERF_FLAG_CONVERGED;
        } else {
            fl[I_DONE] = 0;
        }
    }
}

__global__ void k_dot(const float4* __restrict__ a, const float4* __restrict__ b, int64_t units, double* partials,
                      const int* done) {
    if (*done) return;
    double s = 0.0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x)
        s += dot4(a[u], b[u]);
    block_sum2(s, 0.0, partials + blockIdx.x, nullptr);
}

__global__ void k_pcg_alpha_fin(const double* partials, int64_t nb, double* sc, double* hist, int* fl) {
    if (fl[I_DONE]) return;
    const double pAp = fixed_order_sum(partials, nb);
    if (threadIdx.x == 0) {
        const int it = fl[I_ITERS];
        sc[S_PAP] = pAp;
        hist[4 * it + 3] = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            fl[I_DONE] = 1;
            fl[I_FLAGS] |= PERF_FLAG_BREAKDOWN;
            sc[S_ALPHA] = 0.0;
        } else {
            const double a = sc[S_RZ] / pAp;
            sc[S_ALPHA] = a;
            hist[4 * it + 0] = a;
        }
    }
}

// delta += alpha p; r -= alpha Ap; z = M^-1 r; partials of r.r and r.z
template <int KIND>
__global__ void k_pcg_update(const float* __restrict__ minv, float4* __restrict__ delta, float4* __restrict__ r,
                             float4* __restrict__ z, const float4* __restrict__ p, const float4* __restrict__ Ap,
                             int64_t units, double* partials, const double* sc, const int* fl) {
    if (fl[I_DONE]) return;
    const float a = (float)sc[S_ALPHA];
    double rr = 0.0, rz = 0.0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const float4 pu = p[u], Apu = Ap[u];
        float4 d = delta[u], ru = r[u];
        d.x += a * pu.x; d.y += a * pu.y; d.z += a * pu.z; d.w += a * pu.w;
        ru.x -= a * Apu.x; ru.y -= a * Apu.y; ru.z -= a * Apu.z; ru.w -= a * Apu.w;
        const float4 zu = precond_apply<KIND>(minv, u, ru);
        delta[u] = d;
        r[u] = ru;
        z[u] = zu;
        rr += dot4(ru, ru);
        rz += dot4(ru, zu);
    }
    block_sum2(rr, rz, partials + blockIdx.x, partials + gridDim.x + blockIdx.x);
}

__global__ void k_pcg_update_fin(const double* partials, int64_t nb, double* sc, double* hist, int* fl) {
    if (fl[I_DONE]) return;
    const double R = fixed_order_sum(partials, nb);
    const double rz_new = fixed_order_sum(partials + nb, nb);
    if (threadIdx.x == 0) {
        const int it = fl[I_ITERS];
        hist[4 * it + 2] = R;
        sc[S_R] = R;
        const int k = it + 1;
        fl[I_ITERS] = k;
        int stop = 0;
        if (sc[S_ABSEPS] > 0.0 && R < sc[S_ABSEPS]) {
            stop = 1;
            fl[I_FLAGS] |= PERF_FLAG_CONVERGED;
        } else if (sc[S_RELTOL] > 0.0 && sqrt(R / sc[S_R0]) <= sc[S_RELTOL]) {
            stop = 1;
            fl[I_FLAGS] |= PERF_FLAG_CONVERGED;
        } else if (sc[S_STALL] > 0.0 && R / sc[S_RPREV] > sc[S_STALL]) {
            stop = 1;
            fl[I_FLAGS] |= PERF_FLAG_STALL;
        } else if (k >= (int)sc[S_MAXITERS]) {
            stop = 1;
        }
        if (stop) {
            fl[I_DONE] = 1;
        } else {
            sc[S_RPREV] = R;
            const double beta = rz_new / sc[S_RZ];
            sc[S_BETA] = beta;
            sc[S_RZ] = rz_new;
            hist[4 * it + 1] = beta;
        }
    }
}

__global__ void k_pcg_direction(const float4* __restrict__ z, float4* __restrict__ p, int64_t units, const double* sc,
                                const int* fl) {
    if (fl[I_DONE]) return;
    const float beta = (float)sc[S_BETA];
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const float4 zu = z[u];
        float4 pu = p[u];
        pu.x = zu.x + beta * pu.x;
        pu.y = zu.y + beta * pu.y;
        pu.z = zu.z + beta * pu.z;
        pu.w = zu.w + beta * pu.w;
        p[u] = pu;
    }
}

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
    const unsigned r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}

// xt = proj(x + gamma delta): sigma >= 0 on voxels, alpha in [0,1] on texels
__global__ void k_trial(const float4* __restrict__ x, const float4* __restrict__ delta, float gamma, int64_t units,
                        int nvox, float4* __restrict__ xt, ushort4* __restrict__ xb) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        float4 v = x[u];
        if (delta) {
            const float4 d = delta[u];
            v.x += gamma * d.x;
            v.y += gamma * d.y;
            v.z += gamma * d.z;
            v.w += gamma * d.w;
            v.w = (u < nvox) ? fmaxf(v.w, 0.0f) : fminf(fmaxf(v.w, 0.0f), 1.0f);
        }
        if (xt) xt[u] = v;
        if (xb) {
            ushort4 q;
            q.x = f32_to_bf16_rne(v.x);
            q.y = f32_to_bf16_rne(v.y);
            q.z = f32_to_bf16_rne(v.z);
            q.w = f32_to_bf16_rne(v.w);
            xb[u] = q;
        }
    }
}

__global__ void k_pack_bf16(const float* __restrict__ in, unsigned short* __restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f32_to_bf16_rne(in[i]);
}

__global__ void k_check_finite(const float* __restrict__ p, int64_t n, int* flag) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) atomicOr(flag, 1);
}

// features [units][PERF_MLP_NFEAT] from the parameters and the blocks of the gradient pass:
// sigma/alpha, colour (3), log d, log f
__device__ __forceinline__ float bf16f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

__global__ void k_features(const void* __restrict__ xp, int x_bf16, const float* __restrict__ blocks, int64_t units,
                           float* __restrict__ feat) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        float4 xv;
        if (x_bf16) {
            const ushort4 q = reinterpret_cast<const ushort4*>(xp)[u];
            xv = make_float4(bf16f(q.x), bf16f(q.y), bf16f(q.z), bf16f(q.w));
        } else {
            xv = reinterpret_cast<const float4*>(xp)[u];
        }
        const float* b = blocks + 5 * u;
        float* f = feat + PERF_MLP_NFEAT * u;
        f[0] = xv.w;
        f[1] = xv.x;
        f[2] = xv.y;
        f[3] = xv.z;
        f[4] = logf(fmaxf(b[0], 0.0f) + 1e-12f);
        f[5] = logf(fmaxf(b[4], 0.0f) + 1e-12f);
    }
}

// Training rows of the learned preconditioner: every unit some ray touches (max(d, f) > 0) is
// kept with probability keep, decided by a counter-based hash of (seed, unit), and the kept
// rows are packed in unit order.  Workgroup g of a fixed grid owns one contiguous chunk of
// units: it counts its kept rows, one workgroup turns the counts into offsets, and each
// workgroup then writes its rows at its offset in order (deterministic output).
__device__ __forceinline__ unsigned mix32(unsigned h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
// A row is eligible when some ray touches the unit and its block and features are finite (a unit
// whose parameters ran off during a poorly conditioned step can carry infinite sums).
__device__ __forceinline__ bool keep_row(const float* __restrict__ feat, const float* __restrict__ blocks, int64_t u,
                                         unsigned seed, unsigned thresh) {
    const float* b = blocks + 5 * u;
    bool ok = fmaxf(b[0], b[4]) > 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) ok &= isfinite(b[i]);
#pragma unroll
    for (int i = 0; i < PERF_MLP_NFEAT; ++i) ok &= isfinite(feat[PERF_MLP_NFEAT * u + i]);
    return ok && mix32(seed ^ mix32((unsigned)u ^ (unsigned)(u >> 32) * 0x9e3779b9u)) < thresh;
}

// kept rows of the workgroup's chunk before each thread's unit in this pass of the chunk
__device__ __forceinline__ int block_exclusive_count(bool flag, int* total) {
    __shared__ int wsum[kVecBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(flag);
    const int before_in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int before = before_in_wave, all = 0;
#pragma unroll
    for (int i = 0; i < kVecBlock / 64; ++i) {
        before += (i < wave) ? wsum[i] : 0;
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before;
}

__global__ __launch_bounds__(kVecBlock) void k_rows_count(const float* __restrict__ feat,
                                                          const float* __restrict__ blocks, int64_t units,
                                                          int64_t chunk, unsigned seed, unsigned thresh,
                                                          long long* counts) {
    const int64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, units);
    long long c = 0;
    for (int64_t base = lo; base < hi; base += kVecBlock) {
        const int64_t u = base + threadIdx.x;
        int total;
        (void)block_exclusive_count(u < hi && keep_row(feat, blocks, u, seed, thresh), &total);
        c += total;
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void k_rows_offsets(long long* counts, int nb) {
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int i = 0; i < nb; ++i) {
            const long long c = counts[i];
            counts[i] = run;
            run += c;
        }
        counts[nb] = run;
    }
}

__global__ __launch_bounds__(kVecBlock) void k_rows_write(const float* __restrict__ feat, const float* __restrict__ blocks,
                                                          int64_t units, int64_t chunk, unsigned seed, unsigned thresh,
                                                          const long long* offsets, int64_t cap,
                                                          float* __restrict__ feat_out, float* __restrict__ blocks_out) {
    const int64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, units);
    long long at = offsets[blockIdx.x];
    for (int64_t base = lo; base < hi; base += kVecBlock) {
        const int64_t u = base + threadIdx.x;
        const bool k = u < hi && keep_row(feat, blocks, u, seed, thresh);
        int total;
        const int before = block_exclusive_count(k, &total);
        const long long dst = at + before;
        if (k && dst < cap) {
#pragma unroll
            for (int i = 0; i < PERF_MLP_NFEAT; ++i) feat_out[PERF_MLP_NFEAT * dst + i] = feat[PERF_MLP_NFEAT * u + i];
#pragma unroll
            for (int i = 0; i < 5; ++i) blocks_out[5 * dst + i] = blocks[5 * u + i];
        }
        at += total;
    }
}

unsigned grid_for(int64_t n) {
    int64_t g = (n + kVecBlock - 1) / kVecBlock;
    if (g > kVecGrid) g = kVecGrid;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_zero(float* p, int64_t n, hipStream_t st, const int* done) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kVecBlock), 0, st, p, n, done);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n)), dim3(kVecBlock), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int64_t n, double scale, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kVecBlock), 0, st, partials, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_precond_invert(int kind, const float* blocks, int64_t units, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_invert, dim3(grid_for(units)), dim3(kVecBlock), 0, st, kind, blocks, units, out);
    return hipGetLastError();
}

hipError_t launch_pcg_init(int kind, const float* b, const float* minv, float* r, float* z, float* p, float* delta,
                           int64_t units, double* partials, double* scalars, int* iflags, hipStream_t st) {
    const unsigned g = grid_for(units);
    auto B = reinterpret_cast<const float4*>(b);
    auto R = reinterpret_cast<float4*>(r);
    auto Z = reinterpret_cast<float4*>(z);
    auto Pp = reinterpret_cast<float4*>(p);
    auto D = reinterpret_cast<float4*>(delta);
    switch (kind) {
        case PERF_PRECOND_NONE:
            hipLaunchKernelGGL(k_pcg_init<PERF_PRECOND_NONE>, dim3(g), dim3(kVecBlock), 0, st, B, minv, R, Z, Pp, D,
                               units, partials);
            break;
        case PERF_PRECOND_JACOBI:
            hipLaunchKernelGGL(k_pcg_init<PERF_PRECOND_JACOBI>, dim3(g), dim3(kVecBlock), 0, st, B, minv, R, Z, Pp, D,
                               units, partials);
            break;
        case PERF_PRECOND_BLOCK4:
            hipLaunchKernelGGL(k_pcg_init<PERF_PRECOND_BLOCK4>, dim3(g), dim3(kVecBlock), 0, st, B, minv, R, Z, Pp, D,
                               units, partials);
            break;
        default:
            hipLaunchKernelGGL(k_pcg_init<PERF_PRECOND_LEARNED>, dim3(g), dim3(kVecBlock), 0, st, B, minv, R, Z, Pp,
                               D, units, partials);
            break;
    }
    hipLaunchKernelGGL(k_pcg_init_fin, dim3(1), dim3(kVecBlock), 0, st, partials, (int64_t)g, scalars, iflags);
    return hipGetLastError();
}

hipError_t launch_pcg_alpha(const float* p, const float* Ap, int64_t units, double* partials, double* scalars,
                            double* hist, int* iflags, hipStream_t st) {
    const unsigned g = grid_for(units);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kVecBlock), 0, st, reinterpret_cast<const float4*>(p),
                       reinterpret_cast<const float4*>(Ap), units, partials, iflags + I_DONE);
    hipLaunchKernelGGL(k_pcg_alpha_fin, dim3(1), dim3(kVecBlock), 0, st, partials, (int64_t)g, scalars, hist, iflags);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int kind, const float* minv, float* delta, float* r, float* z, const float* p,
                             const float* Ap, int64_t units, double* partials, double* scalars, double* hist,
                             int* iflags, hipStream_t st) {
    const unsigned g = grid_for(units);
    auto D = reinterpret_cast<float4*>(delta);
    auto R = reinterpret_cast<float4*>(r);
    auto Z = reinterpret_cast<float4*>(z);
    auto Pp = reinterpret_cast<const float4*>(p);
    auto A = reinterpret_cast<const float4*>(Ap);
    switch (kind) {
        case PERF_PRECOND_NONE:
            hipLaunchKernelGGL(k_pcg_update<PERF_PRECOND_NONE>, dim3(g), dim3(kVecBlock), 0, st, minv, D, R, Z, Pp, A,
                               units, partials, scalars, iflags);
            break;
        case PERF_PRECOND_JACOBI:
            hipLaunchKernelGGL(k_pcg_update<PERF_PRECOND_JACOBI>, dim3(g), dim3(kVecBlock), 0, st, minv, D, R, Z, Pp,
                               A, units, partials, scalars, iflags);
            break;
        case PERF_PRECOND_BLOCK4:
            hipLaunchKernelGGL(k_pcg_update<PERF_PRECOND_BLOCK4>, dim3(g), dim3(kVecBlock), 0, st, minv, D, R, Z, Pp,
                               A, units, partials, scalars, iflags);
            break;
        default:
            hipLaunchKernelGGL(k_pcg_update<PERF_PRECOND_LEARNED>, dim3(g), dim3(kVecBlock), 0, st, minv, D, R, Z, Pp,
                               A, units, partials, scalars, iflags);
            break;
    }
    hipLaunchKernelGGL(k_pcg_update_fin, dim3(1), dim3(kVecBlock), 0, st, partials, (int64_t)g, scalars, hist, iflags);
    return hipGetLastError();
}

hipError_t launch_pcg_direction(const float* z, float* p, int64_t units, const double* scalars, const int* iflags,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_direction, dim3(grid_for(units)), dim3(kVecBlock), 0, st,
                       reinterpret_cast<const float4*>(z), reinterpret_cast<float4*>(p), units, scalars, iflags);
    return hipGetLastError();
}

hipError_t launch_trial(const float* x, const float* delta, float gamma, int64_t units, int nvox, float* xt,
                        uint16_t* xb16, hipStream_t st) {
    hipLaunchKernelGGL(k_trial, dim3(grid_for(units)), dim3(kVecBlock), 0, st, reinterpret_cast<const float4*>(x),
                       reinterpret_cast<const float4*>(delta), gamma, units, nvox, reinterpret_cast<float4*>(xt),
                       reinterpret_cast<ushort4*>(xb16));
    return hipGetLastError();
}

hipError_t launch_pack_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_bf16, dim3(grid_for(n)), dim3(kVecBlock), 0, st, in, out, n);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n)), dim3(kVecBlock), 0, st, p, n, flag);
    return hipGetLastError();
}

hipError_t launch_training_rows(const float* feat, const float* blocks, int64_t units, unsigned seed, float keep,
                                float* feat_out, float* blocks_out, int64_t cap, long long* counts, hipStream_t st) {
    const int nb = kVecGrid;
    const int64_t chunk = (units + nb - 1) / nb;
    const double t = fmin(fmax((double)keep, 0.0), 1.0) * 4294967296.0;
    const unsigned thresh = t >= 4294967295.0 ? 0xffffffffu : (unsigned)t;
    hipLaunchKernelGGL(k_rows_count, dim3(nb), dim3(kVecBlock), 0, st, feat, blocks, units, chunk, seed, thresh,
                       counts);
    hipLaunchKernelGGL(k_rows_offsets, dim3(1), dim3(64), 0, st, counts, nb);
    hipLaunchKernelGGL(k_rows_write, dim3(nb), dim3(kVecBlock), 0, st, feat, blocks, units, chunk, seed, thresh, counts,
                       cap, feat_out, blocks_out);
    return hipGetLastError();
}

hipError_t launch_unit_features(const void* x, int x_dtype, const float* blocks, int64_t units, float* feat,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3(grid_for(units)), dim3(kVecBlock), 0, st, x, x_dtype == PERF_BF16 ? 1 : 0,
                       blocks, units, feat);
    return hipGetLastError();
}

}  // namespace perf
