// Learned block preconditioner on gfx950: per-unit MLP 10 -> 64 -> 64 -> 10 with bfloat16
// operands on the matrix cores (v_mfma_f32_32x32x8_bf16) and FP32 accumulation.
//
// Not part of the paper: Sec. III-G preconditions PCG with the diagonal of J^T J; here the
// exact 4x4 block of each unit (three colours and the opacity) is the training target and
// the network predicts its inverse from cheap per-unit features (the unit's parameters and the
// diagonals of its block).  The output is a lower
// triangular factor L (softplus on the diagonal), so M^-1 = D^-1/2 L L^T D^-1/2 is symmetric
// positive definite by construction; D = diag(d, d, d, f) + ridge.
//
// The network's input is the standardised feature vector clamp((f - mu) s, -8, 8), with mu and
// s = 1 / max(std, 1e-3) taken from the training set (norm [32] = mu[16], s[16]), followed by
// the normalised colour-density coupling e~ of the unit's block (three values in (-1, 1)) and the
// log of 1 / sqrt of its Schur complement.  At inference
// a unit whose prediction misses its own normalised block by q = ||L L^T B~ - I||_F^2 above a
// threshold takes the exact block inverse instead (plain block-Jacobi as the fallback).
//
// Every product is C[M x N] = A[M x K] * Bt[N x K]^T with both operands bfloat16 in LDS,
// K contiguous, rows padded to avoid bank conflicts.  One wave owns a tile of 64 units.
// MFMA operand layout (checked on the device): lane l holds A[l%32][4(l/32)+j] and
// B[4(l/32)+j][l%32], j < 4; result register v of lane l is C[8(v/4)+4(l/32)+v%4][l%32].
#include "perf_internal.h"

#include <math.h>

#include <mutex>

namespace perf {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
#define LDS __attribute__((address_space(3)))
typedef LDS unsigned short lds_bf;

constexpr int NIN = PERF_MLP_NFEAT, NIP = 16, NH = 64, NO = 10, NOP = 16;
constexpr int NNET = NIN + 4;  // network inputs: the stored features, the block's coupling and its Schur log
constexpr float kSchurCap = 8.0f;  // cap on the Schur log input
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIP, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOP * NH, NW = OFF_B3 + NOP;
static_assert(NW == PERF_MLP_NW, "packed weight layout");
constexpr int TU = 64;   // units per wave tile
constexpr int LD16 = 20, LD32 = 36, LD64 = 68;  // padded row strides (elements)
constexpr float kRidge = 1e-6f;
constexpr float kKappa = 4.0f;  // per-unit loss is quadratic up to ||E||^2 = kKappa, linear in ||E|| above
constexpr float kClamp = 8.0f;  // standardised inputs are clamped to [-kClamp, kClamp]

__device__ __forceinline__ unsigned short f2bf(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }
__device__ __forceinline__ int lane() { return threadIdx.x & 63; }

// acc[mb][nb] += A[(mb*32+..) x K] * Bt[(nb*32+..) x K]^T
template <int MB, int NB, int KS>
__device__ __forceinline__ void wgemm(const lds_bf* A, int lda, const lds_bf* Bt, int ldb, f16v (&acc)[MB][NB]) {
    const int r = lane() & 31, h = lane() >> 5;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        s4 a[MB], b[NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb] = *(const LDS s4*)(A + (mb * 32 + r) * lda + ks * 8 + 4 * h);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb] = *(const LDS s4*)(Bt + (nb * 32 + r) * ldb + ks * 8 + 4 * h);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
}

template <int MB, int NB>
__device__ __forceinline__ void zero(f16v (&acc)[MB][NB]) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;
}

// row / column of result register v of this lane in block (mb, nb)
__device__ __forceinline__ int crow(int mb, int v) { return mb * 32 + 8 * (v >> 2) + 4 * (lane() >> 5) + (v & 3); }
__device__ __forceinline__ int ccol(int nb) { return nb * 32 + (lane() & 31); }

struct Weights {  // bfloat16 weights in LDS, rows K-contiguous
    lds_bf* W1;   // [64][LD16]  (h, i)
    lds_bf* W2;   // [64][LD64]  (h_out, h_in)
    lds_bf* W3;   // [32][LD64]  (o, h), rows >= 16 zero
    float* b1;
    float* b2;
    float* b3;
};

// Cooperative load of the packed bf16 weights (whole workgroup, then a barrier).
__device__ void load_weights(const unsigned short* __restrict__ w, Weights W, lds_bf* W2t, lds_bf* W3t) {
    for (int i = threadIdx.x; i < NH * NIP; i += blockDim.x) W.W1[(i / NIP) * LD16 + i % NIP] = w[OFF_W1 + i];
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {
        const int ho = i / NH, hi = i % NH;
        W.W2[ho * LD64 + hi] = w[OFF_W2 + i];
        if (W2t) W2t[hi * LD64 + ho] = w[OFF_W2 + i];
    }
    for (int i = threadIdx.x; i < 32 * NH; i += blockDim.x) {
        const int o = i / NH, hh = i % NH;
        const unsigned short v = o < NOP ? w[OFF_W3 + i] : (unsigned short)0;
        W.W3[o * LD64 + hh] = v;
        if (W3t) W3t[hh * LD32 + o] = v;
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        W.b1[i] = bf2f(w[OFF_B1 + i]);
        W.b2[i] = bf2f(w[OFF_B2 + i]);
    }
    for (int i = threadIdx.x; i < NOP; i += blockDim.x) W.b3[i] = bf2f(w[OFF_B3 + i]);
    __syncthreads();
}

// Forward pass of one tile: X (bf16 [TU][LD16]) -> H1, H2 (bf16 [TU][LD64]) -> O (fp32 [TU][17]).
// With Xt/H1t/H2t non-null the transposed activations ([feature][unit]) are written too.
__device__ void forward_tile(const Weights& W, const lds_bf* Xs, lds_bf* H1s, lds_bf* H2s, float* Os, lds_bf* H1t,
                             lds_bf* H2t) {
    {
        f16v acc[2][2];
        zero(acc);
        wgemm<2, 2, NIP / 8>(Xs, LD16, W.W1, LD16, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int u = crow(mb, v), hh = ccol(nb);
                    const unsigned short q = f2bf(fmaxf(acc[mb][nb][v] + W.b1[hh], 0.0f));
                    H1s[u * LD64 + hh] = q;
                    if (H1t) H1t[hh * LD64 + u] = q;
                }
    }
    {
        f16v acc[2][2];
        zero(acc);
        wgemm<2, 2, NH / 8>(H1s, LD64, W.W2, LD64, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int u = crow(mb, v), hh = ccol(nb);
                    const unsigned short q = f2bf(fmaxf(acc[mb][nb][v] + W.b2[hh], 0.0f));
                    H2s[u * LD64 + hh] = q;
                    if (H2t) H2t[hh * LD64 + u] = q;
                }
    }
    {
        f16v acc[2][1];
        zero(acc);
        wgemm<2, 1, NH / 8>(H2s, LD64, W.W3, LD64, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int u = crow(mb, v), o = ccol(0);
                if (o < NOP) Os[u * 17 + o] = acc[mb][0][v] + W.b3[o];
            }
    }
}

__device__ __forceinline__ float softplus(float x) { return x > 20.0f ? x : log1pf(expf(x)); }
__device__ __forceinline__ float sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }

// lower-triangular L from the 10 raw outputs, rows (0,0),(1,0),(1,1),(2,0),...,(3,3)
__device__ __forceinline__ void make_L(const float raw[NO], float L[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) L[i][j] = 0.0f;
    int k = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j, ++k) L[i][j] = (i == j) ? softplus(raw[k]) : raw[k];
}

// standardised features of one unit into the X tile row (bf16, zero padded): clamp((f - mu) s)
// The block inputs of a unit's block [d, e (3), f]: the normalised colour-density coupling
// e~ = e / sqrt((d + rho)(f + rho)) (|e~| < 1 for a positive semi-definite block), then
// -1/2 log(1 - |e~|^2), the log of 1 / sqrt of the Schur complement of the normalised block (the
// inverse's entries grow as its inverse), 8 where the complement is at most exp(-16).  All zero
// for a unit no ray touches or a non-finite block.  In double: d may be subnormal, and
// 1 - |e~|^2 cancels.
__device__ __forceinline__ void block_inputs(const float* __restrict__ b, float e[4]) {
    const float d = b[0], f = b[4];
    const float m = fmaxf(d, f);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 5; ++i) finite &= isfinite(b[i]);
    if (!(m > 0.0f) || !finite) {
        e[0] = e[1] = e[2] = e[3] = 0.0f;
        return;
    }
    const double rho = (double)kRidge * m;
    const double s = 1.0 / sqrt(((double)d + rho) * ((double)f + rho));
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double ei = b[1 + i] * s;
        e[i] = (float)ei;
        n2 += ei * ei;
    }
    const double sc = 1.0 - n2;  // at most exp(-2 cap), or below zero where rounding left the block indefinite: the cap
    e[3] = sc > exp(-2.0 * (double)kSchurCap) ? (float)(-0.5 * log(sc)) : kSchurCap;
}

// one unit's network inputs, rounded to bfloat16: its standardised stored features (clamped),
// then the block inputs as they are, then zeros
__device__ __forceinline__ void load_features(const float* __restrict__ feat, const float* __restrict__ norm,
                                              const float* __restrict__ blocks, int64_t unit, int64_t n,
                                              lds_bf* Xrow, lds_bf* Xt, int col) {
    float cpl[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (unit < n) block_inputs(blocks + 5 * unit, cpl);
#pragma unroll
    for (int i = 0; i < NIP; ++i) {
        float v = 0.0f;
        if (unit < n && i < NIN) v = fminf(fmaxf((feat[NIN * unit + i] - norm[i]) * norm[NIP + i], -kClamp), kClamp);
        else if (unit < n && i < NNET) v = cpl[i - NIN];
        const unsigned short q = f2bf(v);
        Xrow[i] = q;
        if (Xt) Xt[i * LD64 + col] = q;
    }
    if (Xt) {
#pragma unroll
        for (int i = NIP; i < 32; ++i) Xt[i * LD64 + col] = 0;
    }
}

// ------------------------------------------------------------------ inference
constexpr int kInferWaves = 4;

__global__ __launch_bounds__(64 * kInferWaves) void k_mlp_infer(const unsigned short* __restrict__ w,
                                                                const float* __restrict__ norm, float q_fallback,
                                                                const float* __restrict__ feat,
                                                                const float* __restrict__ blocks, int64_t units,
                                                                float* __restrict__ minv) {
    __shared__ unsigned short sW1[NH * LD16], sW2[NH * LD64], sW3[32 * LD64];
    __shared__ float sb1[NH], sb2[NH], sb3[NOP];
    __shared__ unsigned short sX[kInferWaves][TU * LD16], sH1[kInferWaves][TU * LD64], sH2[kInferWaves][TU * LD64];
    __shared__ float sO[kInferWaves][TU * 17];
    Weights W{(lds_bf*)sW1, (lds_bf*)sW2, (lds_bf*)sW3, sb1, sb2, sb3};
    load_weights(w, W, nullptr, nullptr);
    const int wv = threadIdx.x >> 6, l = lane();
    lds_bf* Xs = (lds_bf*)sX[wv];
    lds_bf* H1s = (lds_bf*)sH1[wv];
    lds_bf* H2s = (lds_bf*)sH2[wv];
    float* Os = sO[wv];
    const int64_t n_tiles = (units + TU - 1) / TU;
    for (int64_t tile = (int64_t)blockIdx.x * kInferWaves + wv; tile < n_tiles; tile += (int64_t)gridDim.x * kInferWaves) {
        const int64_t unit = tile * TU + l;
        load_features(feat, norm, blocks, unit, units, Xs + l * LD16, nullptr, 0);
        forward_tile(W, Xs, H1s, H2s, Os, nullptr, nullptr);
        if (unit < units) {
            const float* b = blocks + 5 * unit;
            float4* o = reinterpret_cast<float4*>(minv) + 3 * unit;
            const float d = b[0], f = b[4];
            const float m = fmaxf(d, f);
            bool finite = true;
#pragma unroll
            for (int i = 0; i < 5; ++i) finite &= isfinite(b[i]);
            if (!(m > 0.0f) || !finite) {  // no ray, or a non-finite block: an empty unit
                o[0] = o[1] = o[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                float raw[NO];
#pragma unroll
                for (int i = 0; i < NO; ++i) raw[i] = Os[l * 17 + i];
                float L[4][4];
                make_L(raw, L);
                // D^-1/2 and the normalised coupling in double (d may be subnormal)
                const double rho = (double)kRidge * m;
                const double tdd = 1.0 / sqrt((double)d + rho), tfd = 1.0 / sqrt((double)f + rho);
                const double a0 = b[1] * tdd * tfd, a1 = b[2] * tdd * tfd, a2 = b[3] * tdd * tfd;
                const float td = (float)tdd, tf = (float)tfd;
                const float e[3] = {(float)a0, (float)a1, (float)a2};
                // q = ||L L^T B~ - I||_F^2 with B~ = [[I, e], [e^T, 1]]
                float P[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float p = 0.0f;
#pragma unroll
                        for (int k = 0; k < 4; ++k) p += L[i][k] * L[j][k];
                        P[i][j] = p;
                    }
                float q = 0.0f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const float v = P[i][j] + P[i][3] * e[j] - (i == j ? 1.0f : 0.0f);
                        q += v * v;
                    }
                    const float v3 = P[i][0] * e[0] + P[i][1] * e[1] + P[i][2] * e[2] + P[i][3] - (i == 3 ? 1.0f : 0.0f);
                    q += v3 * v3;
                }
                if (!(q <= q_fallback)) {  // (a non-finite prediction falls back too)
                    // the exact block inverse in the elimination form of the block preconditioner,
                    // marked by a negative t_d
                    const double is = 1.0 / (1.0 - (a0 * a0 + a1 * a1 + a2 * a2));
                    o[0] = make_float4(-td, tf, e[0], e[1]);
                    o[1] = make_float4(e[2], (float)is, 0.0f, 0.0f);
                    o[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                } else {
                    o[0] = make_float4(td, tf, L[0][0], L[1][0]);
                    o[1] = make_float4(L[1][1], L[2][0], L[2][1], L[2][2]);
                    o[2] = make_float4(L[3][0], L[3][1], L[3][2], L[3][3]);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ training step
// One wave per workgroup (the activations of a tile are kept in both orientations).
__global__ __launch_bounds__(64) void k_mlp_train(const unsigned short* __restrict__ w,
                                                  const float* __restrict__ norm,
                                                  const float* __restrict__ feat, const float* __restrict__ blocks,
                                                  int n, float inv_n, float damp, float* __restrict__ grad,
                                                  float* __restrict__ loss) {
    __shared__ unsigned short sW1[NH * LD16], sW2[NH * LD64], sW3[32 * LD64], sW2t[NH * LD64], sW3t[NH * LD32];
    __shared__ float sb1[NH], sb2[NH], sb3[NOP];
    __shared__ unsigned short sX[TU * LD16], sXt[32 * LD64], sH1[TU * LD64], sH1t[NH * LD64], sH2[TU * LD64],
        sH2t[NH * LD64], sdO[TU * LD32], sdOt[32 * LD64], sdZ2[TU * LD64], sdZ2t[NH * LD64], sdZ1t[NH * LD64];
    __shared__ float sO[TU * 17];
    Weights W{(lds_bf*)sW1, (lds_bf*)sW2, (lds_bf*)sW3, sb1, sb2, sb3};
    load_weights(w, W, (lds_bf*)sW2t, (lds_bf*)sW3t);
    const int l = lane();
    const int64_t unit = (int64_t)blockIdx.x * TU + l;
    load_features(feat, norm, blocks, unit, n, (lds_bf*)sX + l * LD16, (lds_bf*)sXt, l);
    forward_tile(W, (lds_bf*)sX, (lds_bf*)sH1, (lds_bf*)sH2, sO, (lds_bf*)sH1t, (lds_bf*)sH2t);

    // robust loss of E = L L^T (B~ + damp I) - I for this unit and its gradient w.r.t. the raw outputs
    float dr[NO];
#pragma unroll
    for (int i = 0; i < NO; ++i) dr[i] = 0.0f;
    float lu = 0.0f;
    if (unit < n) {
        const float* b = blocks + 5 * unit;
        const float d = b[0], f = b[4];
        const float m = fmaxf(d, f);
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 5; ++i) finite &= isfinite(b[i]);
        if (m > 0.0f && finite) {  // (a non-finite block contributes nothing)
            // normalised block D^-1/2 (B + rho I) D^-1/2: unit diagonal, e / sqrt(d f) off it; in
            // double, as in inference (the ridge of a block in the subnormal range underflows FP32)
            const double rho = (double)kRidge * m;
            const double sdf = 1.0 / sqrt(((double)d + rho) * ((double)f + rho));
            const float e0 = (float)(b[1] * sdf), e1 = (float)(b[2] * sdf), e2 = (float)(b[3] * sdf);
            const float g1 = 1.0f + damp;
            const float Bn[4][4] = {{g1, 0.0f, 0.0f, e0}, {0.0f, g1, 0.0f, e1}, {0.0f, 0.0f, g1, e2},
                                    {e0, e1, e2, g1}};
            float raw[NO];
#pragma unroll
            for (int i = 0; i < NO; ++i) raw[i] = sO[l * 17 + i];
            float L[4][4];
            make_L(raw, L);
            float P[4][4], E[4][4], G[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float p = 0.0f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) p += L[i][q] * L[j][q];
                    P[i][j] = p;
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float e = (i == j) ? -1.0f : 0.0f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) e += P[i][q] * Bn[q][j];
                    E[i][j] = e;
                    lu += e * e;
                }
            float scale = 1.0f;  // d loss / d ||E||^2 of the robust per-unit loss
            if (lu > kKappa) {
                scale = sqrtf(kKappa / lu);
                lu = 2.0f * sqrtf(kKappa * lu) - kKappa;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float g = 0.0f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) g += E[i][q] * Bn[q][j];
                    G[i][j] = 2.0f * inv_n * scale * g;
                }
            int k = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j, ++k) {
                    float dl = 0.0f;  // ((G + G^T) L)_ij
#pragma unroll
                    for (int q = 0; q < 4; ++q) dl += (G[i][q] + G[q][i]) * L[q][j];
                    dr[k] = (i == j) ? dl * sigmoid(raw[k]) : dl;
                }
        }
    }
    // loss sum
    {
        float t = lu * inv_n;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        if (l == 0) atomicAdd(loss, t);
    }
    // dO rows (this unit) and columns (transpose)
    lds_bf* dOs = (lds_bf*)sdO;
    lds_bf* dOt = (lds_bf*)sdOt;
#pragma unroll
    for (int o = 0; o < 32; ++o) {
        const unsigned short q = f2bf(o < NO ? dr[o] : 0.0f);
        dOs[l * LD32 + o] = q;
        dOt[o * LD64 + l] = q;
    }
    // dH2 = dO W3, dZ2 = dH2 * (H2 > 0)
    {
        f16v acc[2][2];
        zero(acc);
        wgemm<2, 2, 32 / 8>(dOs, LD32, (lds_bf*)sW3t, LD32, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int u = crow(mb, v), hh = ccol(nb);
                    const float hv = bf2f(((lds_bf*)sH2)[u * LD64 + hh]);
                    const unsigned short q = f2bf(hv > 0.0f ? acc[mb][nb][v] : 0.0f);
                    ((lds_bf*)sdZ2)[u * LD64 + hh] = q;
                    ((lds_bf*)sdZ2t)[hh * LD64 + u] = q;
                }
    }
    // dH1 = dZ2 W2, dZ1 = dH1 * (H1 > 0) (only its transpose is needed)
    {
        f16v acc[2][2];
        zero(acc);
        wgemm<2, 2, NH / 8>((lds_bf*)sdZ2, LD64, (lds_bf*)sW2t, LD64, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int u = crow(mb, v), hh = ccol(nb);
                    const float hv = bf2f(((lds_bf*)sH1)[u * LD64 + hh]);
                    ((lds_bf*)sdZ1t)[hh * LD64 + u] = f2bf(hv > 0.0f ? acc[mb][nb][v] : 0.0f);
                }
    }
    // weight gradients: contractions over the tile's units
    {
        f16v acc[1][2];  // dW3[o][h] = sum_u dO[u][o] H2[u][h]
        zero(acc);
        wgemm<1, 2, TU / 8>(dOt, LD64, (lds_bf*)sH2t, LD64, acc);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int o = crow(0, v), hh = ccol(nb);
                if (o < NO && acc[0][nb][v] != 0.0f) atomicAdd(grad + OFF_W3 + o * NH + hh, acc[0][nb][v]);
            }
    }
    {
        f16v acc[2][2];  // dW2[ho][hi] = sum_u dZ2[u][ho] H1[u][hi]
        zero(acc);
        wgemm<2, 2, TU / 8>((lds_bf*)sdZ2t, LD64, (lds_bf*)sH1t, LD64, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int ho = crow(mb, v), hi = ccol(nb);
                    if (acc[mb][nb][v] != 0.0f) atomicAdd(grad + OFF_W2 + ho * NH + hi, acc[mb][nb][v]);
                }
    }
    {
        f16v acc[2][1];  // dW1[h][i] = sum_u dZ1[u][h] X[u][i]
        zero(acc);
        wgemm<2, 1, TU / 8>((lds_bf*)sdZ1t, LD64, (lds_bf*)sXt, LD64, acc);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int hh = crow(mb, v), i = ccol(0);
                if (i < NNET && acc[mb][0][v] != 0.0f) atomicAdd(grad + OFF_W1 + hh * NIP + i, acc[mb][0][v]);
            }
    }
    // bias gradients: row sums of the transposed gradients
    {
        float s1 = 0.0f, s2 = 0.0f;
        for (int u = 0; u < TU; ++u) {
            s1 += bf2f(((lds_bf*)sdZ1t)[l * LD64 + u]);
            s2 += bf2f(((lds_bf*)sdZ2t)[l * LD64 + u]);
        }
        if (s1 != 0.0f) atomicAdd(grad + OFF_B1 + l, s1);
        if (s2 != 0.0f) atomicAdd(grad + OFF_B2 + l, s2);
        if (l < NO) {
            float s3 = 0.0f;
            for (int u = 0; u < TU; ++u) s3 += bf2f(dOt[l * LD64 + u]);
            if (s3 != 0.0f) atomicAdd(grad + OFF_B3 + l, s3);
        }
    }
}

// Adam on the FP32 master weights; refreshes the bfloat16 copy and clears the gradient.
__global__ void k_adam(float* __restrict__ w32, unsigned short* __restrict__ wbf, float* __restrict__ m,
                       float* __restrict__ v, float* __restrict__ g, int t, float lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NW; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w32[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w32[i] = wi;
        wbf[i] = f2bf(wi);
        g[i] = 0.0f;
    }
}

// Standardisation of a training set: workgroup i sums feature i over the n rows in FP64, in a
// fixed order (deterministic), and writes mu_i and s_i = 1 / max(std_i, 1e-3), std the
// population standard deviation; the padding inputs get 0.
constexpr int kStatsBlock = 256;
__global__ __launch_bounds__(kStatsBlock) void k_feature_stats(const float* __restrict__ feat, int64_t n,
                                                               float* __restrict__ norm) {
    __shared__ double red[2][kStatsBlock];
    const int i = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += kStatsBlock) {
        const double v = feat[NIN * r + i];
        s1 += v;
        s2 += v * v;
    }
    red[0][threadIdx.x] = s1;
    red[1][threadIdx.x] = s2;
    __syncthreads();
    for (int h = kStatsBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = n > 0 ? red[0][0] / (double)n : 0.0;
        const double var = n > 0 ? fmax(red[1][0] / (double)n - mu * mu, 0.0) : 0.0;
        norm[i] = (float)mu;
        norm[NIP + i] = (float)(1.0 / fmax(sqrt(var), 1e-3));
    }
    // workgroup i also zeroes padding slots NIN + i, NIN + i + NIN, ... of both halves
    if (threadIdx.x == 0) {
        for (int j = NIN + i; j < NIP; j += NIN) {
            norm[j] = 0.0f;
            norm[NIP + j] = 0.0f;
        }
    }
}

__global__ void k_zero1(float* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

}  // namespace

hipError_t launch_mlp_infer(const uint16_t* w, const float* norm, float q_fallback, const float* feat,
                            const float* blocks, int64_t units, float* minv, hipStream_t st) {
    const int64_t tiles = (units + TU - 1) / TU;
    int64_t g = (tiles + kInferWaves - 1) / kInferWaves;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)g), dim3(64 * kInferWaves), 0, st, w, norm, q_fallback, feat, blocks,
                       units, minv);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float* w32, uint16_t* wbf, float* m, float* v, int t, float lr, float damp,
                            const float* norm, const float* feat, const float* blocks, int n, float* loss, float* grad,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, st, loss, 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_mlp_train, dim3((unsigned)((n + TU - 1) / TU)), dim3(64), 0, st, wbf, norm, feat, blocks,
                           n, 1.0f / (float)n, damp, grad, loss);
    }
    hipLaunchKernelGGL(k_adam, dim3((NW + 255) / 256), dim3(256), 0, st, w32, wbf, m, v, grad, t, lr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free training step
// The gradient accumulator of a training step for callers that cannot allocate device memory: a
// file-scope device array of one gradient (PERF_MLP_NW floats), one copy per GPU, held until the
// process ends.  On the host the array's name is only a stand-in: its device address is looked
// up once per device (the device current at the first call) with hipGetSymbolAddress and kept,
// and kernels receive that address.  Every call on a GPU shares its copy, so calls that overlap
// on one GPU race; each call clears it first.
constexpr int kStaticGradFloats = ((NW + 63) / 64) * 64;
static __device__ __align__(256) float scratch[kStaticGradFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices];

hipError_t static_grad_scratch(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

hipError_t launch_mlp_train_static(float* w32, uint16_t* wbf, float* m, float* v, int t, float lr, float damp,
                                   const float* norm, const float* feat, const float* blocks, int n, float* loss,
                                   hipStream_t st) {
    float* grad = nullptr;
    hipError_t e = static_grad_scratch(&grad);
    if (e != hipSuccess) return e;
    // an earlier call that failed part-way may have left partial sums: start from zero (a fill
    // kernel, no memset)
    hipLaunchKernelGGL(k_zero1, dim3((kStaticGradFloats + 255) / 256), dim3(256), 0, st, grad, kStaticGradFloats);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mlp_train(w32, wbf, m, v, t, lr, damp, norm, feat, blocks, n, loss, grad, st);
}

hipError_t launch_feature_stats(const float* feat, int64_t n, float* norm, hipStream_t st) {
    hipLaunchKernelGGL(k_feature_stats, dim3(NIN), dim3(kStatsBlock), 0, st, feat, n, norm);
    return hipGetLastError();
}

}  // namespace perf
