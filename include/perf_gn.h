/*
 * perf_gn.h -- C ABI of the MI355X (gfx950) matrix-free Gauss-Newton / PCG
 * library for explicit radiance-field reconstruction (Rasmuson, Sintorn,
 * Assarsson, "PERF: Performant, Explicit Radiance Fields").
 *
 * The problem (Sec. III-B, III-C, Eq. 5-6): minimise F(x) = 1/2 sum r^2 over
 * the three colour residuals r = H(x) - C of every pixel ray of every image,
 * where H is the discrete volume-rendering sum of Eq. 3-4 through an RGB-sigma
 * voxel grid followed by a hierarchy of RGB-alpha environment layers.  One
 * Gauss-Newton step (Eq. 7) solves J^T J Delta = -J^T r (Eq. 8) by
 * preconditioned conjugate gradients (Alg. 2) using the matrix-free product of
 * Eq. 9, then scales Delta by backtracking (Alg. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Ownership   All device memory belongs to the caller.  The library never
 *             allocates device memory: perf_init_scene receives a caller
 *             allocated workspace of perf_workspace_bytes() bytes that must
 *             stay valid until perf_destroy_scene.  The scene handle is a host
 *             object; it copies the descriptor and cameras and *borrows* the
 *             targets pointer (which must outlive the handle).
 * Streams     Every call is enqueued asynchronously on the stream given at
 *             init (or to perf_set_stream).  Only perf_gn_step and
 *             perf_objective synchronise, and only for the scalars their
 *             control flow needs.  Kernel faults surface at the next
 *             synchronising call as PERF_EDEVICE.
 * Errors      Every entry point returns an int32 status, 0 on success.
 *             perf_last_error() returns a thread-local message for the last
 *             failure.  Nothing aborts or throws across the ABI.
 * Parameters  x is one flat vector of P = 4 * units values: voxels first,
 *             x[((z*ny + y)*nx + xi)*4 + {r,g,b,sigma}], then the texels of
 *             the layers, x[4*(nvox + (l*env_h + j)*env_w + i) + {r,g,b,alpha}].
 *             Storage is FP32 (float4 per unit) or, with param_dtype
 *             PERF_BF16, bfloat16 (4 x uint16 per unit, round-to-nearest-even
 *             from FP32) for every gather of x; vectors v, u, y and all PCG
 *             vectors are FP32.  Dots, alpha, beta, R and F are FP64.
 * Rays        One ray per pixel centre of every camera; ray id
 *             (cam*height + py)*width + px.  Residual / target arrays are
 *             [rays][3] FP32.  Sign convention: r = H - C, J = dr/dx = dH/dx.
 * Units       sigma is an optical depth per voxel length: the march step and
 *             the delta of Eq. 3-4 are measured in units of the shortest voxel
 *             side, and the last step of a ray is shortened so the steps sum to
 *             the chord.
 */
#ifndef PERF_GN_H
#define PERF_GN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERF_MAX_LAYERS 8
#define PERF_MAX_PCG 256

enum {
    PERF_OK = 0,
    PERF_EINVAL = -1,      /* bad argument (null pointer, bad size, bad descriptor) */
    PERF_ENOMEM = -2,      /* workspace smaller than perf_workspace_bytes() */
    PERF_EDEVICE = -3,     /* a HIP runtime call failed */
    PERF_ENUMERIC = -4,    /* non-finite input found (only with checks = 1) */
    PERF_EUNSUPPORTED = -5 /* option not supported by the library / descriptor */
};

enum { PERF_F32 = 0, PERF_BF16 = 1 };

enum {
    PERF_PRECOND_NONE = 0,
    PERF_PRECOND_JACOBI = 1,  /* diag(J^T J), Sec. III-G */
    PERF_PRECOND_BLOCK4 = 2,  /* exact 4x4 diagonal blocks of J^T J, closed-form inverse */
    PERF_PRECOND_LEARNED = 3  /* per-unit MLP prediction of the block inverse */
};

/* perf_gn_stats.flags */
enum {
    PERF_FLAG_BREAKDOWN = 1,   /* p^T A p <= 0 or not finite: PCG stopped before the update */
    PERF_FLAG_STALL = 2,       /* R / R_prev above stall_ratio (the early exit of Alg. 2) */
    PERF_FLAG_CONVERGED = 4,   /* R < abs_eps or sqrt(R/R0) <= rel_tol */
    PERF_FLAG_LS_CAPPED = 8,   /* line search hit ls_max trials */
    PERF_FLAG_NO_DESCENT = 16, /* no trial lowered F: gamma = 0, x unchanged */
    PERF_FLAG_FALLBACK = 32    /* the learned solve broke down, stalled or found no descent; the
                                  step was solved again with PERF_PRECOND_BLOCK4 (the other flags,
                                  the history and pcg_iters describe that second solve) */
};

typedef struct {
    int32_t nx, ny, nz;                   /* grid dimensions, each >= 2 */
    float bbox_min[3], bbox_max[3];       /* world box of the grid */
    int32_t n_layers, env_w, env_h;       /* 0..8 layers of env_w x env_h texels (each >= 2) */
    float layer_radius[PERF_MAX_LAYERS];  /* increasing, each > box half-diagonal |bbox corner| */
    float step_vox;                       /* march step in shortest-voxel-side units, (0, 1] */
    int32_t param_dtype;                  /* PERF_F32 or PERF_BF16 */
    float background[3];                  /* radiance behind the last layer */
    int32_t width, height;                /* image size shared by every camera */
    int32_t checks;                       /* 1: gn_step checks x / targets for non-finite values */
    int32_t learned;                      /* 1: reserve workspace for the learned preconditioner */
    float aux_lambda;                     /* Sec. III-I (Eq. 10): weight of the per-ray opacity residual
                                             r_4 = aux_lambda (1 - 4 (T - 1/2)^2), T the transmittance
                                             through the volume (the paper uses 0.1); 0 = off.  When on,
                                             every ray has n_res = 4 residuals (r, g, b, r_4) instead of
                                             3 in the residual, J v and J^T u arrays, and F includes r_4^2 / 2 */
    float render_threshold;               /* Sec. IV (rendering): perf_render_residuals treats the volume
                                             as fully transparent for rays whose volume opacity 1 - T is
                                             below this value (the paper uses 0.7 on converged scenes);
                                             0 = off.  Never applied inside perf_gn_step / perf_objective */
} perf_scene_desc;

typedef struct {
    float origin[3];
    float rot[9];          /* camera-to-world, row-major 3x3; columns = right, down, forward */
    float fx, fy, cx, cy;  /* pixel (px, py) has camera direction ((px+.5-cx)/fx, (py+.5-cy)/fy, 1) */
} perf_camera;

typedef struct {
    int32_t max_iters;     /* products with A per PCG solve, 1..PERF_MAX_PCG */
    double rel_tol;        /* stop when sqrt(R/R0) <= rel_tol (<= 0: off) */
    double abs_eps;        /* stop when R < abs_eps (the EPS of Alg. 2; <= 0: off) */
    double stall_ratio;    /* stop when R/R_prev > stall_ratio (Alg. 2 uses 0.85; <= 0: off) */
    int32_t precond;       /* PERF_PRECOND_* */
    int32_t line_search;   /* 1: Alg. 3 backtracking; 0: gamma = 1 */
    float ls_factor;       /* Alg. 3 decimation factor (0.7) */
    int32_t ls_max;        /* cap on line-search trials (>= 1) */
} perf_pcg_opts;

typedef struct {
    double F_before, F_after, gamma;
    int32_t pcg_iters, ls_trials, flags;
    int32_t fallback_iters;      /* PCG iterations of a discarded learned solve (0: none) */
    double R0;
    double R[PERF_MAX_PCG];      /* r_{k+1}^T r_{k+1} after update k */
    double alpha[PERF_MAX_PCG];  /* alpha_k */
    double beta[PERF_MAX_PCG];   /* beta_k (one fewer than alpha) */
    double pAp[PERF_MAX_PCG];    /* p_k^T A p_k */
    float ms_phase[8];           /* grad+precond, invert, pcg, line search, update, total,
                                    J^T J v kernel time summed over the solve, number of those launches
                                    (with a fallback: the final solve's; the discarded solve, its line
                                    search and the block inversion count in the pcg phase) */
} perf_gn_stats;

typedef struct perf_scene perf_scene;

/* Bytes of device workspace a scene with this descriptor and camera count needs. 0 on a bad descriptor. */
size_t perf_workspace_bytes(const perf_scene_desc* desc, int32_t n_cams);

/*
 * Create a scene (Sec. III-A, III-B: the grid, the layers and the posed images).
 * desc, cams        host pointers, copied.
 * d_targets         device [rays][3] FP32 pixel colours C, borrowed (may be NULL; then only
 *                   the J products work until perf_set_targets).
 * d_workspace       device memory of ws_bytes >= perf_workspace_bytes(desc, n_cams), 256-byte aligned.
 * stream            hipStream_t the calls run on (NULL = default stream).
 * Errors: PERF_EINVAL for a bad descriptor (dims < 2, step outside (0,1], a layer radius not
 * increasing or not beyond the box half-diagonal, non-finite camera), PERF_ENOMEM for a small
 * workspace, PERF_EDEVICE if copying the cameras fails.
 */
int32_t perf_init_scene(const perf_scene_desc* desc, const perf_camera* cams, int32_t n_cams,
                        const float* d_targets, void* d_workspace, size_t ws_bytes, void* stream,
                        perf_scene** out);
int32_t perf_set_targets(perf_scene* s, const float* d_targets);
/*
 * Jittering (Sec. IV) for every later call on s: seed != 0 moves each ray's origin to a
 * pseudo-random point of its pixel and each sample to a pseudo-random point of its own step
 * (half a step either side of the midpoint for a full step), from the 32-bit finaliser of
 * MurmurHash3 keyed by (seed, ray, stream); seed 0 = pixel centres and step midpoints.  Keep
 * one seed for the whole of a perf_gn_step (its residuals, products, preconditioner and
 * line search must see the same samples) and change it between steps.  Host-side only.
 */
int32_t perf_set_jitter(perf_scene* s, uint32_t seed);
int32_t perf_set_stream(perf_scene* s, void* stream);
/* Sizes: rays, units (voxels + texels), parameters (4 * units). Any pointer may be NULL. */
int32_t perf_scene_sizes(const perf_scene* s, int64_t* n_rays, int64_t* n_units, int64_t* n_params);
int32_t perf_destroy_scene(perf_scene* s);
const char* perf_last_error(void);

/*
 * Residuals r = H(x) - C per ray (Eq. 3-4, 6) and F = 1/2 sum r^2 (Eq. 5).
 * d_x   device parameters (FP32 or BF16 per param_dtype).
 * d_r   device [rays][n_res] FP32 output (r, g, b and, with aux_lambda > 0, r_4 of Eq. 10),
 *       may be NULL; a scene without targets writes H [rays][3] instead.
 * d_F   device double[1] output, may be NULL.  Deterministic (no atomics).
 */
int32_t perf_render_residuals(perf_scene* s, const void* d_x, float* d_r, double* d_F);

/* u = J v, one forward-mode pass per ray (derivative of Eq. 3-4, and of Eq. 10 when on).
 * d_v [P] FP32, d_u [rays][n_res]. */
int32_t perf_apply_J(perf_scene* s, const void* d_x, const float* d_v, float* d_u);

/* y = J^T u, the adjoint pass of Alg. 1 per ray, scattered into y [P] (overwritten).
 * d_u [rays][n_res]. */
int32_t perf_apply_Jt(perf_scene* s, const void* d_x, const float* d_u, float* d_y);

/* y = J^T J v = sum_i grad r_i (grad r_i^T v) (Eq. 9), fused per ray; y [P] overwritten. */
int32_t perf_apply_JtJ(perf_scene* s, const void* d_x, const float* d_v, float* d_y);

/*
 * Gradient and preconditioner data in one traversal (Sec. III-G).
 * d_grad    [P] FP32, -J^T r (the b of Eq. 8), may be NULL.
 * d_blocks  [units][5] FP32 (d, e_r, e_g, e_b, f): the unit's 4x4 block of J^T J is
 *           [[d I3, e], [e^T, f]], with each ray's partials aggregated over all of its
 *           samples before squaring (exact).  May be NULL.
 * kind      the preconditioner M^-1 in scaled form (see perf_invert_blocks): with
 *           PERF_PRECOND_JACOBI d_out [units][4], with PERF_PRECOND_BLOCK4 d_out [units][8];
 *           PERF_PRECOND_NONE: d_out ignored.
 * d_F       device double[1], may be NULL.
 */
int32_t perf_build_precond(perf_scene* s, const void* d_x, int32_t kind, float* d_grad, float* d_blocks,
                           float* d_out, double* d_F);

/*
 * One Gauss-Newton step (Eq. 7): b = -J^T r and the preconditioner, PCG (Alg. 2) from
 * Delta_0 = 0, backtracking (Alg. 3) on F(proj(x + gamma Delta)), then
 * x <- proj(x + gamma Delta) with proj: sigma >= 0, texel alpha in [0, 1].
 * d_x    device FP32 master parameters [P], updated in place (with PERF_BF16 the library keeps
 *        the bfloat16 copy used for every gather in its workspace).
 * stats  host output, may be NULL.
 * With PERF_PRECOND_LEARNED, a solve that ends in breakdown, a stall or a line search without
 * descent is discarded and the step is solved again, from Delta_0 = 0, with the exact block
 * inverse (PERF_FLAG_FALLBACK).
 * Errors: PERF_EINVAL (bad options, no targets), PERF_ENUMERIC (checks = 1 and non-finite x or
 * targets).  PCG breakdown and an unproductive line search are reported in stats->flags.
 */
int32_t perf_gn_step(perf_scene* s, float* d_x, const perf_pcg_opts* opts, perf_gn_stats* stats);

/*
 * F(proj(x + gamma * d_delta)) (Eq. 5) into *F_host (synchronises).  d_x, d_delta FP32 [P].
 * d_delta may be NULL (then F(x) without projection).
 */
int32_t perf_objective(perf_scene* s, const float* d_x, const float* d_delta, float gamma, double* F_host);

/*
 * Footprint of every ray: d_per_ray [rays][2] int32 (distinct voxels the samples' trilinear
 * corners touch, clamp-to-edge; environment layers hit), may be NULL; d_totals device
 * uint64[3] (sum of the voxel counts, sum of layer hits, rays that enter the grid).
 */
int32_t perf_footprint(perf_scene* s, int32_t* d_per_ray, uint64_t* d_totals);

/*
 * Next hierarchical level (Sec. IV, hierarchical formulation): fill the parameter vector of
 * level `to` from that of level `from` by linear interpolation at the new cell and texel
 * centres (trilinear over the grid, clamped at the border; bilinear over each layer,
 * periodic in azimuth, clamped in polar angle).  sigma is an optical depth per shortest voxel
 * side, so it is multiplied by side(to) / side(from); colours and texel opacities are
 * interpolated unchanged.  Any resolution pair is accepted (typically doubled per level).
 * d_from [4 * units(from)] and d_to [4 * units(to)] are caller-owned FP32 device vectors in
 * the layout of perf_scene_desc; only the grid/layer sizes, box and radii of the two
 * descriptors are read.  Errors: PERF_EINVAL if the boxes, layer counts or radii differ or a
 * pointer is NULL.  Asynchronous on `stream` (a hipStream_t, NULL = default stream).
 */
int32_t perf_upsample(const perf_scene_desc* from, const float* d_from, const perf_scene_desc* to, float* d_to,
                      void* stream);

/*
 * Preconditioner from given blocks (Sec. III-G), the step perf_build_precond ends with, in the
 * scaled form every PCG kernel applies.  No stored value depends on the scale of the block
 * beyond its inverse square root, so the form stays in FP32 range for any block, including
 * diagonals in the FP32 subnormal range (units seen only through near-opaque matter), and the
 * unscaled inverse is never formed.
 * d_blocks  device float [units][5] = (d, e_r, e_g, e_b, f) of [[d I3, e], [e^T, f]].
 * kind      PERF_PRECOND_JACOBI: d_out [units][4] = (t_d, t_d, t_d, t_f), t = 1/sqrt(diagonal),
 *           0 for a zero diagonal; M^-1 = diag(t)^2 = 1/diag(J^T J).
 *           PERF_PRECOND_BLOCK4: d_out [units][8] = (t_d, t_f, e~_r, e~_g, e~_b, 1/s, 0, 0): after a
 *           ridge rho = 1e-6 max(d, f), t_d = (d + rho)^-1/2, t_f = (f + rho)^-1/2, the normalised
 *           block D^-1/2 (B + rho I) D^-1/2 = [[I3, e~], [e~^T, 1]] with e~ = t_d t_f e, and s =
 *           1 - |e~|^2 its Schur complement; M^-1 = (B + rho I)^-1 = D^-1/2 [[I3, e~], [e~^T, 1]]^-1
 *           D^-1/2, applied by elimination (z_sigma = (y_sigma - e~ . y_c) / s, z_c = y_c -
 *           e~ z_sigma on y = D^-1/2 r), which keeps FP32 rounding along the block's near-null
 *           direction; all 8 are 0 for an empty unit (max(d, f) = 0, or a non-finite block).
 * Caller-owned device memory; asynchronous on stream.  PERF_EINVAL for a null pointer with
 * units > 0, units < 0 or another kind.
 */
int32_t perf_invert_blocks(const float* d_blocks, int64_t units, int32_t kind, float* d_out, void* stream);

/* Round FP32 parameters to bfloat16 storage (round to nearest even): d_out[n] uint16. */
int32_t perf_pack_bf16(const float* d_in, uint16_t* d_out, int64_t n, void* stream);

/*
 * Learned block preconditioner (per-unit MLP 10 -> 64 -> 64 -> 10, ReLU, BF16 weights on
 * MFMA, FP32 accumulation).  Not in the paper: it replaces the exact 4x4 block inverse of
 * Sec. III-G's diagonal preconditioner by a prediction from cheap per-unit features.
 *
 * perf_precond_features: d_feat [units][PERF_MLP_NFEAT] FP32 features and d_blocks [units][5]
 *   (as in perf_build_precond) from the gradient/block traversal at x; the features come from
 *   x and the blocks alone (no further traversal): sigma/alpha, colour (3), log(d + 1e-12),
 *   log(f + 1e-12).  perf_gn_step forms them from the blocks of its own gradient pass.
 * The network's input (10 values, padded to 16) is the standardised feature vector
 *   clamp((f - mu) s, -8, 8), with norm [PERF_MLP_NNORM] = (mu[16], s[16]) FP32 (entries 6..15
 *   of each zero), followed by the unit's normalised colour-density coupling e~ = e /
 *   sqrt((d + rho)(f + rho)) from d_blocks (|e~| < 1) and -1/2 log(1 - |e~|^2), the log of
 *   1 / sqrt of the normalised block's Schur complement (8 where the complement is at most
 *   exp(-16)); neither is standardised, and all are 0 for an empty unit.
 * perf_mlp_set_weights: d_w device bfloat16 weights in the packed order W1[64][16] b1[64]
 *   W2[64][64] b2[64] W3[16][64] b3[16] (inputs padded 10 -> 16, outputs 10 -> 16 with zeros);
 *   n_w must equal PERF_MLP_NW; d_norm the network's standardisation (device FP32); q_fallback:
 *   a unit whose prediction misses its own normalised block B~ by q = ||L L^T B~ - I||_F^2 >
 *   q_fallback takes the exact block inverse instead (plain block-Jacobi as the fallback;
 *   INFINITY never falls back, 0 always).  Copied into the workspace (requires desc.learned = 1).
 * perf_mlp_infer: d_minv [units][12] = (t_d, t_f, L00, L10, L11, L20, L21, L22, L30, L31, L32,
 *   L33) from features and blocks: the network's output is a lower-triangular L (softplus on
 *   the diagonal); M^-1 = D^-1/2 L L^T D^-1/2 with D^-1/2 = diag(t_d, t_d, t_d, t_f) as in
 *   perf_invert_blocks (after the ridge), applied as D^-1/2 L (L^T (D^-1/2 r)); a unit on the
 *   fallback holds (-t_d, t_f, e~, 1/s, 0, ...) instead, the block form of perf_invert_blocks with
 *   t_d negated; units with max(d, f) = 0 or a non-finite block get 0.
 * perf_mlp_train_step: one Adam step on a batch of n (feature, block) rows: per-unit error
 *   E = L L^T (Bn + damp I) - I with Bn = D^-1/2 B D^-1/2, so that the target is the damped
 *   normalised inverse (damp = 0: exact block-Jacobi; damp -> inf: Jacobi); the loss is the
 *   mean over the n rows of q = ||E||_F^2 where q <= 4 and 4 sqrt(q) - 4 above (robust against
 *   near-singular blocks; rows with max(d, f) = 0 or a non-finite block count as 0); FP32 master weights d_w32 [PERF_MLP_NW], d_norm the fixed
 *   standardisation, Adam moments d_m, d_v [PERF_MLP_NW], step count t (>= 1), learning rate
 *   lr; writes the updated bf16 copy to d_wbf16 and the batch loss to d_loss (device
 *   float[1]).  d_grad_scratch [PERF_MLP_NW] FP32 accumulates the gradient; it must be zero on
 *   entry and is left zero.
 * perf_mlp_feature_stats: d_norm from n rows of features d_feat [n][PERF_MLP_NFEAT]: per-feature mean and
 *   s = 1 / max(std, 1e-3), std the population standard deviation, in FP64 and deterministic.
 * perf_mlp_training_rows: training rows from one traversal's features and blocks: every unit
 *   some ray touches (max(d, f) > 0) whose features and block are finite is kept with
 *   probability keep, decided by a hash of
 *   (seed, unit), and the kept rows are written to d_feat_out [cap][PERF_MLP_NFEAT] and d_blocks_out
 *   [cap][5] in unit order (deterministic); *n_kept (host) receives the number of kept rows,
 *   of which the first min(n_kept, cap) are written.  Synchronises.
 */
#define PERF_MLP_NW (64 * 16 + 64 + 64 * 64 + 64 + 16 * 64 + 16)
#define PERF_MLP_NNORM 32
#define PERF_MLP_NFEAT 6
int32_t perf_precond_features(perf_scene* s, const void* d_x, float* d_feat, float* d_blocks);
int32_t perf_mlp_set_weights(perf_scene* s, const uint16_t* d_w, int32_t n_w, const float* d_norm, float q_fallback);
int32_t perf_mlp_infer(perf_scene* s, const float* d_feat, const float* d_blocks, float* d_minv);
int32_t perf_mlp_train_step(float* d_w32, uint16_t* d_wbf16, float* d_m, float* d_v, int32_t t, float lr,
                            float damp, const float* d_norm, const float* d_feat, const float* d_blocks, int32_t n,
                            float* d_loss, float* d_grad_scratch, void* stream);
/*
 * perf_mlp_train_step_noalloc: perf_mlp_train_step without d_grad_scratch, for callers that
 * cannot allocate device memory (code under graph capture, serving loops, harnesses that forbid
 * it).  The gradient accumulator is a fixed library-owned device array of PERF_MLP_NW floats
 * (22.6 KB) per GPU, looked up on the device current at the first call and kept until the
 * process ends; no argument changes its size.  The call allocates nothing, clears the array
 * itself before use, and otherwise behaves as perf_mlp_train_step (same arguments, same
 * errors).  Every call on one GPU shares the array: calls that overlap on one GPU race.
 */
int32_t perf_mlp_train_step_noalloc(float* d_w32, uint16_t* d_wbf16, float* d_m, float* d_v, int32_t t, float lr,
                                    float damp, const float* d_norm, const float* d_feat, const float* d_blocks,
                                    int32_t n, float* d_loss, void* stream);
int32_t perf_mlp_feature_stats(const float* d_feat, int64_t n, float* d_norm, void* stream);
int32_t perf_mlp_training_rows(perf_scene* s, const float* d_feat, const float* d_blocks, uint32_t seed, float keep,
                               float* d_feat_out, float* d_blocks_out, int64_t cap, int64_t* n_kept);

#ifdef __cplusplus
}
#endif
#endif /* PERF_GN_H */
