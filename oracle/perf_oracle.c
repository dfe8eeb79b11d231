/*
 * FP64 CPU oracle for the PERF Gauss-Newton path (Rasmuson, Sintorn, Assarsson,
 * "PERF: Performant, Explicit Radiance Fields").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the tests, by the smoke check
 * and by the benchmark's CPU-baseline leg.  It shares no code with the HIP path
 * and must never be called from the product path.
 *
 * Plain, slow, obviously correct: every ray is traced in double precision, its
 * samples are listed explicitly, the partial derivatives of the discrete
 * rendering sum are written out from their definition, and the ray's gradient
 * row (a small sparse map unit -> partials) is formed by sorting and merging.
 * J*v, J^T*u, J^T*J*v, the gradient and the diagonal blocks of J^T*J are then
 * plain sparse linear algebra over those rows.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - sigma is an optical depth per voxel length: delta is measured in units of
 *    the shortest voxel side (Sec. III-A, Eq. 3-4; Sec. IV-C step length).
 *  - the last step of a ray is shortened so that the steps sum to the chord.
 *  - samples sit at the midpoints of their steps; trilinear interpolation is
 *    cell centred with clamp-to-edge (Sec. IV "hardware interpolation").
 *  - environment layers are spheres centred at the origin, hit at the far root,
 *    composited outward with the texel opacity used directly as alpha, then a
 *    constant background colour (Sec. III-A, Fig. "scene", Sec. IV-C).
 *  - T is exclusive: the first sample sees T = 1 (expanded form in Sec. III-E).
 *  - the partial with respect to sigma includes the dependence of everything
 *    behind the sample, environment layers and background included
 *    (Alg. 1 with its accumulator started at the environment contribution).
 *
 * Parity unpinned: nothing.  Every function is pinned by the CPU tests
 * (closed forms, finite differences, dense brute force, textbook identities).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LAYERS 8

typedef struct {
    int32_t nx, ny, nz;
    double bmin[3], bmax[3];
    int32_t n_layers, env_w, env_h;
    double radius[ORC_MAX_LAYERS];
    double step;          /* Delta, in units of the shortest voxel side */
    double bg[3];
    int32_t n_cams, width, height;
    const double *cam_origin; /* [n_cams][3] */
    const double *cam_rot;    /* [n_cams][9] row-major, columns right/down/forward */
    const double *cam_intr;   /* [n_cams][4] fx, fy, cx, cy */
    double aux_lambda;        /* Sec. III-I: weight of the opacity residual, 0 = off */
    uint32_t jitter_seed;     /* Sec. IV (jittering): 0 = pixel centres and step midpoints */
} orc_scene;

/* One entry of a ray's Jacobian before merging: parameter unit, dH/dc (same for
 * the three colour channels of that unit) and dH/d(sigma or alpha) per channel. */
typedef struct {
    int64_t unit;
    double a;
    double s[3];
    double q;           /* d r_4 / d sigma of the auxiliary residual (0 for texels or when off) */
} orc_entry;

typedef struct {
    double H[3];
    double T_exit;      /* transmittance through the voxel grid */
    double T_end;       /* transmittance after the last environment layer */
    double aux;         /* the auxiliary residual r_4 (0 when off) */
    int32_t hit_box;
    int32_t n_layers_hit;
    int64_t n_samples;
    int64_t n_entries;  /* after merging */
    int64_t n_vox_units;/* unique voxel units after merging */
    orc_entry *entries; /* caller-provided buffer */
} orc_ray_out;

static int64_t orc_nvox(const orc_scene *s) { return (int64_t)s->nx * s->ny * s->nz; }
static int64_t orc_units(const orc_scene *s) {
    return orc_nvox(s) + (int64_t)s->n_layers * s->env_w * s->env_h;
}
static double orc_hmin(const orc_scene *s) {
    double hx = (s->bmax[0] - s->bmin[0]) / s->nx;
    double hy = (s->bmax[1] - s->bmin[1]) / s->ny;
    double hz = (s->bmax[2] - s->bmin[2]) / s->nz;
    double h = hx < hy ? hx : hy;
    return h < hz ? h : hz;
}

/* Largest number of samples any ray can take: the box diagonal over the step. */
static int64_t orc_max_samples(const orc_scene *s) {
    double dx = s->bmax[0] - s->bmin[0], dy = s->bmax[1] - s->bmin[1], dz = s->bmax[2] - s->bmin[2];
    double diag = sqrt(dx * dx + dy * dy + dz * dz);
    return (int64_t)ceil(diag / orc_hmin(s) / s->step) + 2;
}

int64_t orc_entry_capacity(const orc_scene *s) {
    return orc_max_samples(s) * 8 + (int64_t)s->n_layers * 4 + 8;
}

/*
 * Jittering (Sec. IV): uniform numbers in [0, 1) from a counter-based generator, the
 * 32-bit finaliser of MurmurHash3 (Appleby): stream 0 and 1 are a ray's sub-pixel offsets,
 * stream 2 + k the position of its sample k inside its step.  u = (h >> 8) 2^-24, exact in
 * single and double precision.  Seed 0 switches jittering off (pixel centre, step midpoint).
 */
static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
static uint32_t jitter_key(uint32_t seed, int64_t ray) { return fmix32(fmix32(seed) ^ (uint32_t)ray); }
static double jitter_u(uint32_t key, uint32_t stream) {
    return (double)(fmix32(key + stream * 0x9e3779b9u) >> 8) * (1.0 / 16777216.0);
}

double orc_jitter_u(uint32_t seed, int64_t ray, uint32_t stream) { return jitter_u(jitter_key(seed, ray), stream); }

/* Pinhole ray through pixel (px, py) of camera cam: its centre, or a jittered point inside it. */
void orc_ray(const orc_scene *s, int64_t ray, double o[3], double d[3]) {
    int64_t per_cam = (int64_t)s->width * s->height;
    int64_t cam = ray / per_cam;
    int64_t pix = ray % per_cam;
    int64_t py = pix / s->width, px = pix % s->width;
    const double *R = s->cam_rot + 9 * cam;
    const double *K = s->cam_intr + 4 * cam;
    double ox = 0.5, oy = 0.5;
    if (s->jitter_seed) {
        uint32_t key = jitter_key(s->jitter_seed, ray);
        ox = jitter_u(key, 0);
        oy = jitter_u(key, 1);
    }
    double dc[3] = {((double)px + ox - K[2]) / K[0], ((double)py + oy - K[3]) / K[1], 1.0};
    double n = 0.0;
    for (int i = 0; i < 3; ++i) {
        o[i] = s->cam_origin[3 * cam + i];
        d[i] = R[3 * i + 0] * dc[0] + R[3 * i + 1] * dc[1] + R[3 * i + 2] * dc[2];
        n += d[i] * d[i];
    }
    n = sqrt(n);
    for (int i = 0; i < 3; ++i) d[i] /= n;
}

/* Ray / axis-aligned box: entry and exit parameters, entry clipped at 0. */
static int orc_slab(const orc_scene *s, const double o[3], const double d[3], double *tn, double *tf) {
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < s->bmin[a] || o[a] > s->bmax[a]) return 0;
            continue;
        }
        double ta = (s->bmin[a] - o[a]) / d[a];
        double tb = (s->bmax[a] - o[a]) / d[a];
        double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
        if (lo > t0) t0 = lo;
        if (hi < t1) t1 = hi;
    }
    if (t0 < 0.0) t0 = 0.0;
    *tn = t0;
    *tf = t1;
    return t1 > t0;
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Trilinear corners of world point p: cell-centred, clamp-to-edge.  Writes 8
 * voxel indices and weights (duplicates possible at the border). */
static void orc_trilinear(const orc_scene *s, const double p[3], int64_t idx[8], double w[8]) {
    int64_t n[3] = {s->nx, s->ny, s->nz};
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double h = (s->bmax[a] - s->bmin[a]) / (double)n[a];
        double g = (p[a] - s->bmin[a]) / h - 0.5;
        double fl = floor(g);
        i0[a] = (int64_t)fl;
        f[a] = g - fl;
    }
    for (int c = 0; c < 8; ++c) {
        int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        int64_t ix = clampi(i0[0] + bx, 0, n[0] - 1);
        int64_t iy = clampi(i0[1] + by, 0, n[1] - 1);
        int64_t iz = clampi(i0[2] + bz, 0, n[2] - 1);
        idx[c] = (iz * n[1] + iy) * n[0] + ix;
        w[c] = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
    }
}

/* Equirectangular bilinear lookup on layer l at unit direction om: 4 texel
 * units (global unit index) and weights; wrap in u, clamp in v. */
static void orc_env_lookup(const orc_scene *s, int l, const double om[3], int64_t unit[4], double w[4]) {
    const double pi = 3.14159265358979323846;
    double zc = om[2] < -1.0 ? -1.0 : (om[2] > 1.0 ? 1.0 : om[2]);
    double u = (atan2(om[1], om[0]) / (2.0 * pi) + 0.5) * s->env_w - 0.5;
    double v = acos(zc) / pi * s->env_h - 0.5;
    double fu0 = floor(u), fv0 = floor(v);
    double fu = u - fu0, fv = v - fv0;
    int64_t i0 = (int64_t)fu0, j0 = (int64_t)fv0;
    int64_t W = s->env_w, Hh = s->env_h;
    int64_t ia = ((i0 % W) + W) % W, ib = (((i0 + 1) % W) + W) % W;
    int64_t ja = clampi(j0, 0, Hh - 1), jb = clampi(j0 + 1, 0, Hh - 1);
    int64_t base = orc_nvox(s) + (int64_t)l * W * Hh;
    unit[0] = base + ja * W + ia; w[0] = (1.0 - fu) * (1.0 - fv);
    unit[1] = base + ja * W + ib; w[1] = fu * (1.0 - fv);
    unit[2] = base + jb * W + ia; w[2] = (1.0 - fu) * fv;
    unit[3] = base + jb * W + ib; w[3] = fu * fv;
}

/* Far root of |o + t d| = R (d unit); returns 0 if there is no real root. */
static int orc_far_root(const double o[3], const double d[3], double R, double *t) {
    double b = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    double c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - R * R;
    double disc = b * b - c;
    if (disc < 0.0) return 0;
    *t = -b + sqrt(disc);
    return 1;
}

static int cmp_entry(const void *a, const void *b) {
    int64_t ua = ((const orc_entry *)a)->unit, ub = ((const orc_entry *)b)->unit;
    return (ua > ub) - (ua < ub);
}

/* Per-sample working storage for one ray. */
typedef struct {
    double delta, sigma, c[3], T, alpha;
    int64_t idx[8];
    double w[8];
} orc_sample;

typedef struct {
    int used;
    double alpha, c[3], T;
    int64_t unit[4];
    double w[4];
} orc_layer;

/*
 * Trace one ray with parameters x (P doubles).  Fills the sample list, the
 * layer list and H.  Returns the number of samples.
 */
static int64_t orc_trace_t(const orc_scene *s, const double *x, int64_t ray, orc_sample *smp,
                           orc_layer *lay, double H[3], double *T_exit, double *T_end,
                           int *hit_box, double *t_far, double thresh);

static int64_t orc_trace(const orc_scene *s, const double *x, int64_t ray, orc_sample *smp,
                         orc_layer *lay, double H[3], double *T_exit, double *T_end,
                         int *hit_box, double *t_far) {
    return orc_trace_t(s, x, ray, smp, lay, H, T_exit, T_end, hit_box, t_far, 0.0);
}

/*
 * thresh > 0 is the rendering rule of Sec. IV (rendering): if the volume's total opacity
 * 1 - T_exit is below thresh, the volume counts as fully transparent (its colour is
 * dropped and the layers are seen with transmittance 1).  T_exit is still reported.
 */
static int64_t orc_trace_t(const orc_scene *s, const double *x, int64_t ray, orc_sample *smp,
                           orc_layer *lay, double H[3], double *T_exit, double *T_end,
                           int *hit_box, double *t_far, double thresh) {
    double o[3], d[3], tn = 0.0, tf = 0.0;
    orc_ray(s, ray, o, d);
    *hit_box = orc_slab(s, o, d, &tn, &tf);
    double h = orc_hmin(s);
    int64_t K = 0;
    H[0] = H[1] = H[2] = 0.0;
    double T = 1.0;
    uint32_t jkey = s->jitter_seed ? jitter_key(s->jitter_seed, ray) : 0u;
    if (*hit_box) {
        double L = (tf - tn) / h;              /* chord in voxel lengths */
        K = (int64_t)ceil(L / s->step);
        for (int64_t k = 0; k < K; ++k) {
            orc_sample *q = &smp[k];
            double dk = L - (double)k * s->step;
            q->delta = dk < s->step ? dk : s->step;     /* shortened last step */
            /* the step's midpoint, or with jittering a uniform point of the step itself
             * (half a step either side of the midpoint for full steps) */
            double u = s->jitter_seed ? jitter_u(jkey, (uint32_t)(2 + k)) : 0.5;
            double t = tn + h * ((double)k * s->step + u * q->delta);
            double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            orc_trilinear(s, p, q->idx, q->w);
            q->sigma = 0.0;
            q->c[0] = q->c[1] = q->c[2] = 0.0;
            for (int j = 0; j < 8; ++j) {
                const double *v = x + 4 * q->idx[j];
                q->c[0] += q->w[j] * v[0];
                q->c[1] += q->w[j] * v[1];
                q->c[2] += q->w[j] * v[2];
                q->sigma += q->w[j] * v[3];
            }
            /* Eq. 3-4: T is the exclusive product, alpha = 1 - exp(-sigma delta) */
            q->T = T;
            q->alpha = 1.0 - exp(-q->sigma * q->delta);
            for (int ch = 0; ch < 3; ++ch) H[ch] += q->T * q->alpha * q->c[ch];
            T = T * exp(-q->sigma * q->delta);
        }
    }
    *T_exit = T;
    *t_far = *hit_box ? tf : 0.0;
    if (thresh > 0.0 && 1.0 - T < thresh) {
        H[0] = H[1] = H[2] = 0.0;
        T = 1.0;
    }
    /* environment layers, outward from where the ray leaves the grid */
    double tmin = *hit_box ? tf : 0.0;
    for (int l = 0; l < s->n_layers; ++l) {
        orc_layer *e = &lay[l];
        double t;
        e->used = orc_far_root(o, d, s->radius[l], &t) && t > tmin;
        if (!e->used) continue;
        double om[3] = {(o[0] + t * d[0]) / s->radius[l], (o[1] + t * d[1]) / s->radius[l],
                        (o[2] + t * d[2]) / s->radius[l]};
        orc_env_lookup(s, l, om, e->unit, e->w);
        e->alpha = 0.0;
        e->c[0] = e->c[1] = e->c[2] = 0.0;
        for (int j = 0; j < 4; ++j) {
            const double *v = x + 4 * e->unit[j];
            e->c[0] += e->w[j] * v[0];
            e->c[1] += e->w[j] * v[1];
            e->c[2] += e->w[j] * v[2];
            e->alpha += e->w[j] * v[3];
        }
        e->T = T;
        for (int ch = 0; ch < 3; ++ch) H[ch] += T * e->alpha * e->c[ch];
        T = T * (1.0 - e->alpha);
    }
    for (int ch = 0; ch < 3; ++ch) H[ch] += T * s->bg[ch];
    *T_end = T;
    return K;
}

/*
 * Per-sample partial derivatives of H, from the definition (Sec. III-E):
 *   dH/dc_k       = T_k alpha_k                         (same for each channel)
 *   dH/dsigma_k   = delta_k (T_{k+1} c_k - G_k)
 *   G_k           = sum_{m>k} T_m alpha_m c_m + (environment + background seen at exit)
 * and for an environment layer l with transmittance T_l in front of it:
 *   dH/dc_l       = T_l alpha_l
 *   dH/dalpha_l   = T_l (c_l - S_{l+1}),   S = radiance behind layer l, unattenuated.
 * The suffix sums are formed explicitly.  `mode` 1 instead runs Alg. 1 (back to
 * front with two accumulators: V the optical depth, G the colour behind);
 * `mode` 2 is Alg. 1 with G started at zero, as printed (it misses the
 * environment term and exists only so a test can show that).
 */
static void orc_partials(const orc_scene *s, const orc_sample *smp, int64_t K, const orc_layer *lay,
                         double T_exit, int mode, double *dHdc, double *dHds /*[K][3]*/,
                         double *dLc, double *dLa /*[L][3]*/) {
    /* environment: S from the back */
    double S[3] = {s->bg[0], s->bg[1], s->bg[2]};
    for (int l = s->n_layers - 1; l >= 0; --l) {
        const orc_layer *e = &lay[l];
        if (!e->used) { dLc[l] = 0.0; dLa[3 * l] = dLa[3 * l + 1] = dLa[3 * l + 2] = 0.0; continue; }
        dLc[l] = e->T * e->alpha;
        for (int ch = 0; ch < 3; ++ch) dLa[3 * l + ch] = e->T * (e->c[ch] - S[ch]);
        for (int ch = 0; ch < 3; ++ch) S[ch] = e->alpha * e->c[ch] + (1.0 - e->alpha) * S[ch];
    }
    /* S is now the environment radiance seen from the grid exit */
    double E[3] = {T_exit * S[0], T_exit * S[1], T_exit * S[2]};
    if (mode == 0) {
        double G[3] = {E[0], E[1], E[2]};
        for (int64_t k = K - 1; k >= 0; --k) {
            const orc_sample *q = &smp[k];
            double Tn = q->T * exp(-q->sigma * q->delta); /* T_{k+1} */
            dHdc[k] = q->T * q->alpha;
            for (int ch = 0; ch < 3; ++ch) dHds[3 * k + ch] = q->delta * (Tn * q->c[ch] - G[ch]);
            for (int ch = 0; ch < 3; ++ch) G[ch] += q->T * q->alpha * q->c[ch];
        }
    } else {
        /* Alg. 1: V is the optical depth (the reading that makes e^{-V} the
         * transmittance after the decrement) */
        double V = 0.0;
        for (int64_t k = 0; k < K; ++k) V += smp[k].sigma * smp[k].delta;
        double G[3] = {0.0, 0.0, 0.0};
        if (mode == 1) { G[0] = E[0]; G[1] = E[1]; G[2] = E[2]; }
        for (int64_t i = K - 1; i >= 0; --i) {
            const orc_sample *q = &smp[i];
            V = V - q->sigma * q->delta;
            double eV = exp(-V), es = exp(-q->sigma * q->delta);
            dHdc[i] = eV * (1.0 - es);
            for (int ch = 0; ch < 3; ++ch) dHds[3 * i + ch] = eV * q->delta * es * q->c[ch] - q->delta * G[ch];
            for (int ch = 0; ch < 3; ++ch) G[ch] += eV * (1.0 - es) * q->c[ch];
        }
    }
}

/* Thread-local scratch for one ray. */
typedef struct {
    orc_sample *smp;
    orc_layer lay[ORC_MAX_LAYERS];
    double *dHdc, *dHds;
    orc_entry *ent;
} orc_scratch;

static void scratch_init(const orc_scene *s, orc_scratch *w) {
    int64_t K = orc_max_samples(s);
    w->smp = (orc_sample *)malloc(sizeof(orc_sample) * (size_t)K);
    w->dHdc = (double *)malloc(sizeof(double) * (size_t)K);
    w->dHds = (double *)malloc(sizeof(double) * 3 * (size_t)K);
    w->ent = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)orc_entry_capacity(s));
}
static void scratch_free(orc_scratch *w) {
    free(w->smp); free(w->dHdc); free(w->dHds); free(w->ent);
}

/*
 * The gradient row of one ray: every (unit, dH/dc, dH/dsigma) contribution of
 * every sample corner and texel, chained through the interpolation weights,
 * then sorted by unit and merged so each unit appears once.
 */
static void orc_row(const orc_scene *s, const double *x, int64_t ray, orc_scratch *w, int mode,
                    orc_ray_out *out) {
    double Hc[3], T_exit, T_end, tfar;
    int hit;
    int64_t K = orc_trace(s, x, ray, w->smp, w->lay, Hc, &T_exit, &T_end, &hit, &tfar);
    double dLc[ORC_MAX_LAYERS], dLa[3 * ORC_MAX_LAYERS];
    orc_partials(s, w->smp, K, w->lay, T_exit, mode, w->dHdc, w->dHds, dLc, dLa);
    /* Sec. III-I (Eq. 10): r_4 = lambda (1 - 4 (T - 1/2)^2) = 4 lambda T (1 - T) with T the
     * transmittance through the volume, T = exp(-sum_k sigma_k delta_k), so
     * d r_4 / d sigma_k = 4 lambda (1 - 2T) dT/dsigma_k = -4 lambda (1 - 2T) T delta_k. */
    double lam = s->aux_lambda, g4 = 0.0, r4 = 0.0;
    if (lam > 0.0) {
        r4 = 4.0 * lam * T_exit * (1.0 - T_exit);
        g4 = -4.0 * lam * (1.0 - 2.0 * T_exit) * T_exit;
    }
    int64_t n = 0;
    for (int64_t k = 0; k < K; ++k) {
        for (int j = 0; j < 8; ++j) {
            orc_entry *e = &w->ent[n++];
            double wj = w->smp[k].w[j];
            e->unit = w->smp[k].idx[j];
            e->a = wj * w->dHdc[k];
            for (int ch = 0; ch < 3; ++ch) e->s[ch] = wj * w->dHds[3 * k + ch];
            e->q = wj * g4 * w->smp[k].delta;
        }
    }
    int nl = 0;
    for (int l = 0; l < s->n_layers; ++l) {
        if (!w->lay[l].used) continue;
        ++nl;
        for (int j = 0; j < 4; ++j) {
            orc_entry *e = &w->ent[n++];
            double wj = w->lay[l].w[j];
            e->unit = w->lay[l].unit[j];
            e->a = wj * dLc[l];
            for (int ch = 0; ch < 3; ++ch) e->s[ch] = wj * dLa[3 * l + ch];
            e->q = 0.0;
        }
    }
    qsort(w->ent, (size_t)n, sizeof(orc_entry), cmp_entry);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (m > 0 && w->ent[m - 1].unit == w->ent[i].unit) {
            w->ent[m - 1].a += w->ent[i].a;
            for (int ch = 0; ch < 3; ++ch) w->ent[m - 1].s[ch] += w->ent[i].s[ch];
            w->ent[m - 1].q += w->ent[i].q;
        } else {
            w->ent[m++] = w->ent[i];
        }
    }
    int64_t nv = 0;
    for (int64_t i = 0; i < m; ++i) nv += w->ent[i].unit < orc_nvox(s);
    for (int ch = 0; ch < 3; ++ch) out->H[ch] = Hc[ch];
    out->T_exit = T_exit;
    out->T_end = T_end;
    out->aux = r4;
    out->hit_box = hit;
    out->n_layers_hit = nl;
    out->n_samples = K;
    out->n_entries = m;
    out->n_vox_units = nv;
    out->entries = w->ent;
}

/* ---------------------------------------------------------------- exported API */

int64_t orc_n_units(const orc_scene *s) { return orc_units(s); }
int64_t orc_n_rays(const orc_scene *s) { return (int64_t)s->n_cams * s->width * s->height; }

static int64_t ray_at(const int64_t *rays, int64_t i) { return rays ? rays[i] : i; }

static int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
static int orc_tid(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* Eq. 3 for the listed rays (all rays if rays == NULL): H [n][3], residual
 * r = H - C [n][3] when targets is given (targets indexed by ray id), and the
 * objective F = 0.5 sum r^2 (Eq. 5-6), summed in ray order.  With the auxiliary
 * residual on (Sec. III-I), aux_out [n] gets r_4 and F includes 0.5 r_4^2. */
int orc_render(const orc_scene *s, const double *x, const float *targets, const int64_t *rays,
               int64_t n, double *H_out, double *r_out, double *F_out, double *T_exit_out, double *aux_out) {
    double *rr = (double *)calloc((size_t)n, sizeof(double));
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t ray = ray_at(rays, i);
            double H[3], Te, Tn, tf; int hit;
            orc_trace(s, x, ray, w.smp, w.lay, H, &Te, &Tn, &hit, &tf);
            for (int ch = 0; ch < 3; ++ch) {
                if (H_out) H_out[3 * i + ch] = H[ch];
                if (targets) {
                    double r = H[ch] - (double)targets[3 * ray + ch];
                    if (r_out) r_out[3 * i + ch] = r;
                    rr[i] += r * r;
                }
            }
            if (T_exit_out) T_exit_out[i] = Te;
            double r4 = s->aux_lambda > 0.0 ? 4.0 * s->aux_lambda * Te * (1.0 - Te) : 0.0;
            if (aux_out) aux_out[i] = r4;
            if (targets) rr[i] += r4 * r4;
        }
        scratch_free(&w);
    }
    double F = 0.0;
    for (int64_t i = 0; i < n; ++i) F += rr[i];
    if (F_out) *F_out = 0.5 * F;
    free(rr);
    return 0;
}

/* Rendering of Sec. IV: H [n][3] with the opacity threshold rule (thresh > 0), T_exit [n]
 * (the volume's transmittance the rule was decided on), and, with targets, the mean squared
 * colour error over the listed rays (for PSNR). */
int orc_render_image(const orc_scene *s, const double *x, double thresh, const float *targets,
                     const int64_t *rays, int64_t n, double *H_out, double *T_exit_out, double *mse_out) {
    double *se = (double *)calloc((size_t)n, sizeof(double));
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t ray = ray_at(rays, i);
            double H[3], Te, Tn, tf; int hit;
            orc_trace_t(s, x, ray, w.smp, w.lay, H, &Te, &Tn, &hit, &tf, thresh);
            for (int ch = 0; ch < 3; ++ch) {
                if (H_out) H_out[3 * i + ch] = H[ch];
                if (targets) {
                    double r = H[ch] - (double)targets[3 * ray + ch];
                    se[i] += r * r;
                }
            }
            if (T_exit_out) T_exit_out[i] = Te;
        }
        scratch_free(&w);
    }
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += se[i];
    if (mse_out) *mse_out = n > 0 ? acc / (3.0 * (double)n) : 0.0;
    free(se);
    return 0;
}

/* u = J v for the listed rays, u [n][nr] with nr = 4 when the auxiliary residual is
 * on (fourth column d r_4) and 3 otherwise. */
int orc_apply_J(const orc_scene *s, const double *x, const double *v, const int64_t *rays, int64_t n,
                double *u) {
    const int nr = s->aux_lambda > 0.0 ? 4 : 3;
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            orc_ray_out ro;
            orc_row(s, x, ray_at(rays, i), &w, 0, &ro);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t e = 0; e < ro.n_entries; ++e) {
                const orc_entry *q = &ro.entries[e];
                const double *vv = v + 4 * q->unit;
                for (int ch = 0; ch < 3; ++ch) acc[ch] += q->a * vv[ch] + q->s[ch] * vv[3];
                acc[3] += q->q * vv[3];
            }
            for (int ch = 0; ch < nr; ++ch) u[nr * i + ch] = acc[ch];
        }
        scratch_free(&w);
    }
    return 0;
}

/* Sum over rays of per-thread FP64 buffers, reduced in thread order. */
static void reduce_buffers(double **buf, int nt, int64_t len, double *out) {
    for (int64_t j = 0; j < len; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) acc += buf[t][j];
        out[j] = acc;
    }
}

/*
 * y = J^T u (mode 0) or y = J^T J v (mode 1, u ignored) over the listed rays,
 * y has P = 4 * units entries and is overwritten.
 */
static int orc_adjoint(const orc_scene *s, const double *x, const double *u, const double *v, int jtj,
                       const int64_t *rays, int64_t n, double *y) {
    int64_t P = 4 * orc_units(s);
    const int nr = s->aux_lambda > 0.0 ? 4 : 3;
    int nt = orc_threads();
    double **buf = (double **)malloc(sizeof(double *) * (size_t)nt);
    for (int t = 0; t < nt; ++t) buf[t] = (double *)calloc((size_t)P, sizeof(double));
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        double *yb = buf[orc_tid()];
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            orc_ray_out ro;
            orc_row(s, x, ray_at(rays, i), &w, 0, &ro);
            double uu[4] = {0.0, 0.0, 0.0, 0.0};
            if (jtj) {
                for (int64_t e = 0; e < ro.n_entries; ++e) {
                    const orc_entry *q = &ro.entries[e];
                    const double *vv = v + 4 * q->unit;
                    for (int ch = 0; ch < 3; ++ch) uu[ch] += q->a * vv[ch] + q->s[ch] * vv[3];
                    uu[3] += q->q * vv[3];
                }
            } else {
                for (int ch = 0; ch < nr; ++ch) uu[ch] = u[nr * i + ch];
            }
            for (int64_t e = 0; e < ro.n_entries; ++e) {
                const orc_entry *q = &ro.entries[e];
                double *yy = yb + 4 * q->unit;
                for (int ch = 0; ch < 3; ++ch) yy[ch] += q->a * uu[ch];
                yy[3] += q->s[0] * uu[0] + q->s[1] * uu[1] + q->s[2] * uu[2] + q->q * uu[3];
            }
        }
        scratch_free(&w);
    }
    reduce_buffers(buf, nt, P, y);
    for (int t = 0; t < nt; ++t) free(buf[t]);
    free(buf);
    return 0;
}

int orc_apply_Jt(const orc_scene *s, const double *x, const double *u, const int64_t *rays, int64_t n,
                 double *y) {
    return orc_adjoint(s, x, u, NULL, 0, rays, n, y);
}

/* Eq. 9: A p = sum_i grad r_i (grad r_i^T p). */
int orc_apply_JtJ(const orc_scene *s, const double *x, const double *v, const int64_t *rays, int64_t n,
                  double *y) {
    return orc_adjoint(s, x, NULL, v, 1, rays, n, y);
}

/*
 * Gradient and diagonal blocks of J^T J in one traversal (Sec. III-G).
 * grad [P] = -J^T r (the right-hand side b of Eq. 8); blocks [units][5] =
 * (d, e_r, e_g, e_b, f) with, per ray and unit, the partials aggregated over
 * all of the ray's samples before squaring:
 *   d += a^2, e_ch += a s_ch, f += sum_ch s_ch^2,
 * so the unit's 4x4 block is [[d I, e], [e^T, f]] and diag(J^T J) = (d, d, d, f).
 * F_out = 0.5 sum r^2.
 */
int orc_grad_blocks(const orc_scene *s, const double *x, const float *targets, const int64_t *rays,
                    int64_t n, double *grad, double *blocks, double *F_out) {
    int64_t U = orc_units(s), P = 4 * U;
    int nt = orc_threads();
    double **buf = (double **)malloc(sizeof(double *) * (size_t)nt);
    for (int t = 0; t < nt; ++t) buf[t] = (double *)calloc((size_t)(P + 5 * U), sizeof(double));
    double *rr = (double *)calloc((size_t)n, sizeof(double));
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        double *gb = buf[orc_tid()];
        double *bb = gb + P;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t ray = ray_at(rays, i);
            orc_ray_out ro;
            orc_row(s, x, ray, &w, 0, &ro);
            double r[3];
            for (int ch = 0; ch < 3; ++ch) {
                r[ch] = ro.H[ch] - (double)targets[3 * ray + ch];
                rr[i] += r[ch] * r[ch];
            }
            rr[i] += ro.aux * ro.aux;
            for (int64_t e = 0; e < ro.n_entries; ++e) {
                const orc_entry *q = &ro.entries[e];
                double *g = gb + 4 * q->unit;
                for (int ch = 0; ch < 3; ++ch) g[ch] -= q->a * r[ch];
                g[3] -= q->s[0] * r[0] + q->s[1] * r[1] + q->s[2] * r[2] + q->q * ro.aux;
                double *b = bb + 5 * q->unit;
                b[0] += q->a * q->a;
                for (int ch = 0; ch < 3; ++ch) b[1 + ch] += q->a * q->s[ch];
                b[4] += q->s[0] * q->s[0] + q->s[1] * q->s[1] + q->s[2] * q->s[2] + q->q * q->q;
            }
        }
        scratch_free(&w);
    }
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(P + 5 * U));
    reduce_buffers(buf, nt, P + 5 * U, tmp);
    memcpy(grad, tmp, sizeof(double) * (size_t)P);
    memcpy(blocks, tmp + P, sizeof(double) * (size_t)(5 * U));
    free(tmp);
    double F = 0.0;
    for (int64_t i = 0; i < n; ++i) F += rr[i];
    if (F_out) *F_out = 0.5 * F;
    for (int t = 0; t < nt; ++t) free(buf[t]);
    free(buf);
    free(rr);
    return 0;
}

/*
 * Footprint of each listed ray: the number of distinct voxel units its samples
 * touch (U), the number of environment layers it hits, and its sample count.
 */
int orc_footprint(const orc_scene *s, const int64_t *rays, int64_t n, int64_t *U_out, int32_t *layers_out,
                  int64_t *K_out) {
    int64_t P = 4 * orc_units(s);
    double *zero = (double *)calloc((size_t)P, sizeof(double));
    #pragma omp parallel
    {
        orc_scratch w; scratch_init(s, &w);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            orc_ray_out ro;
            orc_row(s, zero, ray_at(rays, i), &w, 0, &ro);
            if (U_out) U_out[i] = ro.n_vox_units;
            if (layers_out) layers_out[i] = ro.n_layers_hit;
            if (K_out) K_out[i] = ro.n_samples;
        }
        scratch_free(&w);
    }
    free(zero);
    return 0;
}

/* One ray's merged gradient row: up to cap entries (unit, a, s_r, s_g, s_b).
 * Returns the entry count (or -needed if cap is too small).  H_out gets H. */
int64_t orc_ray_row(const orc_scene *s, const double *x, int64_t ray, int mode, int64_t cap,
                    int64_t *unit, double *a, double *sv, double *H_out) {
    orc_scratch w; scratch_init(s, &w);
    orc_ray_out ro;
    orc_row(s, x, ray, &w, mode, &ro);
    int64_t m = ro.n_entries;
    if (m > cap) { scratch_free(&w); return -m; }
    for (int64_t i = 0; i < m; ++i) {
        unit[i] = ro.entries[i].unit;
        a[i] = ro.entries[i].a;
        for (int ch = 0; ch < 3; ++ch) sv[3 * i + ch] = ro.entries[i].s[ch];
    }
    if (H_out) for (int ch = 0; ch < 3; ++ch) H_out[ch] = ro.H[ch];
    scratch_free(&w);
    return m;
}

/* Per-sample view of one ray for tests: delta_k, sigma_k, T_k, alpha_k, c_k and
 * the per-sample partials (mode as in orc_partials).  Returns K. */
int64_t orc_ray_samples(const orc_scene *s, const double *x, int64_t ray, int mode, int64_t cap,
                        double *delta, double *sigma, double *T, double *alpha, double *c,
                        double *dHdc, double *dHds, double *H_out, double *Tend_out) {
    orc_scratch w; scratch_init(s, &w);
    double H[3], Te, Tn, tf; int hit;
    int64_t K = orc_trace(s, x, ray, w.smp, w.lay, H, &Te, &Tn, &hit, &tf);
    if (K > cap) { scratch_free(&w); return -K; }
    double dLc[ORC_MAX_LAYERS], dLa[3 * ORC_MAX_LAYERS];
    orc_partials(s, w.smp, K, w.lay, Te, mode, w.dHdc, w.dHds, dLc, dLa);
    for (int64_t k = 0; k < K; ++k) {
        delta[k] = w.smp[k].delta; sigma[k] = w.smp[k].sigma; T[k] = w.smp[k].T; alpha[k] = w.smp[k].alpha;
        for (int ch = 0; ch < 3; ++ch) { c[3 * k + ch] = w.smp[k].c[ch]; dHds[3 * k + ch] = w.dHds[3 * k + ch]; }
        dHdc[k] = w.dHdc[k];
    }
    for (int ch = 0; ch < 3; ++ch) H_out[ch] = H[ch];
    *Tend_out = Tn;
    scratch_free(&w);
    return K;
}

/* Trilinear sample of voxel channel ch at world point p (tests of the sampler). */
double orc_sample_field(const orc_scene *s, const double *x, const double p[3], int ch) {
    int64_t idx[8]; double w[8];
    orc_trilinear(s, p, idx, w);
    double v = 0.0;
    for (int j = 0; j < 8; ++j) v += w[j] * x[4 * idx[j] + ch];
    return v;
}

int orc_num_threads(void) { return orc_threads(); }

