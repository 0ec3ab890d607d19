/*
 * Plain CPU oracle for grid-based NeRF rendering and sparse radiance warping.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU path.
 *
 * What it computes, and where the paper states it (arXiv 2404.11852):
 *   - Indexing (Sec. II-B, "Indexing"): one ray per pixel, samples along the
 *     ray, the voxel that holds each sample.
 *   - Feature Gathering (Sec. II-B): the eight vertex values of that voxel,
 *     trilinearly interpolated.
 *   - Feature Computation (Sec. II-B): a small MLP per sample; the final pixel
 *     value is accumulated over the samples of the ray (Fig. 1 caption, which
 *     defers to the standard volume-rendering quadrature of NeRF).
 *   - Sparse radiance warping (Sec. III-B, Eq. 1-4): point-cloud conversion of
 *     the reference frame by its depth, rigid transform into the target
 *     camera, perspective re-projection, and NeRF rendering of the pixels no
 *     reference pixel lands on; pixels whose depth is infinite are not
 *     re-rendered (Sec. III-B, last paragraph).
 *   - The adjoint of the rendering quadrature (not in the paper, which is
 *     inference only; it is the derivative of the same formulas).
 *
 * Precision.  Interpolation, density activation, MLP, compositing and all
 * gradients are float64.  Ray generation, the ray/box interval, sample
 * positions, the voxel index of each sample, the occupancy decision and the
 * warp's projection are float32 with an explicit expression order (the file
 * is compiled with -ffp-contract=off), because each of them decides an
 * integer (hit or miss, which voxel, skip or not, which pixel) and the GPU
 * path takes those decisions in float32.  The float32 fraction inside the
 * voxel is promoted to float64 before the trilinear weights are formed.
 *
 * Readings taken where the paper leaves a point open:
 * softplus density with an additive shift applied after interpolation,
 * per-ray step delta = (t_far - t_near)/N at interval midpoints,
 * align-corners vertex placement, early termination when transmittance
 * falls below a threshold, expected depth, and the z-buffer rule (smallest
 * depth, then smallest source index; points at infinity splat by rotation
 * only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Multi-level feature encoding (the hierarchical encodings of Sec. IV-A's
 * last paragraph, in the form of a multiresolution hash grid): level l has
 * res[l] cells per axis over the box; its vertex (x, y, z) is entry
 * (x (N+1) + y)(N+1) + z of the level's table when (N+1)^3 fits the table,
 * else the spatial hash (x * 1 ^ y * 2654435761 ^ z * 805459861) mod T in
 * 32-bit unsigned arithmetic (T a power of two).  The feature vector is the
 * levels' trilinearly interpolated entries, level-major. */
typedef struct {
    int32_t levels;          /* L */
    int32_t feat_per_level;  /* F; L * F = n_feat */
    int32_t res[8];          /* cells per axis of each level */
    int32_t log2_size;       /* T = 2^log2_size entries per level */
    const float *tables;     /* [L][T][F] */
} orc_hash;

typedef struct {
    int32_t res[3];          /* vertices per axis */
    int32_t n_feat;          /* feature channels per vertex */
    float box_lo[3];
    float box_hi[3];
    float density_shift;     /* added to the interpolated raw density before softplus */
    const float *density;    /* raw density [r0][r1][r2], z fastest */
    const float *features;   /* [r0][r1][r2][n_feat], channel fastest (unused with hash) */
    const uint8_t *occ;      /* [(r0-1)(r1-1)(r2-1)] cell flags, or NULL */
    const orc_hash *hash;    /* NULL: features from the dense grid */
} orc_grid;

typedef struct {
    int32_t in_dim;          /* n_feat + 3 + 6*pe_freqs */
    int32_t hidden;
    int32_t out_dim;         /* 3 */
    int32_t pe_freqs;
    const float *w0, *b0;    /* [hidden][in_dim], [hidden] */
    const float *w1, *b1;    /* [hidden][hidden], [hidden] */
    const float *w2, *b2;    /* [out_dim][hidden], [out_dim] */
    int32_t round_bf16;      /* 1: each layer's inputs and weights rounded to
                                bfloat16 (round to nearest even) before the
                                float64 products (the precision path) */
} orc_mlp;

typedef struct {
    int32_t n_samples;
    float et_threshold;      /* stop when transmittance < this; 0 = never */
    int32_t use_occupancy;
    float bg[3];
    float void_acc;          /* frame depth is +inf when acc < this */
    float warp_max_angle;    /* degrees; 0 = no angle test in the warp */
} orc_opts;

typedef struct {
    int32_t width, height;
    float f, cx, cy;
    float c2w[12];           /* row-major 3x4 [R | eye], OpenCV camera axes */
} orc_camera;

/* ------------------------------------------------------------------ */
/* float32 geometry (decides integers; same precision as the GPU path) */
/* ------------------------------------------------------------------ */

/* Pixel (i, j) -> world ray.  Pixel centres at (i+1/2, j+1/2); camera-space
 * direction (a, b, 1) rotated to world and normalised (Sec. II-B Indexing,
 * "a ray for each pixel"; Eq. 1 uses the same pinhole intrinsics). */
static void pixel_ray_f32(const orc_camera *c, int i, int j, float o[3], float d[3])
{
    float a = (((float)i + 0.5f) - c->cx) / c->f;
    float b = (((float)j + 0.5f) - c->cy) / c->f;
    float dx = (c->c2w[0] * a + c->c2w[1] * b) + c->c2w[2];
    float dy = (c->c2w[4] * a + c->c2w[5] * b) + c->c2w[6];
    float dz = (c->c2w[8] * a + c->c2w[9] * b) + c->c2w[10];
    float n = sqrtf((dx * dx + dy * dy) + dz * dz);
    d[0] = dx / n;
    d[1] = dy / n;
    d[2] = dz / n;
    o[0] = c->c2w[3];
    o[1] = c->c2w[7];
    o[2] = c->c2w[11];
}

/* Slab test against the axis-aligned box; returns 1 on a hit with
 * 0 <= t_near < t_far. */
static int ray_box_f32(const float o[3], const float d[3], const float lo[3],
                       const float hi[3], float *tn_out, float *tf_out)
{
    float tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        float inv = 1.0f / d[a];
        float t0 = (lo[a] - o[a]) * inv;
        float t1 = (hi[a] - o[a]) * inv;
        tn = fmaxf(tn, fminf(t0, t1));
        tf = fminf(tf, fmaxf(t0, t1));
    }
    tn = fmaxf(tn, 0.0f);
    *tn_out = tn;
    *tf_out = tf;
    return tn < tf;
}

/* Sample position -> lower vertex index of its voxel and the fraction
 * inside the voxel, per axis (align-corners grid on the box). */
static void locate_f32(const orc_grid *g, const float x[3], int i0[3], float fr[3])
{
    for (int a = 0; a < 3; ++a) {
        float scale = (float)(g->res[a] - 1) / (g->box_hi[a] - g->box_lo[a]);
        float u = (x[a] - g->box_lo[a]) * scale;
        int i = (int)floorf(u);
        if (i < 0) i = 0;
        if (i > g->res[a] - 2) i = g->res[a] - 2;
        float f = u - (float)i;
        f = fminf(fmaxf(f, 0.0f), 1.0f);
        i0[a] = i;
        fr[a] = f;
    }
}

static int64_t cell_index(const orc_grid *g, const int i0[3])
{
    return ((int64_t)i0[0] * (g->res[1] - 1) + i0[1]) * (int64_t)(g->res[2] - 1) + i0[2];
}

static int64_t vertex_index(const orc_grid *g, int x, int y, int z)
{
    return ((int64_t)x * g->res[1] + y) * (int64_t)g->res[2] + z;
}

/* ------------------------------------------------------------------ */
/* float64 arithmetic                                                  */
/* ------------------------------------------------------------------ */

/* Trilinear weights of the eight voxel vertices, ordered (dx,dy,dz) with
 * dz fastest, from the per-axis fraction. */
static void trilinear_weights(const float fr[3], double w[8])
{
    double fx = fr[0], fy = fr[1], fz = fr[2];
    for (int v = 0; v < 8; ++v) {
        int dx = (v >> 2) & 1, dy = (v >> 1) & 1, dz = v & 1;
        w[v] = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
    }
}

static void corner_indices(const orc_grid *g, const int i0[3], int64_t idx[8])
{
    for (int v = 0; v < 8; ++v) {
        int dx = (v >> 2) & 1, dy = (v >> 1) & 1, dz = v & 1;
        idx[v] = vertex_index(g, i0[0] + dx, i0[1] + dy, i0[2] + dz);
    }
}

/* One level of the multi-level encoding at position x (float32 locate,
 * float64 interpolation); adds nothing else. */
static void hash_level(const orc_hash *h, int l, const float lo[3], const float hi[3], const float x[3],
                       double *out)
{
    const int N = h->res[l], F = h->feat_per_level;
    const uint32_t T = 1u << h->log2_size;
    const int dense = (int64_t)(N + 1) * (N + 1) * (N + 1) <= (int64_t)T;
    int i0[3];
    float fr[3];
    for (int a = 0; a < 3; ++a) {
        float scale = (float)N / (hi[a] - lo[a]);
        float u = (x[a] - lo[a]) * scale;
        int i = (int)floorf(u);
        if (i < 0) i = 0;
        if (i > N - 1) i = N - 1;
        float f = u - (float)i;
        fr[a] = fminf(fmaxf(f, 0.0f), 1.0f);
        i0[a] = i;
    }
    double w[8];
    trilinear_weights(fr, w);
    const float *tab = h->tables + (size_t)l * T * F;
    for (int f = 0; f < F; ++f) out[f] = 0.0;
    for (int v = 0; v < 8; ++v) {
        uint32_t vx = (uint32_t)(i0[0] + ((v >> 2) & 1)), vy = (uint32_t)(i0[1] + ((v >> 1) & 1)),
                 vz = (uint32_t)(i0[2] + (v & 1));
        uint32_t e = dense ? (vx * (uint32_t)(N + 1) + vy) * (uint32_t)(N + 1) + vz
                           : ((vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u)) & (T - 1u);
        for (int f = 0; f < F; ++f) out[f] += w[v] * (double)tab[(size_t)e * F + f];
    }
}

/* Feature vector of a sample: the dense grid's trilinear interpolation, or
 * the multi-level encoding's levels in order. */
static void sample_features(const orc_grid *g, const float x[3], const double wv[8], const int64_t idx[8],
                            double *feat)
{
    if (g->hash) {
        for (int l = 0; l < g->hash->levels; ++l)
            hash_level(g->hash, l, g->box_lo, g->box_hi, x, feat + l * g->hash->feat_per_level);
        return;
    }
    const int C = g->n_feat;
    for (int ch = 0; ch < C; ++ch) {
        double s = 0.0;
        for (int v = 0; v < 8; ++v) s += wv[v] * (double)g->features[idx[v] * C + ch];
        feat[ch] = s;
    }
}

/* Encode n positions [n][3] with the grid's multi-level encoding (or dense
 * features): out [n][n_feat]. */
void orc_encode(const orc_grid *g, int64_t n, const float *pos, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        int i0[3];
        float fr[3];
        double wv[8];
        int64_t idx[8];
        locate_f32(g, pos + 3 * i, i0, fr);
        trilinear_weights(fr, wv);
        corner_indices(g, i0, idx);
        sample_features(g, pos + 3 * i, wv, idx, out + i * g->n_feat);
    }
}

static double softplus_d(double x)
{
    if (x > 30.0) return x;
    return log1p(exp(x));
}

static double sigmoid_d(double x)
{
    return 1.0 / (1.0 + exp(-x));
}

/* MLP input: interpolated features, then the view direction, then
 * sin(2^m d_c) and cos(2^m d_c) for c in (x, y, z) outer, m inner. */
static void mlp_input(const orc_mlp *m, int n_feat, const double *feat, const float d[3], double *x)
{
    int F = m->pe_freqs;
    for (int c = 0; c < n_feat; ++c) x[c] = feat[c];
    for (int c = 0; c < 3; ++c) x[n_feat + c] = d[c];
    for (int c = 0; c < 3; ++c)
        for (int k = 0; k < F; ++k) {
            double s = ldexp((double)d[c], k);
            x[n_feat + 3 + c * F + k] = sin(s);
            x[n_feat + 3 + 3 * F + c * F + k] = cos(s);
        }
}

/* Round to bfloat16 (8-bit significand), nearest-even, via float32. */
static double bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;   /* inf / nan unchanged */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double wt(const orc_mlp *m, const float *w, int64_t i)
{
    return m->round_bf16 ? bf16_round((double)w[i]) : (double)w[i];
}

static double act(const orc_mlp *m, double v)
{
    return m->round_bf16 ? bf16_round(v) : v;
}

/* Two ReLU hidden layers and a sigmoid output layer; h1, h2 keep the
 * post-activation values, c the output. */
static void mlp_forward(const orc_mlp *m, const double *x, double *h1, double *h2, double *c)
{
    int I = m->in_dim, H = m->hidden, O = m->out_dim;
    for (int o = 0; o < H; ++o) {
        double s = m->b0[o];
        for (int i = 0; i < I; ++i) s += wt(m, m->w0, (int64_t)o * I + i) * act(m, x[i]);
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < H; ++o) {
        double s = m->b1[o];
        for (int i = 0; i < H; ++i) s += wt(m, m->w1, (int64_t)o * H + i) * act(m, h1[i]);
        h2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < O; ++o) {
        double s = m->b2[o];
        for (int i = 0; i < H; ++i) s += wt(m, m->w2, (int64_t)o * H + i) * act(m, h2[i]);
        c[o] = sigmoid_d(s);
    }
}

/* Size of one bfloat16 step at v (8 significant bits): the change of a
 * rounded value when float32 and float64 arithmetic round it to adjacent
 * bfloat16 values. */
static double bf16_ulp(double v)
{
    double a = fabs(v);
    if (a == 0.0) return 0.0;
    int e;
    frexp(a, &e);              /* a = mant * 2^e, mant in [0.5, 1) */
    return ldexp(1.0, e - 8);
}

/* Largest change of the output colour (any channel) that one bfloat16
 * rounding step of one MLP input value could cause at this sample, to first
 * order: for a layer-l input v the output moves by c(1-c) |J[c][v]| ulp(v),
 * where J is the derivative of the output logit with respect to v through
 * the sample's active ReLUs and the (rounded) weights.  j1 [out][hidden] and
 * j0 [out][in] are scratch.  Only meaningful with round_bf16. */
static double bf16_flip_effect(const orc_mlp *m, const double *x, const double *h1, const double *h2,
                               const double *c, double *j1, double *j0)
{
    int I = m->in_dim, H = m->hidden, O = m->out_dim;
    for (int o = 0; o < O; ++o) {
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int k = 0; k < H; ++k)
                if (h2[k] > 0.0) s += wt(m, m->w2, (int64_t)o * H + k) * wt(m, m->w1, (int64_t)k * H + j);
            j1[o * H + j] = s;
        }
        for (int i = 0; i < I; ++i) {
            double s = 0.0;
            for (int j = 0; j < H; ++j)
                if (h1[j] > 0.0) s += j1[o * H + j] * wt(m, m->w0, (int64_t)j * I + i);
            j0[o * I + i] = s;
        }
    }
    double worst = 0.0;
    for (int o = 0; o < O && o < 3; ++o) {
        double g = 0.0, e;
        for (int k = 0; k < H; ++k)
            if ((e = fabs(wt(m, m->w2, (int64_t)o * H + k)) * bf16_ulp(act(m, h2[k]))) > g) g = e;
        for (int j = 0; j < H; ++j)
            if ((e = fabs(j1[o * H + j]) * bf16_ulp(act(m, h1[j]))) > g) g = e;
        for (int i = 0; i < I; ++i)
            if ((e = fabs(j0[o * I + i]) * bf16_ulp(act(m, x[i]))) > g) g = e;
        g *= c[o] * (1.0 - c[o]);
        if (g > worst) worst = g;
    }
    return worst;
}

/* Per-sample record kept by the forward pass for the adjoint. */
typedef struct {
    int k;
    float tk;
    int i0[3];
    float fr[3];
    double raw;      /* interpolated raw density (before shift) */
    double sigma;
    double w;        /* T_k * alpha_k */
    double T_next;   /* T_{k+1} = T_k * exp(-sigma_k * delta) */
} sample_rec;

typedef struct {
    double rgb[3];
    double depth_t;  /* sum_k w_k t_k */
    double acc;      /* 1 - T_stop */
    double T_stop;
    double delta;
    int32_t n_eval;  /* samples that went through the MLP */
    double margin;   /* min over termination decisions of |T/thr - 1| */
    uint64_t relu_sig;
    double flip;     /* max over samples of w_k times bf16_flip_effect (when asked) */
} ray_out;

/* Render one ray (Sec. II-B; compositing as the standard quadrature).
 * If recs != NULL (capacity n_samples), live samples and their MLP
 * activations are stored for the adjoint. */
static void render_ray(const orc_grid *g, const orc_mlp *m, const orc_opts *op,
                       const float o[3], const float d[3], ray_out *out,
                       sample_rec *recs, double *xs, double *h1s, double *h2s, double *cs, int want_flip)
{
    int N = op->n_samples, C = g->n_feat;
    int I = m->in_dim, H = m->hidden, O = m->out_dim;
    double feat[64], x[256], h1[1024], h2[1024], c[8];
    double j1[8 * 1024], j0[8 * 256];
    double wv[8];
    int64_t idx[8];

    memset(out, 0, sizeof(*out));
    out->T_stop = 1.0;
    out->margin = INFINITY;
    float tn, tf;
    if (!ray_box_f32(o, d, g->box_lo, g->box_hi, &tn, &tf)) {
        for (int ch = 0; ch < 3; ++ch) out->rgb[ch] = op->bg[ch];
        return;
    }
    float delta = (tf - tn) / (float)N;
    out->delta = delta;
    double T = 1.0;
    double thr = op->et_threshold;
    for (int k = 0; k < N; ++k) {
        if (thr > 0.0) {
            double mg = fabs(T / thr - 1.0);
            if (mg < out->margin) out->margin = mg;
            if (T < thr) break;
        }
        float tk = tn + ((float)k + 0.5f) * delta;
        float xp[3];
        for (int a = 0; a < 3; ++a) xp[a] = o[a] + tk * d[a];
        int i0[3];
        float fr[3];
        locate_f32(g, xp, i0, fr);
        if (op->use_occupancy && g->occ && !g->occ[cell_index(g, i0)]) continue;
        trilinear_weights(fr, wv);
        corner_indices(g, i0, idx);
        double raw = 0.0;
        for (int v = 0; v < 8; ++v) raw += wv[v] * (double)g->density[idx[v]];
        double sigma = softplus_d(raw + (double)g->density_shift);
        double att = exp(-sigma * (double)delta);
        double alpha = 1.0 - att;
        double w = T * alpha;
        sample_features(g, xp, wv, idx, feat);
        mlp_input(m, C, feat, d, x);
        mlp_forward(m, x, h1, h2, c);
        for (int u = 0; u < H; ++u) {
            if (h1[u] > 0.0) out->relu_sig += (uint64_t)(u + 1) * (uint64_t)(k + 1) * 2654435761ull;
            if (h2[u] > 0.0) out->relu_sig += (uint64_t)(u + 1 + H) * (uint64_t)(k + 1) * 40503ull;
        }
        for (int ch = 0; ch < O && ch < 3; ++ch) out->rgb[ch] += w * c[ch];
        out->depth_t += w * (double)tk;
        if (want_flip) {
            double fe = w * bf16_flip_effect(m, x, h1, h2, c, j1, j0);
            if (fe > out->flip) out->flip = fe;
        }
        if (recs) {
            int n = out->n_eval;
            sample_rec *r = &recs[n];
            r->k = k;
            r->tk = tk;
            for (int a = 0; a < 3; ++a) { r->i0[a] = i0[a]; r->fr[a] = fr[a]; }
            r->raw = raw;
            r->sigma = sigma;
            r->w = w;
            r->T_next = T * att;
            memcpy(xs + (int64_t)n * I, x, sizeof(double) * I);
            memcpy(h1s + (int64_t)n * H, h1, sizeof(double) * H);
            memcpy(h2s + (int64_t)n * H, h2, sizeof(double) * H);
            memcpy(cs + (int64_t)n * O, c, sizeof(double) * O);
        }
        out->n_eval++;
        T = T * att;
    }
    out->T_stop = T;
    for (int ch = 0; ch < 3; ++ch) out->rgb[ch] += T * (double)op->bg[ch];
    out->acc = 1.0 - T;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Rays for a list of pixels (or all pixels when pix == NULL). */
void orc_generate_rays(const orc_camera *cam, int64_t n, const int64_t *pix, float *o, float *d)
{
    int64_t total = pix ? n : (int64_t)cam->width * cam->height;
    for (int64_t r = 0; r < total; ++r) {
        int64_t p = pix ? pix[r] : r;
        int i = (int)(p % cam->width), j = (int)(p / cam->width);
        pixel_ray_f32(cam, i, j, o + 3 * r, d + 3 * r);
    }
}

/* Ray/box interval in float32: tn, tf per ray and the hit flag. */
void orc_ray_box(int64_t n, const float *o, const float *d, const float lo[3], const float hi[3],
                 float *tn, float *tf, uint8_t *hit)
{
    for (int64_t r = 0; r < n; ++r) hit[r] = (uint8_t)ray_box_f32(o + 3 * r, d + 3 * r, lo, hi, tn + r, tf + r);
}

/* Occupancy flags per voxel: a voxel is occupied when any of its eight
 * vertices has density above occ_sigma, i.e. raw + shift above
 * log(expm1(occ_sigma)); the comparison is made in float32. */
void orc_build_occupancy(const orc_grid *g, float occ_sigma, uint8_t *occ)
{
    float thr = (float)log(expm1((double)occ_sigma));
    int c0 = g->res[0] - 1, c1 = g->res[1] - 1, c2 = g->res[2] - 1;
    for (int x = 0; x < c0; ++x)
        for (int y = 0; y < c1; ++y)
            for (int z = 0; z < c2; ++z) {
                int any = 0;
                for (int v = 0; v < 8; ++v) {
                    int dx = (v >> 2) & 1, dy = (v >> 1) & 1, dz = v & 1;
                    float s = g->density[vertex_index(g, x + dx, y + dy, z + dz)] + g->density_shift;
                    if (s > thr) any = 1;
                }
                occ[((int64_t)x * c1 + y) * c2 + z] = (uint8_t)any;
            }
}

/* Trilinear interpolation of an n_ch-channel vertex field at float32 world
 * positions (used by the tests to pin the gather against closed forms). */
void orc_trilerp(const orc_grid *g, const float *values, int n_ch, int64_t n, const float *pos, double *out)
{
    double wv[8];
    int64_t idx[8];
    for (int64_t s = 0; s < n; ++s) {
        int i0[3];
        float fr[3];
        locate_f32(g, pos + 3 * s, i0, fr);
        trilinear_weights(fr, wv);
        corner_indices(g, i0, idx);
        for (int ch = 0; ch < n_ch; ++ch) {
            double acc = 0.0;
            for (int v = 0; v < 8; ++v) acc += wv[v] * (double)values[idx[v] * n_ch + ch];
            out[s * n_ch + ch] = acc;
        }
    }
}

/* Transpose of orc_trilerp: out_grid[vertex][ch] += sum over positions of
 * weight * y[s][ch]. */
void orc_trilerp_scatter(const orc_grid *g, int n_ch, int64_t n, const float *pos, const double *y, double *out_grid)
{
    double wv[8];
    int64_t idx[8];
    for (int64_t s = 0; s < n; ++s) {
        int i0[3];
        float fr[3];
        locate_f32(g, pos + 3 * s, i0, fr);
        trilinear_weights(fr, wv);
        corner_indices(g, i0, idx);
        for (int v = 0; v < 8; ++v)
            for (int ch = 0; ch < n_ch; ++ch) out_grid[idx[v] * n_ch + ch] += wv[v] * y[s * n_ch + ch];
    }
}

/* MLP on explicit inputs x [n][in_dim] -> c [n][out_dim]. */
void orc_mlp_forward(const orc_mlp *m, int64_t n, const double *x, double *c)
{
    double *h1 = (double *)malloc(sizeof(double) * m->hidden);
    double *h2 = (double *)malloc(sizeof(double) * m->hidden);
    for (int64_t s = 0; s < n; ++s) mlp_forward(m, x + s * m->in_dim, h1, h2, c + s * m->out_dim);
    free(h1);
    free(h2);
}

/* MLP input vector for given interpolated features and direction. */
void orc_mlp_input(const orc_mlp *m, int n_feat, int64_t n, const double *feat, const float *d, double *x)
{
    for (int64_t s = 0; s < n; ++s) mlp_input(m, n_feat, feat + s * n_feat, d + 3 * s, x + s * m->in_dim);
}

/* Render a batch of rays.  rgb [n][3], depth_t [n], acc [n] (float64);
 * n_eval [n], margin [n], relu_sig [n], flip [n] (the bfloat16 rounding-flip
 * diagnostic of orc_render_pixels) may be NULL. */
void orc_render_rays(const orc_grid *g, const orc_mlp *m, const orc_opts *op, int64_t n,
                     const float *o, const float *d, double *rgb, double *depth_t, double *acc,
                     int32_t *n_eval, double *margin, uint64_t *relu_sig, double *flip)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; ++r) {
        ray_out ro;
        render_ray(g, m, op, o + 3 * r, d + 3 * r, &ro, NULL, NULL, NULL, NULL, NULL, flip != NULL);
        if (flip) flip[r] = ro.flip;
        for (int ch = 0; ch < 3; ++ch) rgb[3 * r + ch] = ro.rgb[ch];
        depth_t[r] = ro.depth_t;
        acc[r] = ro.acc;
        if (n_eval) n_eval[r] = ro.n_eval;
        if (margin) margin[r] = ro.margin;
        if (relu_sig) relu_sig[r] = ro.relu_sig;
    }
}

/* Frame depth along the camera axis from expected ray distance: void
 * (+inf) when the ray's opacity is below void_acc. */
static double frame_depth(const orc_camera *cam, const float d[3], double depth_t, double acc, double void_acc)
{
    if (!(acc >= void_acc)) return INFINITY;
    double cosang = (double)d[0] * cam->c2w[2] + (double)d[1] * cam->c2w[6] + (double)d[2] * cam->c2w[10];
    return depth_t / acc * cosang;
}

/* Render pixels of a frame (all when pix == NULL): rgb [n][3], z-depth [n],
 * acc [n]; acc_margin[n] = |acc/void_acc - 1| (may be NULL). */
void orc_render_pixels(const orc_grid *g, const orc_mlp *m, const orc_opts *op, const orc_camera *cam,
                       int64_t n, const int64_t *pix, double *rgb, double *depth_z, double *acc,
                       int32_t *n_eval, double *margin, double *acc_margin, double *flip)
{
    int64_t total = pix ? n : (int64_t)cam->width * cam->height;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < total; ++r) {
        int64_t p = pix ? pix[r] : r;
        float o[3], d[3];
        pixel_ray_f32(cam, (int)(p % cam->width), (int)(p / cam->width), o, d);
        ray_out ro;
        render_ray(g, m, op, o, d, &ro, NULL, NULL, NULL, NULL, NULL, flip != NULL);
        for (int ch = 0; ch < 3; ++ch) rgb[3 * r + ch] = ro.rgb[ch];
        depth_z[r] = frame_depth(cam, d, ro.depth_t, ro.acc, op->void_acc);
        acc[r] = ro.acc;
        if (n_eval) n_eval[r] = ro.n_eval;
        if (margin) margin[r] = ro.margin;
        if (acc_margin) acc_margin[r] = fabs(ro.acc / (double)op->void_acc - 1.0);
        if (flip) flip[r] = ro.flip;
    }
}

/* ------------------------------------------------------------------ */
/* sparse radiance warping, Eq. 1-3 (float32)                          */
/* ------------------------------------------------------------------ */

static uint32_t f32_bits(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    return u;
}

static float bits_f32(uint32_t u)
{
    float v;
    memcpy(&v, &u, 4);
    return v;
}

/* Warp a reference frame into a target camera.
 *   T: row-major 3x4 [R | t] taking reference-camera coordinates to
 *      target-camera coordinates (Eq. 2).
 *   Each reference pixel with finite depth D becomes the point
 *   D * ((i+1/2-cx)/f, (j+1/2-cy)/f, 1) (Eq. 1), is moved by T (Eq. 2) and
 *   projected with the target intrinsics (Eq. 3).  A pixel with infinite
 *   depth is a direction: it is rotated only and carries depth +inf.
 *   Every target pixel keeps the splat with the smallest depth, ties broken
 *   by the smallest reference pixel index.
 * Outputs (target size): rgb [H][W][3], depth [H][W] (target z, +inf for
 * directions, 0 for holes), mask [H][W] (1 = no splat landed), src [H][W]
 * (reference pixel index or -1; may be NULL). */
/* Warping is allowed only where the angle, at the scene point, between the
 * reference camera's ray and the target camera's ray is below a threshold
 * (Sec. III-C, "Deciding When to Warp").  In target-camera coordinates the
 * target centre is the origin and the reference centre is t = (T[3], T[7],
 * T[11]); the test is cos(angle) > cos(max_angle), in float32.  Points at
 * infinity subtend no angle.  max_angle_deg <= 0 disables the test. */
static float cos_limit(float max_angle_deg)
{
    return max_angle_deg > 0.0f ? (float)cos((double)max_angle_deg * 3.14159265358979323846 / 180.0) : -2.0f;
}

static int angle_ok(const float T[12], float Xt, float Yt, float Zt, float cmin)
{
    if (cmin < -1.0f) return 1;
    float rx = Xt - T[3], ry = Yt - T[7], rz = Zt - T[11];
    float dot = (Xt * rx + Yt * ry) + Zt * rz;
    float n1 = sqrtf((Xt * Xt + Yt * Yt) + Zt * Zt);
    float n2 = sqrtf((rx * rx + ry * ry) + rz * rz);
    return dot / (n1 * n2) > cmin;
}

/* Steps 1-2 for one reference pixel: back-project along its ray to depth D
 * (Eq. 1) and move the point into target-camera coordinates (Eq. 2).  A
 * point at infinity moves by the rotation only (a direction); its z-buffer
 * depth is +inf.  Float32, expression order as written. */
static void warp_point(const orc_camera *ref, const float T[12], int i, int j, float D,
                       float *Xt, float *Yt, float *Zt, float *kz)
{
    float a = (((float)i + 0.5f) - ref->cx) / ref->f;
    float b = (((float)j + 0.5f) - ref->cy) / ref->f;
    if (D == INFINITY) {
        *Xt = (T[0] * a + T[1] * b) + T[2];
        *Yt = (T[4] * a + T[5] * b) + T[6];
        *Zt = (T[8] * a + T[9] * b) + T[10];
        *kz = INFINITY;
    } else {
        float X = D * a, Y = D * b, Z = D;
        *Xt = ((T[0] * X + T[1] * Y) + T[2] * Z) + T[3];
        *Yt = ((T[4] * X + T[5] * Y) + T[6] * Z) + T[7];
        *Zt = ((T[8] * X + T[9] * Y) + T[10] * Z) + T[11];
        *kz = *Zt;
    }
}

/* Steps 1-3 of Sec. III-B with the when-to-warp test of Sec. III-C.  The
 * z-buffer decides which reference point is visible at each target pixel
 * (nearest depth, ties to the smaller reference index); the angle test is
 * then applied to that visible point, and a pixel whose point fails it is
 * left for rendering like a disocclusion hole (a failing point does not
 * uncover what lies behind it).  max_angle_deg <= 0 disables the test. */
void orc_warp_angle(const orc_camera *ref, const orc_camera *tgt, const float T[12],
                    const float *ref_rgb, const float *ref_depth, float max_angle_deg,
                    float *tgt_rgb, float *tgt_depth, uint8_t *mask, int32_t *src_out)
{
    const float cmin = cos_limit(max_angle_deg);
    int W = ref->width, H = ref->height, Wt = tgt->width, Ht = tgt->height;
    int64_t np = (int64_t)Wt * Ht;
    uint64_t *zbuf = (uint64_t *)malloc(sizeof(uint64_t) * np);
    for (int64_t p = 0; p < np; ++p) zbuf[p] = UINT64_MAX;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t src = (int64_t)j * W + i;
            float D = ref_depth[src];
            if (D != D) continue;
            float Xt, Yt, Zt, kz;
            warp_point(ref, T, i, j, D, &Xt, &Yt, &Zt, &kz);
            if (!(Zt > 0.0f)) continue;
            float u = tgt->f * (Xt / Zt) + tgt->cx;
            float v = tgt->f * (Yt / Zt) + tgt->cy;
            if (!(u >= 0.0f && u < (float)Wt && v >= 0.0f && v < (float)Ht)) continue;
            int64_t p = (int64_t)floorf(v) * Wt + (int64_t)floorf(u);
            uint64_t key = ((uint64_t)f32_bits(kz) << 32) | (uint64_t)(uint32_t)src;
            if (key < zbuf[p]) zbuf[p] = key;
        }
    for (int64_t p = 0; p < np; ++p) {
        uint64_t key = zbuf[p];
        int hole = key == UINT64_MAX;
        if (!hole && cmin >= -1.0f) {
            uint32_t s = (uint32_t)(key & 0xffffffffu);
            float D = ref_depth[s];
            if (D != INFINITY) {
                float Xt, Yt, Zt, kz;
                warp_point(ref, T, (int)(s % (uint32_t)W), (int)(s / (uint32_t)W), D, &Xt, &Yt, &Zt, &kz);
                hole = !angle_ok(T, Xt, Yt, Zt, cmin);
            }
        }
        if (hole) {
            mask[p] = 1;
            tgt_rgb[3 * p] = tgt_rgb[3 * p + 1] = tgt_rgb[3 * p + 2] = 0.0f;
            tgt_depth[p] = 0.0f;
            if (src_out) src_out[p] = -1;
        } else {
            uint32_t s = (uint32_t)(key & 0xffffffffu);
            mask[p] = 0;
            for (int ch = 0; ch < 3; ++ch) tgt_rgb[3 * p + ch] = ref_rgb[3 * (int64_t)s + ch];
            tgt_depth[p] = bits_f32((uint32_t)(key >> 32));
            if (src_out) src_out[p] = (int32_t)s;
        }
    }
    free(zbuf);
}

void orc_warp(const orc_camera *ref, const orc_camera *tgt, const float T[12],
              const float *ref_rgb, const float *ref_depth,
              float *tgt_rgb, float *tgt_depth, uint8_t *mask, int32_t *src_out)
{
    orc_warp_angle(ref, tgt, T, ref_rgb, ref_depth, 0.0f, tgt_rgb, tgt_depth, mask, src_out);
}

/* Eq. 4: warp, then render the hole pixels with the full model and put them
 * in place.  rgb/depth outputs are float64; mask as in orc_warp.
 * n_masked receives the hole count. */
void orc_sparw(const orc_grid *g, const orc_mlp *m, const orc_opts *op,
               const orc_camera *ref, const float *ref_rgb, const float *ref_depth,
               const orc_camera *tgt, const float T[12],
               double *out_rgb, double *out_depth, uint8_t *mask, int64_t *n_masked)
{
    int64_t np = (int64_t)tgt->width * tgt->height;
    float *wr = (float *)malloc(sizeof(float) * 3 * np);
    float *wd = (float *)malloc(sizeof(float) * np);
    orc_warp_angle(ref, tgt, T, ref_rgb, ref_depth, op->warp_max_angle, wr, wd, mask, NULL);
    int64_t nh = 0;
    for (int64_t p = 0; p < np; ++p) nh += mask[p];
    int64_t *holes = (int64_t *)malloc(sizeof(int64_t) * (nh > 0 ? nh : 1));
    int64_t q = 0;
    for (int64_t p = 0; p < np; ++p)
        if (mask[p]) holes[q++] = p;
    double *hr = (double *)malloc(sizeof(double) * 3 * (nh > 0 ? nh : 1));
    double *hd = (double *)malloc(sizeof(double) * (nh > 0 ? nh : 1));
    double *ha = (double *)malloc(sizeof(double) * (nh > 0 ? nh : 1));
    if (nh > 0) orc_render_pixels(g, m, op, tgt, nh, holes, hr, hd, ha, NULL, NULL, NULL, NULL);
    for (int64_t p = 0; p < np; ++p) {
        for (int ch = 0; ch < 3; ++ch) out_rgb[3 * p + ch] = wr[3 * p + ch];
        out_depth[p] = wd[p];
    }
    for (int64_t h = 0; h < nh; ++h) {
        int64_t p = holes[h];
        for (int ch = 0; ch < 3; ++ch) out_rgb[3 * p + ch] = hr[3 * h + ch];
        out_depth[p] = hd[h];
    }
    *n_masked = nh;
    free(wr); free(wd); free(holes); free(hr); free(hd); free(ha);
}

/* ------------------------------------------------------------------ */
/* adjoint                                                             */
/* ------------------------------------------------------------------ */

/* Gradients of a loss through the rendering of a ray batch.
 * Inputs: upstream d_rgb [n][3], optional d_depth_t [n] and d_acc [n].
 * Outputs (float64, accumulated with +=): d_density [verts],
 * d_features [verts][n_feat], d_w0..d_b2 shaped like the weights.
 * rgb_out/depth_out/acc_out (may be NULL) receive the recomputed forward. */
void orc_render_backward(const orc_grid *g, const orc_mlp *m, const orc_opts *op, int64_t n,
                         const float *o, const float *d, const double *d_rgb,
                         const double *d_depth_t, const double *d_acc,
                         double *d_density, double *d_features,
                         double *d_w0, double *d_b0, double *d_w1, double *d_b1,
                         double *d_w2, double *d_b2,
                         double *rgb_out, double *depth_out, double *acc_out)
{
    if (g->hash) return;   /* the adjoint is defined for the dense feature grid only */
    int N = op->n_samples, C = g->n_feat;
    int I = m->in_dim, H = m->hidden, O = m->out_dim;
    int64_t nw0 = (int64_t)H * I, nw1 = (int64_t)H * H, nw2 = (int64_t)O * H;
#pragma omp parallel
    {
        sample_rec *recs = (sample_rec *)malloc(sizeof(sample_rec) * N);
        double *xs = (double *)malloc(sizeof(double) * (int64_t)N * I);
        double *h1s = (double *)malloc(sizeof(double) * (int64_t)N * H);
        double *h2s = (double *)malloc(sizeof(double) * (int64_t)N * H);
        double *cs = (double *)malloc(sizeof(double) * (int64_t)N * O);
        double *Rs = (double *)malloc(sizeof(double) * (int64_t)N * 3);
        double *Ds = (double *)malloc(sizeof(double) * N);
        double *gw0 = (double *)calloc(nw0, sizeof(double));
        double *gw1 = (double *)calloc(nw1, sizeof(double));
        double *gw2 = (double *)calloc(nw2, sizeof(double));
        double *gb0 = (double *)calloc(H, sizeof(double));
        double *gb1 = (double *)calloc(H, sizeof(double));
        double *gb2 = (double *)calloc(O, sizeof(double));
        double *dh1 = (double *)malloc(sizeof(double) * H);
        double *dp1 = (double *)malloc(sizeof(double) * H);
        double *dp0 = (double *)malloc(sizeof(double) * H);
        double *dx = (double *)malloc(sizeof(double) * I);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < n; ++r) {
            ray_out ro;
            render_ray(g, m, op, o + 3 * r, d + 3 * r, &ro, recs, xs, h1s, h2s, cs, 0);
            if (rgb_out) for (int ch = 0; ch < 3; ++ch) rgb_out[3 * r + ch] = ro.rgb[ch];
            if (depth_out) depth_out[r] = ro.depth_t;
            if (acc_out) acc_out[r] = ro.acc;
            int ne = ro.n_eval;
            if (ne == 0) continue;
            double gr[3] = {d_rgb[3 * r], d_rgb[3 * r + 1], d_rgb[3 * r + 2]};
            double gdep = d_depth_t ? d_depth_t[r] : 0.0;
            double gacc = d_acc ? d_acc[r] : 0.0;
            double delta = ro.delta;
            /* suffix sums: R_k = sum_{j>k} w_j c_j + T_stop*bg,
             * D_k = sum_{j>k} w_j t_j */
            double Rc[3] = {ro.T_stop * op->bg[0], ro.T_stop * op->bg[1], ro.T_stop * op->bg[2]};
            double Dc = 0.0;
            for (int s = ne - 1; s >= 0; --s) {
                for (int ch = 0; ch < 3; ++ch) Rs[3 * s + ch] = Rc[ch];
                Ds[s] = Dc;
                for (int ch = 0; ch < 3; ++ch) Rc[ch] += recs[s].w * cs[(int64_t)s * O + ch];
                Dc += recs[s].w * (double)recs[s].tk;
            }
            for (int s = 0; s < ne; ++s) {
                sample_rec *q = &recs[s];
                const double *c = cs + (int64_t)s * O;
                const double *x = xs + (int64_t)s * I;
                const double *h1 = h1s + (int64_t)s * H;
                const double *h2 = h2s + (int64_t)s * H;
                /* compositing adjoint */
                double dsig = 0.0;
                for (int ch = 0; ch < 3; ++ch) dsig += gr[ch] * (q->T_next * c[ch] - Rs[3 * s + ch]);
                dsig += gdep * (q->T_next * (double)q->tk - Ds[s]);
                dsig += gacc * ro.T_stop;
                dsig *= delta;
                double draw = dsig * sigmoid_d(q->raw + (double)g->density_shift);
                /* MLP adjoint */
                double dlog[8];
                for (int ch = 0; ch < O; ++ch) {
                    double dc = (ch < 3) ? q->w * gr[ch] : 0.0;
                    dlog[ch] = dc * c[ch] * (1.0 - c[ch]);
                    gb2[ch] += dlog[ch];
                    for (int u = 0; u < H; ++u) gw2[(int64_t)ch * H + u] += dlog[ch] * h2[u];
                }
                for (int u = 0; u < H; ++u) {
                    double s2 = 0.0;
                    for (int ch = 0; ch < O; ++ch) s2 += (double)m->w2[(int64_t)ch * H + u] * dlog[ch];
                    dp1[u] = h2[u] > 0.0 ? s2 : 0.0;
                }
                for (int u = 0; u < H; ++u) {
                    gb1[u] += dp1[u];
                    if (dp1[u] != 0.0)
                        for (int v = 0; v < H; ++v) gw1[(int64_t)u * H + v] += dp1[u] * h1[v];
                }
                for (int v = 0; v < H; ++v) {
                    double s1 = 0.0;
                    for (int u = 0; u < H; ++u) s1 += (double)m->w1[(int64_t)u * H + v] * dp1[u];
                    dh1[v] = s1;
                    dp0[v] = h1[v] > 0.0 ? s1 : 0.0;
                }
                for (int u = 0; u < H; ++u) {
                    gb0[u] += dp0[u];
                    if (dp0[u] != 0.0)
                        for (int i = 0; i < I; ++i) gw0[(int64_t)u * I + i] += dp0[u] * x[i];
                }
                for (int i = 0; i < C; ++i) {
                    double s0 = 0.0;
                    for (int u = 0; u < H; ++u) s0 += (double)m->w0[(int64_t)u * I + i] * dp0[u];
                    dx[i] = s0;
                }
                /* trilinear scatter (transpose of the gather) */
                double wv[8];
                int64_t idx[8];
                trilinear_weights(q->fr, wv);
                corner_indices(g, q->i0, idx);
                for (int v = 0; v < 8; ++v) {
#pragma omp atomic
                    d_density[idx[v]] += wv[v] * draw;
                    for (int ch = 0; ch < C; ++ch) {
#pragma omp atomic
                        d_features[idx[v] * C + ch] += wv[v] * dx[ch];
                    }
                }
            }
        }
#pragma omp critical
        {
            for (int64_t i = 0; i < nw0; ++i) d_w0[i] += gw0[i];
            for (int64_t i = 0; i < nw1; ++i) d_w1[i] += gw1[i];
            for (int64_t i = 0; i < nw2; ++i) d_w2[i] += gw2[i];
            for (int i = 0; i < H; ++i) { d_b0[i] += gb0[i]; d_b1[i] += gb1[i]; }
            for (int i = 0; i < O; ++i) d_b2[i] += gb2[i];
        }
        free(recs); free(xs); free(h1s); free(h2s); free(cs); free(Rs); free(Ds);
        free(gw0); free(gw1); free(gw2); free(gb0); free(gb1); free(gb2);
        free(dh1); free(dp1); free(dp0); free(dx);
    }
}
