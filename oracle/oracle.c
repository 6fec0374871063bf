/*
 * FP64 CPU oracle for Differentiable Radiative Rasterization (DRR) of
 * radiative 3D Gaussians through a circular cone-beam X-ray camera.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Structure (paper: "Radiative Gaussian Splatting for Efficient X-ray Novel
 * View Synthesis", Sec. 3.2 and 3.3):
 *   - camera from scanner parameters ............ Eq. 12, W of Eq. 9
 *   - projection of a Gaussian .................. Eq. 7, Eq. 8, Eq. 9, and the
 *                                                 2-D covariance obtained by
 *                                                 dropping row/col 3 (Sec. 3.2)
 *   - tile assignment and depth ordering ........ Sec. 3.2 (tiles, sorted lists)
 *   - front-to-back blending .................... Eq. 10
 *   - adjoint of the above ...................... exact derivative of Eq. 10
 *                                                 with discrete decisions fixed
 *
 * Readings of the paper used here (each is also listed in the design notes):
 *   - sigma_j of Eq. 10 is the EWA footprint at the pixel centre:
 *     sigma_j = min(alpha_max, o_j * exp(-1/2 d^T Sigma''^-1 d)), d = p + 1/2 - u_j
 *   - a low-pass term k*I is added to Sigma'' (k = 0 is the literal paper)
 *   - evaluations with sigma < alpha_min are skipped; blending stops before
 *     a Gaussian that would push the transmittance below t_min
 *   - order: ascending camera depth t_z (bits of the float32 depth), ties by
 *     ascending Gaussian index; background 0
 *   - a Gaussian is considered at a pixel only if the pixel lies in its
 *     integer bounding rectangle, computed by a fixed float32 operation
 *     sequence ("key path", function key_path below) so that the rectangle
 *     and the depth are reproducible bit for bit by any float32 IEEE
 *     implementation.  Everything else is float64.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math:
 * the key path needs IEEE binary32 round-to-nearest with no contraction).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ABI 4

typedef struct {
    float rot[9];     /* rotation block of M_ext, row-major (Eq. 12) */
    float trans[3];   /* translation column of M_ext: (0, 0, L_SO) */
    float fx, fy;     /* focal lengths in pixels (M_int, Eq. 12) */
    float cx, cy;     /* principal point W/2, H/2 (M_int, Eq. 12) */
    int32_t width, height;
} orc_cam;

typedef struct {
    float lowpass;    /* k added to the diagonal of Sigma'' (px^2) */
    float alpha_min;  /* skip threshold for sigma_j */
    float alpha_max;  /* clamp for sigma_j */
    float t_min;      /* transmittance termination threshold */
    float near_z;     /* cull t_z <= near_z */
    int32_t tile;     /* tile side in pixels (tile assignment only) */
} orc_set;

/* Per (view, Gaussian) projection. */
typedef struct {
    int32_t kept;
    uint32_t depth_bits;      /* float32 bits of t_z from the key path */
    int32_t rect[4];          /* x_lo, x_hi, y_lo, y_hi (inclusive pixels) */
    float key_u[2];           /* float32 centre from the key path */
    float key_s[3];           /* float32 Sxx, Sxy, Syy from the key path */
    double t[3];              /* camera-space centre */
    double u[2];              /* image-space centre */
    double sig[3];            /* Sigma'' = (Sxx, Sxy, Syy), incl. low-pass */
    double conic[3];          /* Sigma''^-1 = (A, B, C) */
} orc_proj;

int orc_abi_version(void) { return ORC_ABI; }

#ifdef _OPENMP
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif

/* ---------------------------------------------------------------------------
 * Camera, Eq. 12: M_ext has rotation rows (-sin phi, cos phi, 0), (0, 0, -1),
 * (-cos phi, -sin phi, 0) and translation (0, 0, L_SO); M_int has the focal
 * length and principal point (W/2, H/2).  The paper uses L_SD directly as
 * the focal length (pixel pitch 1); with a physical detector of side det_w
 * covering W pixels the focal length in pixels is (L_SD * W) / det_w.
 * Computed in float64 and rounded once to float32.
 * ------------------------------------------------------------------------- */
void orc_camera(double phi, double l_so, double l_sd, int32_t w, int32_t h,
                double det_w, double det_h, orc_cam *c)
{
    double s = sin(phi), co = cos(phi);
    double r[9] = {-s, co, 0.0, 0.0, 0.0, -1.0, -co, -s, 0.0};
    for (int k = 0; k < 9; ++k) c->rot[k] = (float)r[k];
    c->trans[0] = 0.0f;
    c->trans[1] = 0.0f;
    c->trans[2] = (float)l_so;
    c->fx = (float)((l_sd * (double)w) / det_w);
    c->fy = (float)((l_sd * (double)h) / det_h);
    c->cx = (float)((double)w / 2.0);
    c->cy = (float)((double)h / 2.0);
    c->width = w;
    c->height = h;
}

/* Squared Mahalanobis radius of the bounding rectangle:
 * o * exp(-m^2/2) >= alpha_min with o <= 1 implies m^2 <= 2 ln(1/alpha_min). */
float orc_kappa(float alpha_min)
{
    return (float)(-2.0 * log((double)alpha_min));
}

/* ---------------------------------------------------------------------------
 * Key path: fixed float32 operation sequence for depth, culling and the
 * integer bounding rectangle.  Every operation is one IEEE binary32
 * round-to-nearest-even operation, evaluated left to right as parenthesised.
 * Returns 1 if the Gaussian is kept.
 * ------------------------------------------------------------------------- */
static int key_path(const double *mean, const double *scale, const double *quat,
                    double opac, const orc_cam *c, const orc_set *st, float kappa,
                    orc_proj *p)
{
    const float *r = c->rot;
    float mx = (float)mean[0], my = (float)mean[1], mz = (float)mean[2];
    /* t = R mu + tau (Eq. 7) */
    float tx = ((r[0] * mx + r[1] * my) + r[2] * mz) + c->trans[0];
    float ty = ((r[3] * mx + r[4] * my) + r[5] * mz) + c->trans[1];
    float tz = ((r[6] * mx + r[7] * my) + r[8] * mz) + c->trans[2];
    if (!(isfinite(tx) && isfinite(ty) && isfinite(tz))) return 0;
    if (!(tz > st->near_z)) return 0;
    /* unit quaternion */
    float qw = (float)quat[0], qx = (float)quat[1], qy = (float)quat[2], qz = (float)quat[3];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(n2 > 0.0f)) return 0;
    float nn = sqrtf(n2);
    float w = qw / nn, x = qx / nn, y = qy / nn, z = qz / nn;
    /* rotation matrix of the unit quaternion (scalar first) */
    float R[9];
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
    float s0 = (float)scale[0], s1 = (float)scale[1], s2 = (float)scale[2];
    float M[9];
    for (int a = 0; a < 3; ++a) {
        M[3 * a + 0] = R[3 * a + 0] * s0;
        M[3 * a + 1] = R[3 * a + 1] * s1;
        M[3 * a + 2] = R[3 * a + 2] * s2;
    }
    /* Jacobian of the projection (Eq. 9), first two rows */
    float tz2 = tz * tz;
    float J00 = c->fx / tz;
    float J11 = c->fy / tz;
    float J02 = -((c->fx * tx) / tz2);
    float J12 = -((c->fy * ty) / tz2);
    /* A = J W (2x3) */
    float A[6];
    for (int k = 0; k < 3; ++k) {
        A[k] = J00 * r[k] + J02 * r[6 + k];
        A[3 + k] = J11 * r[3 + k] + J12 * r[6 + k];
    }
    /* B = A M (2x3) */
    float B[6];
    for (int row = 0; row < 2; ++row)
        for (int col = 0; col < 3; ++col)
            B[3 * row + col] = (A[3 * row + 0] * M[col] + A[3 * row + 1] * M[3 + col])
                               + A[3 * row + 2] * M[6 + col];
    /* Sigma'' = B B^T + k I (Eq. 8 without row/col 3) */
    float sxx = ((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]) + st->lowpass;
    float syy = ((B[3] * B[3] + B[4] * B[4]) + B[5] * B[5]) + st->lowpass;
    float sxy = (B[0] * B[3] + B[1] * B[4]) + B[2] * B[5];
    float det = sxx * syy - sxy * sxy;
    if (!(det > 0.0f)) return 0;
    if (!((float)opac >= st->alpha_min)) return 0;
    /* image-space centre (Eq. 7 with the perspective divide) */
    float ux = c->fx * (tx / tz) + c->cx;
    float uy = c->fy * (ty / tz) + c->cy;
    float rx = sqrtf(kappa * sxx);
    float ry = sqrtf(kappa * syy);
    float xl = ceilf((ux - rx) - 0.5f);
    float xh = floorf((ux + rx) - 0.5f);
    float yl = ceilf((uy - ry) - 0.5f);
    float yh = floorf((uy + ry) - 0.5f);
    float wmax = (float)(c->width - 1), hmax = (float)(c->height - 1);
    /* empty, or wholly outside the image (also rejects NaN) */
    if (!(xl <= xh) || !(xl <= wmax) || !(xh >= 0.0f)) return 0;
    if (!(yl <= yh) || !(yl <= hmax) || !(yh >= 0.0f)) return 0;
    xl = fmaxf(xl, 0.0f);
    xh = fminf(xh, wmax);
    yl = fmaxf(yl, 0.0f);
    yh = fminf(yh, hmax);
    uint32_t bits;
    memcpy(&bits, &tz, 4);
    p->depth_bits = bits;
    p->rect[0] = (int32_t)xl;
    p->rect[1] = (int32_t)xh;
    p->rect[2] = (int32_t)yl;
    p->rect[3] = (int32_t)yh;
    p->key_u[0] = ux;
    p->key_u[1] = uy;
    p->key_s[0] = sxx;
    p->key_s[1] = sxy;
    p->key_s[2] = syy;
    return 1;
}

/* Rotation matrix of a unit quaternion (w, x, y, z), float64. */
static void quat_rot(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

/* Float64 projection quantities of a kept Gaussian (Eq. 7-9). */
static void project64(const double *mean, const double *scale, const double *quat,
                      const orc_cam *c, const orc_set *st, orc_proj *p)
{
    double r[9];
    for (int k = 0; k < 9; ++k) r[k] = (double)c->rot[k];
    double t[3];
    for (int a = 0; a < 3; ++a)
        t[a] = r[3 * a] * mean[0] + r[3 * a + 1] * mean[1] + r[3 * a + 2] * mean[2]
               + (double)c->trans[a];
    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    double q[4] = {quat[0] / qn, quat[1] / qn, quat[2] / qn, quat[3] / qn};
    double R[9];
    quat_rot(q, R);
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * scale[b];
    double fx = c->fx, fy = c->fy;
    double J[6] = {fx / t[2], 0.0, -fx * t[0] / (t[2] * t[2]),
                   0.0, fy / t[2], -fy * t[1] / (t[2] * t[2])};
    double A[6], B[6];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k)
            A[3 * i + k] = J[3 * i] * r[k] + J[3 * i + 1] * r[3 + k] + J[3 * i + 2] * r[6 + k];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k)
            B[3 * i + k] = A[3 * i] * M[k] + A[3 * i + 1] * M[3 + k] + A[3 * i + 2] * M[6 + k];
    double k = (double)st->lowpass;
    double sxx = B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + k;
    double syy = B[3] * B[3] + B[4] * B[4] + B[5] * B[5] + k;
    double sxy = B[0] * B[3] + B[1] * B[4] + B[2] * B[5];
    double det = sxx * syy - sxy * sxy;
    for (int a = 0; a < 3; ++a) p->t[a] = t[a];
    p->u[0] = fx * t[0] / t[2] + (double)c->cx;
    p->u[1] = fy * t[1] / t[2] + (double)c->cy;
    p->sig[0] = sxx; p->sig[1] = sxy; p->sig[2] = syy;
    p->conic[0] = syy / det;
    p->conic[1] = -sxy / det;
    p->conic[2] = sxx / det;
}

void orc_project(int32_t n, const double *means, const double *scales, const double *quats,
                 const double *opacity, const orc_cam *c, const orc_set *st, orc_proj *out)
{
    float kappa = orc_kappa(st->alpha_min);
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        orc_proj *p = &out[i];
        memset(p, 0, sizeof(*p));
        p->kept = key_path(means + 3 * (int64_t)i, scales + 3 * (int64_t)i, quats + 4 * (int64_t)i,
                           opacity[i], c, st, kappa, p);
        if (p->kept)
            project64(means + 3 * (int64_t)i, scales + 3 * (int64_t)i, quats + 4 * (int64_t)i, c, st, p);
    }
}

/* ---------------------------------------------------------------------------
 * Tile assignment and ordering (Sec. 3.2).  A kept Gaussian is listed in
 * every tile its rectangle touches; within a tile, Gaussians are ordered by
 * ascending depth, ties by ascending index.  Encoded as a 64-bit key
 * (global tile id << 32 | depth bits) and a 32-bit value (Gaussian index).
 * Global tile ids number the tiles of view v after those of views < v,
 * row-major within a view.
 * ------------------------------------------------------------------------- */
static int32_t tiles_x(const orc_cam *c, int32_t tile) { return (c->width + tile - 1) / tile; }
static int32_t tiles_y(const orc_cam *c, int32_t tile) { return (c->height + tile - 1) / tile; }

int64_t orc_total_tiles(int32_t nv, const orc_cam *cams, int32_t tile)
{
    int64_t s = 0;
    for (int v = 0; v < nv; ++v) s += (int64_t)tiles_x(&cams[v], tile) * tiles_y(&cams[v], tile);
    return s;
}

/* Emits the (key, value) pairs of all views, unsorted, in (view, i, ty, tx)
 * order.  With keys == NULL only counts.  Returns the pair count. */
int64_t orc_emit_pairs(int32_t n, const double *means, const double *scales, const double *quats,
                       const double *opacity, int32_t nv, const orc_cam *cams, const orc_set *st,
                       uint64_t *keys, uint32_t *values)
{
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)(n > 0 ? n : 1));
    int64_t count = 0, toff = 0;
    int32_t T = st->tile;
    for (int32_t v = 0; v < nv; ++v) {
        orc_project(n, means, scales, quats, opacity, &cams[v], st, pr);
        int32_t tx_n = tiles_x(&cams[v], T);
        for (int32_t i = 0; i < n; ++i) {
            if (!pr[i].kept) continue;
            for (int32_t ty = pr[i].rect[2] / T; ty <= pr[i].rect[3] / T; ++ty)
                for (int32_t tx = pr[i].rect[0] / T; tx <= pr[i].rect[1] / T; ++tx) {
                    if (keys) {
                        uint64_t g = (uint64_t)(toff + (int64_t)ty * tx_n + tx);
                        keys[count] = (g << 32) | (uint64_t)pr[i].depth_bits;
                        values[count] = (uint32_t)i;
                    }
                    ++count;
                }
        }
        toff += (int64_t)tx_n * tiles_y(&cams[v], T);
    }
    free(pr);
    return count;
}

typedef struct { uint64_t k; uint32_t v; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}

/* Sorts pairs ascending by (key, value). */
void orc_sort_pairs(int64_t p, uint64_t *keys, uint32_t *values)
{
    kv_t *a = (kv_t *)malloc(sizeof(kv_t) * (size_t)(p > 0 ? p : 1));
    for (int64_t i = 0; i < p; ++i) { a[i].k = keys[i]; a[i].v = values[i]; }
    qsort(a, (size_t)p, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < p; ++i) { keys[i] = a[i].k; values[i] = a[i].v; }
    free(a);
}

/* ranges[2g], ranges[2g+1] = [start, end) of tile g in the sorted pairs;
 * (0, 0) for an empty tile. */
void orc_ranges(int64_t p, const uint64_t *keys, int64_t n_tiles, uint32_t *ranges)
{
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)n_tiles);
    for (int64_t i = 0; i < p; ++i) {
        int64_t g = (int64_t)(keys[i] >> 32);
        if (i == 0 || (keys[i - 1] >> 32) != (uint64_t)g) ranges[2 * g] = (uint32_t)i;
        ranges[2 * g + 1] = (uint32_t)(i + 1);
    }
}

/* ---------------------------------------------------------------------------
 * Blending of one pixel (Eq. 10), float64.  `order` lists Gaussian indices
 * in blending order; only those whose rectangle contains the pixel are
 * evaluated.  Margin flags mark decisions taken within a relative margin of
 * a threshold, where float32 and float64 may legitimately branch apart.
 * ------------------------------------------------------------------------- */
#define FLAG_ALPHA_MIN 1
#define FLAG_T_MIN 2
#define FLAG_CLAMP 4
#define DELTA_ALPHA 1e-5
#define DELTA_T 1e-4
#define DELTA_CLAMP 1e-5

typedef struct {
    int32_t idx;       /* Gaussian index */
    int32_t pos;       /* position in the traversed list (0-based) */
    double alpha, a, G, T, dx, dy;
    int clamped;
} contrib_t;

typedef struct {
    double I, T;
    int32_t last_pos;  /* list position of the last contributor, -1 if none */
    int32_t last_idx;  /* Gaussian index of the last contributor, -1 if none */
    int32_t evals;     /* in-rect evaluations incl. the terminating one */
    int32_t flags;     /* FLAG_* bits | (number of flagged decisions << 8) */
    int32_t ncontrib;
} pix_result;

/* flip != 0 renders the other branch of the pixel's first flagged decision
 * (the second admissible result of a pixel with one flagged decision). */
static void blend_pixel(int32_t px, int32_t py, const int32_t *order, int64_t len,
                        const orc_proj *pr, const double *opacity, const double *inten,
                        const orc_set *st, int flip, pix_result *res, contrib_t *out_list)
{
    double T = 1.0, C = 0.0;
    double amin = st->alpha_min, amax = st->alpha_max, tmin = st->t_min;
    /* t_min below the smallest normal float32 acts as that value (2^-126):
     * the float32 transmittance of the GPU path stays normal, so that the
     * recomputing backward can divide it back (the method's t_min, 1e-4,
     * is far above) */
    if (tmin < (double)FLT_MIN) tmin = (double)FLT_MIN;
    int32_t nflag = 0, flags = 0, evals = 0, nc = 0;
    res->last_pos = -1;
    res->last_idx = -1;
    double cxp = px + 0.5, cyp = py + 0.5;
    for (int64_t k = 0; k < len; ++k) {
        int32_t j = order[k];
        const orc_proj *p = &pr[j];
        if (px < p->rect[0] || px > p->rect[1] || py < p->rect[2] || py > p->rect[3]) continue;
        ++evals;
        double dx = cxp - p->u[0], dy = cyp - p->u[1];
        double power = -0.5 * (p->conic[0] * dx * dx + p->conic[2] * dy * dy) - p->conic[1] * dx * dy;
        double G = exp(power);
        double a = opacity[j] * G;
        int clamped = a > amax;
        if (fabs(a - amax) <= DELTA_CLAMP * amax) {
            flags |= FLAG_CLAMP;
            if (++nflag == 1 && flip) clamped = !clamped;
        }
        double alpha = clamped ? amax : a;
        int skip = alpha < amin;
        /* a zero threshold cannot be crossed by rounding (alpha >= 0, T >= 0) */
        if (amin > 0.0 && fabs(alpha - amin) <= DELTA_ALPHA * amin) {
            flags |= FLAG_ALPHA_MIN;
            if (++nflag == 1 && flip) skip = !skip;
        }
        if (skip) continue;
        double Tn = T * (1.0 - alpha);
        int stop = Tn < tmin;
        if (tmin > 0.0 && fabs(Tn - tmin) <= DELTA_T * tmin) {
            flags |= FLAG_T_MIN;
            if (++nflag == 1 && flip) stop = !stop;
        }
        /* the Gaussian that would take T below t_min is not blended, and
         * blending ends there */
        if (stop) break;
        if (out_list) {
            contrib_t *cb = &out_list[nc];
            cb->idx = j; cb->pos = (int32_t)k; cb->alpha = alpha; cb->a = a; cb->G = G;
            cb->T = T; cb->dx = dx; cb->dy = dy; cb->clamped = clamped;
        }
        ++nc;
        C += inten[j] * alpha * T;
        T = Tn;
        res->last_pos = (int32_t)k;
        res->last_idx = j;
    }
    res->I = C;
    res->T = T;
    res->evals = evals;
    res->ncontrib = nc;
    res->flags = flags | (nflag << 8);
}

/* Kept Gaussians of one view in blending order (ascending depth bits, ties by index). */
static const orc_proj *g_sort_pr;
static int order_cmp(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    uint32_t di = g_sort_pr[i].depth_bits, dj = g_sort_pr[j].depth_bits;
    if (di != dj) return di < dj ? -1 : 1;
    return i < j ? -1 : (i > j);
}

static int64_t depth_order(int32_t n, const orc_proj *pr, int32_t *order)
{
    int64_t len = 0;
    for (int32_t i = 0; i < n; ++i)
        if (pr[i].kept) order[len++] = i;
    g_sort_pr = pr;
    qsort(order, (size_t)len, sizeof(int32_t), order_cmp);
    return len;
}

/* Brute-force forward for selected pixels of one view: every kept Gaussian
 * is visited in depth order.  pix[k] = y * width + x.  last[k] = Gaussian
 * index of the last contributor (-1 if none). */
void orc_render_brute(int32_t n, const double *means, const double *scales, const double *quats,
                      const double *opacity, const double *inten, const orc_cam *c,
                      const orc_set *st, int64_t npix, const int32_t *pix, const uint8_t *flip,
                      double *img, double *tfin, int32_t *last, int32_t *evals, int32_t *flags)
{
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)(n > 0 ? n : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_project(n, means, scales, quats, opacity, c, st, pr);
    int64_t len = depth_order(n, pr, order);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; ++k) {
        int32_t px = pix[k] % c->width, py = pix[k] / c->width;
        pix_result r;
        blend_pixel(px, py, order, len, pr, opacity, inten, st, flip ? flip[k] : 0, &r, NULL);
        img[k] = r.I;
        tfin[k] = r.T;
        if (last) last[k] = r.last_idx;
        if (evals) evals[k] = r.evals;
        if (flags) flags[k] = r.flags;
    }
    free(order);
    free(pr);
}

/* Binned forward over all pixels of all views: each pixel traverses its
 * tile's sorted list (values[ranges[2g] .. ranges[2g+1]]).  ncontrib is
 * the 1-based list position of the last contributor (0 if none).  Output
 * arrays are the views' images concatenated, row-major.  flip (nullable,
 * per pixel): render the other branch of the pixel's first flagged
 * decision; only (nullable, per pixel): process just the pixels where it is
 * nonzero, leaving the outputs of the others untouched. */
void orc_render_binned(int32_t n, const double *means, const double *scales, const double *quats,
                       const double *opacity, const double *inten, int32_t nv, const orc_cam *cams,
                       const orc_set *st, const uint32_t *values, const uint32_t *ranges,
                       const uint8_t *flip, const uint8_t *only,
                       double *img, double *tfin, int32_t *ncontrib, int32_t *evals, int32_t *flags)
{
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)(n > 0 ? n : 1));
    int64_t poff = 0, toff = 0;
    int32_t T = st->tile;
    for (int32_t v = 0; v < nv; ++v) {
        const orc_cam *c = &cams[v];
        orc_project(n, means, scales, quats, opacity, c, st, pr);
        int32_t txn = tiles_x(c, T);
        int32_t W = c->width, H = c->height;
        #pragma omp parallel for schedule(dynamic, 1)
        for (int32_t py = 0; py < H; ++py) {
            for (int32_t px = 0; px < W; ++px) {
                int64_t o = poff + (int64_t)py * W + px;
                if (only && !only[o]) continue;
                int64_t g = toff + (int64_t)(py / T) * txn + px / T;
                uint32_t s = ranges[2 * g], e = ranges[2 * g + 1];
                pix_result r;
                blend_pixel(px, py, (const int32_t *)(values + s), (int64_t)e - s, pr, opacity,
                            inten, st, flip ? flip[o] : 0, &r, NULL);
                img[o] = r.I;
                tfin[o] = r.T;
                if (ncontrib) ncontrib[o] = r.last_pos + 1;
                if (evals) evals[o] = r.evals;
                if (flags) flags[o] = r.flags;
            }
        }
        poff += (int64_t)W * H;
        toff += (int64_t)txn * tiles_y(c, T);
    }
    free(pr);
}

/* ---------------------------------------------------------------------------
 * Adjoint.  For a pixel with upstream gradient g and contributors j = 1..n
 * (transmittance T_j before j, I = sum_j i_j alpha_j T_j):
 *   dI/d i_j     = alpha_j T_j
 *   dI/d alpha_j = T_j (i_j - R_j),  R_j = sum_{k>j} i_k alpha_k T_k / T_{j+1}
 *   R_{j-1}      = i_j alpha_j + (1 - alpha_j) R_j,  R_n = 0
 * alpha = min(alpha_max, a), a = o G, G = exp(power),
 * power = -1/2 (A dx^2 + 2 B dx dy + C dy^2), d = pixel centre - u.
 * Per (view, Gaussian) this accumulates the 2-D gradients
 *   g2d = (dL/du_x, dL/du_y, dL/dA, dL/dB, dL/dC, dL/do, dL/di)
 * which chain3d() maps to the 3-D parameters.
 * ------------------------------------------------------------------------- */
static void pixel_adjoint(double g, const contrib_t *cl, int32_t nc, const orc_proj *pr,
                          const double *inten, double *g2d /* [n*7] for this view */)
{
    double R = 0.0;
    for (int32_t m = nc - 1; m >= 0; --m) {
        const contrib_t *cb = &cl[m];
        int32_t j = cb->idx;
        const orc_proj *p = &pr[j];
        double gi = g * cb->alpha * cb->T;
        double galpha = g * cb->T * (inten[j] - R);
        R = inten[j] * cb->alpha + (1.0 - cb->alpha) * R;
        double ga = cb->clamped ? 0.0 : galpha;
        double go = ga * cb->G;
        double gp = ga * cb->a;
        double A = p->conic[0], B = p->conic[1], C = p->conic[2];
        double dx = cb->dx, dy = cb->dy;
        double *o = g2d + 7 * (int64_t)j;
        double v[7] = {gp * (A * dx + B * dy), gp * (B * dx + C * dy),
                       gp * (-0.5 * dx * dx), gp * (-dx * dy), gp * (-0.5 * dy * dy), go, gi};
        for (int q = 0; q < 7; ++q) {
            #pragma omp atomic
            o[q] += v[q];
        }
    }
}

/* Per 8 x 8 pixel block of every view (blocks at multiples of 8 from the
 * view's origin, clipped at its edges): the number of distinct Gaussians
 * that are a contributor of at least one pixel of the block, i.e. the
 * Gaussians whose gradient terms a block-sized group of pixels sums.
 * Written at the block's first pixel (concatenated image layout); every
 * other pixel gets 0.  Pixels traverse their tiles' lists (values, ranges). */
void orc_block_contributors(int32_t n, const double *means, const double *scales,
                            const double *quats, const double *opacity, const double *inten,
                            int32_t nv, const orc_cam *cams, const orc_set *st,
                            const uint32_t *values, const uint32_t *ranges, int32_t *out)
{
    int32_t nn = n > 0 ? n : 1;
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)nn);
    int64_t poff = 0, toff = 0;
    int32_t T = st->tile;
    for (int32_t v = 0; v < nv; ++v) {
        const orc_cam *c = &cams[v];
        int32_t W = c->width, H = c->height;
        orc_project(n, means, scales, quats, opacity, c, st, pr);
        int32_t txn = tiles_x(c, T);
        int32_t bw = (W + 7) / 8, bh = (H + 7) / 8;
        memset(out + poff, 0, sizeof(int32_t) * (size_t)W * H);
        int64_t ntv = (int64_t)txn * tiles_y(c, T), longest = 1;
        for (int64_t g = toff; g < toff + ntv; ++g)
            if ((int64_t)(ranges[2 * g + 1] - ranges[2 * g]) > longest)
                longest = (int64_t)(ranges[2 * g + 1] - ranges[2 * g]);
        #pragma omp parallel
        {
            contrib_t *cl = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)longest);
            int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
            for (int32_t i = 0; i < nn; ++i) seen[i] = -1;
            #pragma omp for schedule(dynamic, 1)
            for (int32_t by = 0; by < bh; ++by) {
                for (int32_t bx = 0; bx < bw; ++bx) {
                    int64_t blk = (int64_t)by * bw + bx;
                    int32_t cnt = 0;
                    for (int32_t py = 8 * by; py < 8 * by + 8 && py < H; ++py)
                        for (int32_t px = 8 * bx; px < 8 * bx + 8 && px < W; ++px) {
                            int64_t gt = toff + (int64_t)(py / T) * txn + px / T;
                            uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
                            pix_result r;
                            blend_pixel(px, py, (const int32_t *)(values + s), (int64_t)e - s, pr,
                                        opacity, inten, st, 0, &r, cl);
                            for (int32_t m = 0; m < r.ncontrib; ++m)
                                if (seen[cl[m].idx] != blk) { seen[cl[m].idx] = blk; ++cnt; }
                        }
                    out[poff + (int64_t)(8 * by) * W + 8 * bx] = cnt;
                }
            }
            free(seen);
            free(cl);
        }
        poff += (int64_t)W * H;
        toff += (int64_t)txn * tiles_y(c, T);
    }
    free(pr);
}

/* Chain rule from the 2-D gradients of one (view, Gaussian) to the 3-D
 * parameters (mean, scale, unnormalised quaternion), accumulating. */
static void chain3d(const double *scale, const double *quat,
                    const orc_cam *c, const orc_proj *p, const double *g2,
                    double *gm, double *gs, double *gq)
{
    double r[9];
    for (int k = 0; k < 9; ++k) r[k] = (double)c->rot[k];
    double fx = c->fx, fy = c->fy;
    const double *t = p->t;
    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    double q[4] = {quat[0] / qn, quat[1] / qn, quat[2] / qn, quat[3] / qn};
    double R[9];
    quat_rot(q, R);
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * scale[b];
    double J[6] = {fx / t[2], 0.0, -fx * t[0] / (t[2] * t[2]),
                   0.0, fy / t[2], -fy * t[1] / (t[2] * t[2])};
    double A2[6], B[6];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k)
            A2[3 * i + k] = J[3 * i] * r[k] + J[3 * i + 1] * r[3 + k] + J[3 * i + 2] * r[6 + k];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k)
            B[3 * i + k] = A2[3 * i] * M[k] + A2[3 * i + 1] * M[3 + k] + A2[3 * i + 2] * M[6 + k];
    /* conic -> Sigma'': dL/dSigma = -Q G_Q Q with G_Q symmetric,
     * off-diagonal entries carrying half of dL/dB each */
    double QA = p->conic[0], QB = p->conic[1], QC = p->conic[2];
    double Q[4] = {QA, QB, QB, QC};
    double GQ[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    double T1[4], GS[4];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) T1[2 * i + k] = GQ[2 * i] * Q[k] + GQ[2 * i + 1] * Q[2 + k];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) GS[2 * i + k] = -(Q[2 * i] * T1[k] + Q[2 * i + 1] * T1[2 + k]);
    double gxx = GS[0], gyy = GS[3], gxy = GS[1] + GS[2];
    /* Sigma'' = B B^T + k I */
    double GB[6];
    for (int k = 0; k < 3; ++k) {
        GB[k] = 2.0 * gxx * B[k] + gxy * B[3 + k];
        GB[3 + k] = 2.0 * gyy * B[3 + k] + gxy * B[k];
    }
    /* B = A2 M */
    double GA2[6], GM[9];
    for (int i = 0; i < 2; ++i)
        for (int a = 0; a < 3; ++a) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += GB[3 * i + k] * M[3 * a + k];
            GA2[3 * i + a] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) GM[3 * a + k] = A2[a] * GB[k] + A2[3 + a] * GB[3 + k];
    /* M = R diag(s) */
    double GR[9];
    for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int a = 0; a < 3; ++a) s += GM[3 * a + b] * R[3 * a + b];
        gs[b] += s;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GR[3 * a + b] = GM[3 * a + b] * scale[b];
    /* R(q) */
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double dRw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    double dRx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    double dRy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    double dRz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    double gqh[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k) {
        gqh[0] += GR[k] * dRw[k];
        gqh[1] += GR[k] * dRx[k];
        gqh[2] += GR[k] * dRy[k];
        gqh[3] += GR[k] * dRz[k];
    }
    double dot = q[0] * gqh[0] + q[1] * gqh[1] + q[2] * gqh[2] + q[3] * gqh[3];
    for (int k = 0; k < 4; ++k) gq[k] += (gqh[k] - q[k] * dot) / qn;
    /* A2 = J W: dL/dJ = GA2 W^T */
    double GJ[6];
    for (int i = 0; i < 2; ++i)
        for (int a = 0; a < 3; ++a)
            GJ[3 * i + a] = GA2[3 * i] * r[3 * a] + GA2[3 * i + 1] * r[3 * a + 1]
                            + GA2[3 * i + 2] * r[3 * a + 2];
    /* J(t) and u(t) */
    double tz = t[2], tz2 = tz * tz, tz3 = tz2 * tz;
    double gt[3];
    gt[0] = GJ[2] * (-fx / tz2) + g2[0] * (fx / tz);
    gt[1] = GJ[5] * (-fy / tz2) + g2[1] * (fy / tz);
    gt[2] = GJ[0] * (-fx / tz2) + GJ[2] * (2.0 * fx * t[0] / tz3)
            + GJ[4] * (-fy / tz2) + GJ[5] * (2.0 * fy * t[1] / tz3)
            + g2[0] * (-fx * t[0] / tz2) + g2[1] * (-fy * t[1] / tz2);
    /* t = W mu + tau */
    for (int a = 0; a < 3; ++a) gm[a] += r[a] * gt[0] + r[3 + a] * gt[1] + r[6 + a] * gt[2];
}

/* Adjoint of the forward for all views.  dl_di is the upstream gradient of
 * the concatenated images (float32, as fed to the GPU path).  If `binned`,
 * pixels traverse their tile lists (values, ranges as from the sorted pairs);
 * otherwise every kept Gaussian in depth order.  If sel != NULL, only pixels
 * inside the rectangle of a selected Gaussian are processed (gradients of
 * selected Gaussians are then exact; others are partial).  Gradients are
 * accumulated (+=).  g2d_out, if non-NULL, receives the 2-D gradients
 * [nv][n][7]. */
void orc_backward(int32_t n, const double *means, const double *scales, const double *quats,
                  const double *opacity, const double *inten, int32_t nv, const orc_cam *cams,
                  const orc_set *st, const float *dl_di, int32_t binned,
                  const uint32_t *values, const uint32_t *ranges, const uint8_t *sel,
                  const uint8_t *flip,
                  double *g_means, double *g_scales, double *g_quats, double *g_opac,
                  double *g_inten, double *g2d_out)
{
    int32_t nn = n > 0 ? n : 1;
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)nn);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
    double *g2d = (double *)malloc(sizeof(double) * 7 * (size_t)nn);
    int64_t poff = 0, toff = 0;
    int32_t T = st->tile;
    for (int32_t v = 0; v < nv; ++v) {
        const orc_cam *c = &cams[v];
        int32_t W = c->width, H = c->height;
        orc_project(n, means, scales, quats, opacity, c, st, pr);
        int64_t len = depth_order(n, pr, order);
        memset(g2d, 0, sizeof(double) * 7 * (size_t)nn);
        uint8_t *mask = NULL;
        if (sel) {
            mask = (uint8_t *)calloc((size_t)W * H, 1);
            for (int32_t i = 0; i < n; ++i) {
                if (!sel[i] || !pr[i].kept) continue;
                for (int32_t y = pr[i].rect[2]; y <= pr[i].rect[3]; ++y)
                    memset(mask + (int64_t)y * W + pr[i].rect[0], 1,
                           (size_t)(pr[i].rect[1] - pr[i].rect[0] + 1));
            }
        }
        int32_t txn = tiles_x(c, T);
        #pragma omp parallel
        {
            contrib_t *cl = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)(len > 0 ? len : 1));
            #pragma omp for schedule(dynamic, 1)
            for (int32_t py = 0; py < H; ++py) {
                for (int32_t px = 0; px < W; ++px) {
                    int64_t o = (int64_t)py * W + px;
                    if (mask && !mask[o]) continue;
                    double g = (double)dl_di[poff + o];
                    if (g == 0.0) continue;
                    pix_result r;
                    int fl = flip ? flip[poff + o] : 0;
                    if (binned) {
                        int64_t gt = toff + (int64_t)(py / T) * txn + px / T;
                        uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];
                        blend_pixel(px, py, (const int32_t *)(values + s), (int64_t)e - s, pr,
                                    opacity, inten, st, fl, &r, cl);
                    } else {
                        blend_pixel(px, py, order, len, pr, opacity, inten, st, fl, &r, cl);
                    }
                    pixel_adjoint(g, cl, r.ncontrib, pr, inten, g2d);
                }
            }
            free(cl);
        }
        free(mask);
        for (int32_t i = 0; i < n; ++i) {
            if (!pr[i].kept) continue;
            const double *g2 = g2d + 7 * (int64_t)i;
            if (g2d_out) memcpy(g2d_out + 7 * ((int64_t)v * n + i), g2, 7 * sizeof(double));
            chain3d(scales + 3 * (int64_t)i, quats + 4 * (int64_t)i, c,
                    &pr[i], g2, g_means + 3 * (int64_t)i, g_scales + 3 * (int64_t)i,
                    g_quats + 4 * (int64_t)i);
            g_opac[i] += g2[5];
            g_inten[i] += g2[6];
        }
        poff += (int64_t)W * H;
        toff += (int64_t)txn * tiles_y(c, T);
    }
    free(g2d);
    free(order);
    free(pr);
}
