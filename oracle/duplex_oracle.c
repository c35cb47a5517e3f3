/*
 * duplex_oracle.c -- CPU reference of the Duplex-GS proxy-guided renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker the HIP
 * path is compared against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product never does.  It shares no
 * code, header or table with the HIP library.
 *
 * What is computed (Duplex-GS, arXiv 2508.03180):
 *   - Cell rasterization (Sec. IV-B): every ellipsoidal cell proxy is culled
 *     against the near plane, its screen footprint is bounded, it is assigned
 *     to the 16x16 tiles it touches and the (tile, depth) sequence is sorted.
 *   - Hybrid renderer (Sec. V-A, eq. hybrid_renderer with w_n = v_n T_n and
 *     eq. dulpex_T): inside a cell the Gaussians are summed order-free, across
 *     cells the weight is the cell transmittance built from the products
 *     (1 - v_i alpha_{i,k}) of the cells in front.
 *   - Cell-level early termination (Sec. V-B): the walk stops once the
 *     transmittance in front of a cell is below eps.
 *   - False-positive skip (Sec. VI-A): a Gaussian is skipped at pixels outside
 *     its axis-aligned bounding box.
 *   - alpha_i = sigma_i G'_i(x') (eq. alpha_blending); per-Gaussian sorted
 *     alpha blending (eqs. alpha_blending, transmittance) for the baseline.
 *   - Termination ratio counters N^val, N^rendered (Sec. VII ablation, r^ET).
 *
 * Two layers:
 *   discrete layer (IEEE binary32, no contraction, correctly rounded sqrt and
 *   division, the fixed operation order documented in the design notes): every
 *   integer or yes/no decision -- near cull, pixel rectangles, tile rectangles,
 *   depth key bits.  It is evaluated in the renderer's own precision so that
 *   both sides take each decision identically.
 *   continuous layer (binary64): projected means, conics, colours, v_n, alpha
 *   and the per-pixel recurrence.
 *
 * Decisions that a threshold takes on a continuous value (alpha >= alpha_min,
 * T >= eps) are "marginal" when the value lies within a relative band of the
 * threshold; the pixel is then re-evaluated with those decisions flipped and
 * every resulting value is reported as admissible.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16
#define MAX_ALT 8

/* ------------------------------------------------------------------ */
/* camera                                                               */
/* cam[] = R00..R22 (row-major world->camera rotation), t0..t2,          */
/*         fx, fy, cx, cy, width, height, z_near                         */
/* ------------------------------------------------------------------ */
typedef struct {
    float R[9], t[3], fx, fy, cx, cy, znear;
    int W, H, TX, TY;
    float limx, limy;
    double Rd[9], td[3], od[3]; /* camera centre o = -R^T t */
} cam_t;

static void cam_load(const float *c, cam_t *k) {
    for (int i = 0; i < 9; i++) k->R[i] = c[i];
    for (int i = 0; i < 3; i++) k->t[i] = c[9 + i];
    k->fx = c[12]; k->fy = c[13]; k->cx = c[14]; k->cy = c[15];
    k->W = (int)c[16]; k->H = (int)c[17]; k->znear = c[18];
    k->TX = (k->W + TILE - 1) / TILE;
    k->TY = (k->H + TILE - 1) / TILE;
    k->limx = 1.3f * ((0.5f * (float)k->W) / k->fx);
    k->limy = 1.3f * ((0.5f * (float)k->H) / k->fy);
    for (int i = 0; i < 9; i++) k->Rd[i] = k->R[i];
    for (int i = 0; i < 3; i++) k->td[i] = k->t[i];
    for (int j = 0; j < 3; j++)
        k->od[j] = -(k->Rd[0 * 3 + j] * k->td[0] + k->Rd[1 * 3 + j] * k->td[1] + k->Rd[2 * 3 + j] * k->td[2]);
}

/* ================================================================== */
/* Discrete layer, binary32                                             */
/* ================================================================== */

/* world -> camera, one rounding per operation in this order */
static void view32(const cam_t *k, const float *p, float *o) {
    for (int i = 0; i < 3; i++)
        o[i] = ((k->R[i * 3 + 0] * p[0] + k->R[i * 3 + 1] * p[1]) + k->R[i * 3 + 2] * p[2]) + k->t[i];
}

/* quaternion (w,x,y,z) -> rotation, normalised first */
static void quat_rot32(const float *q, float *R) {
    float w = q[0], x = q[1], y = q[2], z = q[3];
    float n = sqrtf(((w * w + x * x) + y * y) + z * z);
    w = w / n; x = x / n; y = y / n; z = z / n;
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
}

/* 2D screen covariance of a 3D Gaussian (EWA splatting, local affine
 * approximation of the perspective map at the centre), returns xx, xy, yy */
static void ewa32(const cam_t *k, const float *tc, const float *s, const float *q, float *cov) {
    float R[9];
    quat_rot32(q, R);
    float M[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i * 3 + j] = R[i * 3 + j] * s[j];
    float S[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            S[i * 3 + j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
    float tz = tc[2];
    float txz = tc[0] / tz, tyz = tc[1] / tz;
    float txc = fminf(k->limx, fmaxf(-k->limx, txz)) * tz;
    float tyc = fminf(k->limy, fmaxf(-k->limy, tyz)) * tz;
    float tz2 = tz * tz;
    float j00 = k->fx / tz, j02 = -(k->fx * txc) / tz2;
    float j11 = k->fy / tz, j12 = -(k->fy * tyc) / tz2;
    float m0[3], m1[3];
    for (int j = 0; j < 3; j++) {
        m0[j] = j00 * k->R[0 * 3 + j] + j02 * k->R[2 * 3 + j];
        m1[j] = j11 * k->R[1 * 3 + j] + j12 * k->R[2 * 3 + j];
    }
    float w0[3], w1[3];
    for (int j = 0; j < 3; j++) {
        w0[j] = (m0[0] * S[0 * 3 + j] + m0[1] * S[1 * 3 + j]) + m0[2] * S[2 * 3 + j];
        w1[j] = (m1[0] * S[0 * 3 + j] + m1[1] * S[1 * 3 + j]) + m1[2] * S[2 * 3 + j];
    }
    cov[0] = (w0[0] * m0[0] + w0[1] * m0[1]) + w0[2] * m0[2];
    cov[1] = (w0[0] * m1[0] + w0[1] * m1[1]) + w0[2] * m1[2];
    cov[2] = (w1[0] * m1[0] + w1[1] * m1[1]) + w1[2] * m1[2];
}

/* inclusive integer pixel rectangle of the pixels whose centres (px + 0.5)
 * lie within [u - h, u + h]; returns 0 when it misses the image */
static int rect32(const cam_t *k, float ux, float uy, float hx, float hy, int32_t *r) {
    float x0 = ceilf((ux - hx) - 0.5f), x1 = floorf((ux + hx) - 0.5f);
    float y0 = ceilf((uy - hy) - 0.5f), y1 = floorf((uy + hy) - 0.5f);
    if (!(x0 <= x1) || !(y0 <= y1)) return 0;
    x0 = fmaxf(x0, 0.0f); x1 = fminf(x1, (float)(k->W - 1));
    y0 = fmaxf(y0, 0.0f); y1 = fminf(y1, (float)(k->H - 1));
    if (!(x0 <= x1) || !(y0 <= y1)) return 0;
    r[0] = (int32_t)x0; r[1] = (int32_t)x1; r[2] = (int32_t)y0; r[3] = (int32_t)y1;
    return 1;
}

static uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* Cell proxies: near cull, depth key, pixel and tile rectangles.
 * kappa scales the proxy ellipse, pad = 3 sqrt(delta) (a member's minimum
 * 3-sigma radius after the screen-space dilation). */
int orc_cells_discrete(int N, const float *pos, const float *scale, const float *rot, const float *camv,
                       float kappa, float delta, uint8_t *visible, uint32_t *depth_bits,
                       int32_t *rect, int32_t *trect, int32_t *ntiles) {
    cam_t k; cam_load(camv, &k);
    float pad = 3.0f * sqrtf(delta);
    for (int n = 0; n < N; n++) {
        float tc[3];
        view32(&k, pos + 3 * n, tc);
        visible[n] = 0; ntiles[n] = 0; depth_bits[n] = fbits(tc[2]);
        for (int i = 0; i < 4; i++) rect[4 * n + i] = trect[4 * n + i] = -1;
        if (!(tc[2] > k.znear)) continue;
        float cov[3];
        ewa32(&k, tc, scale + 3 * n, rot + 4 * n, cov);
        float ux = k.fx * (tc[0] / tc[2]) + k.cx;
        float uy = k.fy * (tc[1] / tc[2]) + k.cy;
        float hx = kappa * sqrtf(cov[0]) + pad;
        float hy = kappa * sqrtf(cov[2]) + pad;
        int32_t r[4];
        if (!rect32(&k, ux, uy, hx, hy, r)) continue;
        visible[n] = 1;
        for (int i = 0; i < 4; i++) { rect[4 * n + i] = r[i]; trect[4 * n + i] = r[i] / TILE; }
        ntiles[n] = (trect[4 * n + 1] - trect[4 * n + 0] + 1) * (trect[4 * n + 3] - trect[4 * n + 2] + 1);
    }
    return 0;
}

/* Gaussians: validity (sigma > 0), near cull, depth key, 3-sigma pixel
 * rectangle of the dilated screen covariance, tile count. */
int orc_gauss_discrete(int M, const float *means, const float *scales, const float *rots,
                       const float *opac, const float *camv, float delta, uint8_t *visible,
                       uint32_t *depth_bits, int32_t *rect, int32_t *ntiles) {
    cam_t k; cam_load(camv, &k);
    for (int g = 0; g < M; g++) {
        float tc[3];
        view32(&k, means + 3 * g, tc);
        visible[g] = 0; ntiles[g] = 0; depth_bits[g] = fbits(tc[2]);
        for (int i = 0; i < 4; i++) rect[4 * g + i] = -1;
        if (!(opac[g] > 0.0f) || !(tc[2] > k.znear)) continue;
        float cov[3];
        ewa32(&k, tc, scales + 3 * g, rots + 4 * g, cov);
        float a = cov[0] + delta, c = cov[2] + delta;
        float ux = k.fx * (tc[0] / tc[2]) + k.cx;
        float uy = k.fy * (tc[1] / tc[2]) + k.cy;
        float hx = 3.0f * sqrtf(a), hy = 3.0f * sqrtf(c);
        int32_t r[4];
        if (!rect32(&k, ux, uy, hx, hy, r)) continue;
        visible[g] = 1;
        for (int i = 0; i < 4; i++) rect[4 * g + i] = r[i];
        ntiles[g] = (r[1] / TILE - r[0] / TILE + 1) * (r[3] / TILE - r[2] / TILE + 1);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* (tile, depth) sequence: one entry per (primitive, touched tile),     */
/* ordered by tile, then depth key bits, then primitive id.             */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t tile, depth; int32_t id; } entry_t;

static int entry_cmp(const void *a, const void *b) {
    const entry_t *x = a, *y = b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Counts the entries of the primitives with visible != 0 over their pixel
 * rectangles (tile = rect / 16).  With out_ids == NULL only the count is
 * returned; otherwise out_ids[count] receives the sorted primitive ids and
 * ranges[2*tiles] the [start, end) of every tile. */
int64_t orc_build_lists(int P, const uint8_t *visible, const uint32_t *depth_bits, const int32_t *rect,
                        int W, int H, int32_t *out_ids, int32_t *out_tiles, int32_t *ranges) {
    int TX = (W + TILE - 1) / TILE, TY = (H + TILE - 1) / TILE;
    int64_t cnt = 0;
    for (int p = 0; p < P; p++)
        if (visible[p])
            cnt += (int64_t)(rect[4 * p + 1] / TILE - rect[4 * p + 0] / TILE + 1) *
                   (rect[4 * p + 3] / TILE - rect[4 * p + 2] / TILE + 1);
    if (!out_ids) return cnt;
    entry_t *e = malloc(sizeof(entry_t) * (cnt > 0 ? cnt : 1));
    int64_t i = 0;
    for (int p = 0; p < P; p++) {
        if (!visible[p]) continue;
        for (int ty = rect[4 * p + 2] / TILE; ty <= rect[4 * p + 3] / TILE; ty++)
            for (int tx = rect[4 * p + 0] / TILE; tx <= rect[4 * p + 1] / TILE; tx++) {
                e[i].tile = (uint32_t)(ty * TX + tx); e[i].depth = depth_bits[p]; e[i].id = p; i++;
            }
    }
    qsort(e, cnt, sizeof(entry_t), entry_cmp);
    for (int t = 0; t < TX * TY; t++) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t j = 0; j < cnt; j++) {
        out_ids[j] = e[j].id;
        if (out_tiles) out_tiles[j] = (int32_t)e[j].tile;
        if (j == 0 || e[j].tile != e[j - 1].tile) ranges[2 * e[j].tile] = (int32_t)j;
        if (j == cnt - 1 || e[j].tile != e[j + 1].tile) ranges[2 * e[j].tile + 1] = (int32_t)(j + 1);
    }
    free(e);
    return cnt;
}

/* ================================================================== */
/* Continuous layer, binary64                                           */
/* ================================================================== */

/* Real spherical harmonics up to degree 3, ordered m = -l..l, with the
 * Condon-Shortley phase kept:  m<0: sqrt2 Im Y_l^|m|,  m=0: Y_l^0,
 * m>0: sqrt2 Re Y_l^m, written as polynomials in the unit direction. */
static void sh_basis(int deg, const double *d, double *Y) {
    const double PI = 3.14159265358979323846;
    double x = d[0], y = d[1], z = d[2];
    Y[0] = 0.5 * sqrt(1.0 / PI);
    if (deg < 1) return;
    double c1 = sqrt(3.0 / (4.0 * PI));
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    if (deg < 2) return;
    double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 0.5 * sqrt(15.0 / PI) * x * y;
    Y[5] = -0.5 * sqrt(15.0 / PI) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / PI) * (2.0 * zz - xx - yy);
    Y[7] = -0.5 * sqrt(15.0 / PI) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / PI) * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.125 * sqrt(70.0 / PI) * y * (3.0 * xx - yy);
    Y[10] = 0.5 * sqrt(105.0 / PI) * x * y * z;
    Y[11] = -0.125 * sqrt(42.0 / PI) * y * (4.0 * zz - xx - yy);
    Y[12] = 0.25 * sqrt(7.0 / PI) * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.125 * sqrt(42.0 / PI) * x * (4.0 * zz - xx - yy);
    Y[14] = 0.25 * sqrt(105.0 / PI) * z * (xx - yy);
    Y[15] = -0.125 * sqrt(70.0 / PI) * x * (xx - 3.0 * yy);
}

int orc_sh_basis(int deg, int n, const double *dirs, double *out) {
    int C = (deg + 1) * (deg + 1);
    for (int i = 0; i < n; i++) sh_basis(deg, dirs + 3 * i, out + (int64_t)C * i);
    return 0;
}

static void quat_rot64(const float *qf, double *R) {
    double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* projected mean u and 2x2 screen covariance (xx, xy, yy) in binary64 */
static void project64(const cam_t *k, const float *pf, const float *sf, const float *qf, double *u, double *cov) {
    double p[3] = {pf[0], pf[1], pf[2]}, t[3];
    for (int i = 0; i < 3; i++) t[i] = k->Rd[3 * i] * p[0] + k->Rd[3 * i + 1] * p[1] + k->Rd[3 * i + 2] * p[2] + k->td[i];
    u[0] = (double)k->fx * t[0] / t[2] + k->cx;
    u[1] = (double)k->fy * t[1] / t[2] + k->cy;
    double R[9], S[9];
    quat_rot64(qf, R);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0;
            for (int m = 0; m < 3; m++) a += R[3 * i + m] * ((double)sf[m] * sf[m]) * R[3 * j + m];
            S[3 * i + j] = a;
        }
    double limx = 1.3 * (0.5 * k->W / (double)k->fx), limy = 1.3 * (0.5 * k->H / (double)k->fy);
    double xc = fmin(limx, fmax(-limx, t[0] / t[2])) * t[2];
    double yc = fmin(limy, fmax(-limy, t[1] / t[2])) * t[2];
    double J[6] = {k->fx / t[2], 0, -k->fx * xc / (t[2] * t[2]), 0, k->fy / t[2], -k->fy * yc / (t[2] * t[2])};
    double Mx[6];
    for (int a = 0; a < 2; a++)
        for (int j = 0; j < 3; j++) Mx[3 * a + j] = J[3 * a] * k->Rd[j] + J[3 * a + 1] * k->Rd[3 + j] + J[3 * a + 2] * k->Rd[6 + j];
    double C2[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            double s = 0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) s += Mx[3 * a + i] * S[3 * i + j] * Mx[3 * b + j];
            C2[2 * a + b] = s;
        }
    cov[0] = C2[0]; cov[1] = 0.5 * (C2[1] + C2[2]); cov[2] = C2[3];
}

typedef struct {
    double u[2], con[3]; /* conic of (cov + delta I): power = -0.5(a dx^2 + 2 b dx dy + c dy^2) */
    double col[3], op;
} g64_t;

static void gauss64(const cam_t *k, int g, const float *means, const float *scales, const float *rots,
                    const float *opac, const float *sh, int sh_deg, double delta, g64_t *o) {
    double cov[3];
    project64(k, means + 3 * g, scales + 3 * g, rots + 4 * g, o->u, cov);
    double a = cov[0] + delta, b = cov[1], c = cov[2] + delta;
    double det = a * c - b * b;
    o->con[0] = c / det; o->con[1] = -b / det; o->con[2] = a / det;
    double d[3];
    for (int i = 0; i < 3; i++) d[i] = (double)means[3 * g + i] - k->od[i];
    double nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; i++) d[i] /= nn;
    double Y[16];
    sh_basis(sh_deg, d, Y);
    int C = (sh_deg + 1) * (sh_deg + 1);
    for (int ch = 0; ch < 3; ch++) {
        double s = 0.5;
        for (int j = 0; j < C; j++) s += Y[j] * sh[((int64_t)g * C + j) * 3 + ch];
        o->col[ch] = s > 0 ? s : 0;
    }
    o->op = opac[g];
}

/* v_n = sigmoid of an SH function of the view direction to the cell centre */
static double cell_v64(const cam_t *k, int n, const float *pos, const float *vsh, int vdeg) {
    double d[3];
    for (int i = 0; i < 3; i++) d[i] = (double)pos[3 * n + i] - k->od[i];
    double nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; i++) d[i] /= nn;
    double Y[16];
    sh_basis(vdeg, d, Y);
    int C = (vdeg + 1) * (vdeg + 1);
    double s = 0;
    for (int j = 0; j < C; j++) s += Y[j] * vsh[(int64_t)n * C + j];
    return 1.0 / (1.0 + exp(-s));
}

/* ------------------------------------------------------------------ */
/* per-pixel walks                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    double eps, amin, amax, band_a, band_T, bg[3];
    int no_et;
} ropt_t;

typedef struct {
    int nmarg;       /* marginal decisions seen so far */
    unsigned flip;   /* mask of marginal decisions to flip (by encounter order) */
} dec_t;

/* one thresholded decision "x >= thr" with marginal-band bookkeeping */
static int decide_ge(dec_t *st, double x, double thr, double band) {
    int r = x >= thr;
    if (fabs(x - thr) <= band * thr) {
        if (st->nmarg < 31 && ((st->flip >> st->nmarg) & 1u)) r = !r;
        st->nmarg++;
    }
    return r;
}

typedef struct { double C[3], D, T; int32_t last, nrend, nval; } pix_t;

typedef struct {
    const cam_t *k;
    const g64_t *G;
    const uint8_t *gvis;
    const int32_t *grect;
    const double *v;      /* per cell (duplex) */
    const int32_t *first; /* [N+1]: the members of cell n are Gaussians first[n] .. first[n+1]-1 */
    const int32_t *ids;
    const int32_t *ranges;
    ropt_t o;
} ctx_t;

static int in_rect(const int32_t *r, int px, int py) {
    return px >= r[0] && px <= r[1] && py >= r[2] && py <= r[3];
}

/* Duplex walk over the tile list of pixel (px, py). */
static void walk_duplex(const ctx_t *c, int px, int py, dec_t *st, int no_et, pix_t *out) {
    int tile = (py / TILE) * c->k->TX + (px / TILE);
    int s = c->ranges[2 * tile], e = c->ranges[2 * tile + 1];
    double qx = px + 0.5, qy = py + 0.5;
    double T = 1.0, N[3] = {0, 0, 0}, D = 0.0;
    int32_t last = 0, nrend = 0;
    for (int i = s; i < e; i++) {
        if (!no_et && !decide_ge(st, T, c->o.eps, c->o.band_T)) break; /* cell-level ET */
        int n = c->ids[i];
        double v = c->v[n];
        double A[3] = {0, 0, 0}, B = 0.0, P = 1.0;
        int cnt = 0;
        for (int g = c->first[n]; g < c->first[n + 1]; g++) {
            if (!c->gvis[g] || !in_rect(c->grect + 4 * g, px, py)) continue; /* AABB skip */
            const g64_t *G = c->G + g;
            double dx = qx - G->u[0], dy = qy - G->u[1];
            double pw = -0.5 * (G->con[0] * dx * dx + 2.0 * G->con[1] * dx * dy + G->con[2] * dy * dy);
            double alpha = G->op * exp(pw);
            if (alpha > c->o.amax) alpha = c->o.amax;
            if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;
            for (int ch = 0; ch < 3; ch++) A[ch] += alpha * G->col[ch];
            B += alpha;
            P *= 1.0 - v * alpha;
            cnt++;
        }
        for (int ch = 0; ch < 3; ch++) N[ch] += v * T * A[ch];
        D += v * T * B;
        T *= P;
        if (cnt) { last = i - s + 1; nrend += cnt; }
    }
    for (int ch = 0; ch < 3; ch++) out->C[ch] = D > 0 ? N[ch] / D : c->o.bg[ch];
    out->D = D; out->T = T; out->last = last; out->nrend = nrend;
}

/* "w/o T^cell" ablation (Sec. VII, cell-level transmittance): the pipeline of
 * the Duplex walk with the cell transmittance replaced by the LC-WSR weight
 * (eqs. WSR and LC-WSR, background weight 0): c->v[n] already holds
 * w_n = v_n max(0, 1 - d_n / tau), and the colour is
 *   C = sum_n w_n sum_i alpha_i c_i / sum_n w_n sum_i alpha_i.
 * Nothing decays along the list, so nothing terminates. */
static void walk_lcwsr(const ctx_t *c, int px, int py, dec_t *st, pix_t *out) {
    int tile = (py / TILE) * c->k->TX + (px / TILE);
    int s = c->ranges[2 * tile], e = c->ranges[2 * tile + 1];
    double qx = px + 0.5, qy = py + 0.5;
    double N[3] = {0, 0, 0}, D = 0.0;
    int32_t last = 0, nrend = 0;
    for (int i = s; i < e; i++) {
        int n = c->ids[i];
        double w = c->v[n];
        int cnt = 0;
        for (int g = c->first[n]; g < c->first[n + 1]; g++) {
            if (!c->gvis[g] || !in_rect(c->grect + 4 * g, px, py)) continue;
            const g64_t *G = c->G + g;
            double dx = qx - G->u[0], dy = qy - G->u[1];
            double pw = -0.5 * (G->con[0] * dx * dx + 2.0 * G->con[1] * dx * dy + G->con[2] * dy * dy);
            double alpha = G->op * exp(pw);
            if (alpha > c->o.amax) alpha = c->o.amax;
            if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;
            for (int ch = 0; ch < 3; ch++) N[ch] += w * alpha * G->col[ch];
            D += w * alpha;
            cnt++;
        }
        if (cnt) { last = i - s + 1; nrend += cnt; }
    }
    for (int ch = 0; ch < 3; ch++) out->C[ch] = D > 0 ? N[ch] / D : c->o.bg[ch];
    out->D = D; out->T = 1.0; out->last = last; out->nrend = nrend;
}

/* camera-space depth of a cell centre in binary64 */
static double cell_depth64(const cam_t *k, int n, const float *pos) {
    return k->Rd[6] * pos[3 * n] + k->Rd[7] * pos[3 * n + 1] + k->Rd[8] * pos[3 * n + 2] + k->td[2];
}

/* Per-Gaussian sorted alpha blending over the tile list of pixel (px, py). */
static void walk_alpha(const ctx_t *c, int px, int py, dec_t *st, int no_et, pix_t *out) {
    int tile = (py / TILE) * c->k->TX + (px / TILE);
    int s = c->ranges[2 * tile], e = c->ranges[2 * tile + 1];
    double qx = px + 0.5, qy = py + 0.5;
    double T = 1.0, Cc[3] = {0, 0, 0};
    int32_t last = 0, nrend = 0;
    for (int i = s; i < e; i++) {
        if (!no_et && !decide_ge(st, T, c->o.eps, c->o.band_T)) break;
        int g = c->ids[i];
        if (!in_rect(c->grect + 4 * g, px, py)) continue;
        const g64_t *G = c->G + g;
        double dx = qx - G->u[0], dy = qy - G->u[1];
        double pw = -0.5 * (G->con[0] * dx * dx + 2.0 * G->con[1] * dx * dy + G->con[2] * dy * dy);
        double alpha = G->op * exp(pw);
        if (alpha > c->o.amax) alpha = c->o.amax;
        if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;
        for (int ch = 0; ch < 3; ch++) Cc[ch] += T * alpha * G->col[ch];
        T *= 1.0 - alpha;
        last = i - s + 1; nrend++;
    }
    for (int ch = 0; ch < 3; ch++) out->C[ch] = Cc[ch] + T * c->o.bg[ch];
    out->D = 1.0 - T; out->T = T; out->last = last; out->nrend = nrend;
}

/*
 * Render the requested pixels (pix[2*i] = x, pix[2*i+1] = y; pix == NULL means
 * the whole image in row-major order).
 *   mode 0: Duplex hybrid renderer; mode 1: per-Gaussian alpha blending;
 *   mode 2: the Duplex pipeline with LC-WSR cell weights ("w/o T^cell").
 * Cell n emits the Gaussians offsets[n] .. offsets[n+1]-1 (Sec. IV-A: each
 * cell spawns its own Gaussians), M_in in total; offsets == NULL means K per
 * cell, Gaussians n*K .. n*K+K-1, M = N*K.
 *   ropt[] = eps, alpha_min, alpha_max, delta, kappa, bg0, bg1, bg2,
 *            v_one, no_et, band_alpha, band_T, tau (mode 2)
 * Outputs per pixel: color[3], D, T, last, nrend, nval, status
 * (0 exact, 1 marginal with n_alt admissible alternatives, 2 unverifiable).
 * Alternatives (C[3], D, T per entry, up to 8 per pixel) go to alt[] in
 * slots taken from *alt_count (capacity alt_cap); alt_slot[i] = slot or -1.
 * Returns the total number of (tile, primitive) entries, or -1 on error
 * (offsets not starting at 0, decreasing, or not ending at M_in).
 */
int64_t orc_render(int mode, int N, int K, const int32_t *offsets, int M_in, const float *cell_pos,
                   const float *cell_scale,
                   const float *cell_rot, const float *cell_vsh, int vdeg, const float *means,
                   const float *scales, const float *rots, const float *opac, const float *sh, int sh_deg,
                   const float *camv, const double *ropt, int npix, const int32_t *pix,
                   double *color, double *Dout, double *Tout, int32_t *last, int32_t *nrend, int32_t *nval,
                   int8_t *status, int32_t *n_alt, int32_t *alt_slot, double *alt, int32_t alt_cap,
                   int32_t *alt_count, int32_t *lists_out_len) {
    cam_t k; cam_load(camv, &k);
    /* members of each cell: K per cell in id order, or the CSR offsets */
    int32_t *first = malloc(sizeof(int32_t) * (N + 1));
    for (int n = 0; n <= N; n++) first[n] = offsets ? offsets[n] : n * K;
    int M = offsets ? M_in : N * K;
    if (first[0] != 0 || first[N] != M) { free(first); return -1; }
    for (int n = 0; n < N; n++)
        if (first[n + 1] < first[n]) { free(first); return -1; }
    /* the cell of every Gaussian */
    int32_t *gcell = malloc(sizeof(int32_t) * (M ? M : 1));
    for (int n = 0; n < N; n++)
        for (int g = first[n]; g < first[n + 1]; g++) gcell[g] = n;
    float delta = (float)ropt[3], kappa = (float)ropt[4];
    ctx_t c; memset(&c, 0, sizeof c);
    c.k = &k; c.first = first;
    c.o.eps = ropt[0]; c.o.amin = ropt[1]; c.o.amax = ropt[2];
    c.o.bg[0] = ropt[5]; c.o.bg[1] = ropt[6]; c.o.bg[2] = ropt[7];
    int v_one = (int)ropt[8];
    c.o.no_et = (int)ropt[9];
    c.o.band_a = ropt[10]; c.o.band_T = ropt[11];

    uint8_t *gvis = malloc(M ? M : 1);
    uint32_t *gdep = malloc(sizeof(uint32_t) * (M ? M : 1));
    int32_t *grect = malloc(sizeof(int32_t) * 4 * (M ? M : 1));
    int32_t *gnt = malloc(sizeof(int32_t) * (M ? M : 1));
    orc_gauss_discrete(M, means, scales, rots, opac, camv, delta, gvis, gdep, grect, gnt);

    int ntile = k.TX * k.TY;
    int32_t *ranges = malloc(sizeof(int32_t) * 2 * ntile);
    int32_t *ids = NULL;
    int64_t cnt;
    double *vv = NULL;
    uint8_t *cvis = NULL;
    if (mode == 0 || mode == 2) {
        cvis = malloc(N ? N : 1);
        uint32_t *cdep = malloc(sizeof(uint32_t) * (N ? N : 1));
        int32_t *crect = malloc(sizeof(int32_t) * 4 * (N ? N : 1));
        int32_t *ctr = malloc(sizeof(int32_t) * 4 * (N ? N : 1));
        int32_t *cnt_t = malloc(sizeof(int32_t) * (N ? N : 1));
        orc_cells_discrete(N, cell_pos, cell_scale, cell_rot, camv, kappa, delta, cvis, cdep, crect, ctr, cnt_t);
        cnt = orc_build_lists(N, cvis, cdep, crect, k.W, k.H, NULL, NULL, ranges);
        ids = malloc(sizeof(int32_t) * (cnt > 0 ? cnt : 1));
        orc_build_lists(N, cvis, cdep, crect, k.W, k.H, ids, NULL, ranges);
        vv = malloc(sizeof(double) * (N ? N : 1));
        for (int n = 0; n < N; n++) vv[n] = v_one ? 1.0 : cell_v64(&k, n, cell_pos, cell_vsh, vdeg);
        if (mode == 2) {
            double tau = ropt[12];
            for (int n = 0; n < N; n++) {
                double lin = 1.0 - cell_depth64(&k, n, cell_pos) / tau;
                vv[n] *= lin > 0 ? lin : 0.0;
            }
        }
        free(cdep); free(crect); free(ctr); free(cnt_t);
    } else {
        cnt = orc_build_lists(M, gvis, gdep, grect, k.W, k.H, NULL, NULL, ranges);
        ids = malloc(sizeof(int32_t) * (cnt > 0 ? cnt : 1));
        orc_build_lists(M, gvis, gdep, grect, k.W, k.H, ids, NULL, ranges);
    }
    /* continuous per-Gaussian values; only those that can be reached */
    g64_t *G = calloc(M ? M : 1, sizeof(g64_t));
#pragma omp parallel for schedule(static)
    for (int g = 0; g < M; g++)
        if (gvis[g] && (mode == 1 || cvis[gcell[g]])) gauss64(&k, g, means, scales, rots, opac, sh, sh_deg, delta, &G[g]);
    c.G = G; c.gvis = gvis; c.grect = grect; c.v = vv; c.ids = ids; c.ranges = ranges;

    int total = pix ? npix : k.W * k.H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < total; i++) {
        int px = pix ? pix[2 * i] : i % k.W, py = pix ? pix[2 * i + 1] : i / k.W;
        pix_t r, rv;
        dec_t st = {0, 0};
        if (mode == 0) walk_duplex(&c, px, py, &st, c.o.no_et, &r);
        else if (mode == 2) walk_lcwsr(&c, px, py, &st, &r);
        else walk_alpha(&c, px, py, &st, c.o.no_et, &r);
        /* N^val: gated members of every listed cell, without termination */
        dec_t sv = {0, 0};
        if (mode == 0) walk_duplex(&c, px, py, &sv, 1, &rv);
        else if (mode == 2) walk_lcwsr(&c, px, py, &sv, &rv);
        else walk_alpha(&c, px, py, &sv, 1, &rv);
        for (int ch = 0; ch < 3; ch++) color[3 * i + ch] = r.C[ch];
        Dout[i] = r.D; Tout[i] = r.T; last[i] = r.last; nrend[i] = r.nrend; nval[i] = rv.nrend;
        status[i] = 0; n_alt[i] = 0; alt_slot[i] = -1;
        int m = st.nmarg;
        if (m == 0) continue;
        if (m > 3) { status[i] = 2; continue; }
        int slot;
#pragma omp atomic capture
        slot = (*alt_count)++;
        status[i] = 1;
        if (slot >= alt_cap) { status[i] = 2; continue; }
        alt_slot[i] = slot;
        int na = 0;
        for (unsigned f = 1; f < (1u << m) && na < MAX_ALT; f++) {
            dec_t s2 = {0, f};
            pix_t a;
            if (mode == 0) walk_duplex(&c, px, py, &s2, c.o.no_et, &a);
            else if (mode == 2) walk_lcwsr(&c, px, py, &s2, &a);
            else walk_alpha(&c, px, py, &s2, c.o.no_et, &a);
            double *o = alt + ((int64_t)slot * MAX_ALT + na) * 5;
            o[0] = a.C[0]; o[1] = a.C[1]; o[2] = a.C[2]; o[3] = a.D; o[4] = a.T;
            na++;
        }
        n_alt[i] = na;
    }
    if (lists_out_len) *lists_out_len = (int32_t)cnt;
    free(G); free(gvis); free(gdep); free(grect); free(gnt); free(ranges); free(ids);
    free(vv); free(cvis); free(first); free(gcell);
    return cnt;
}

/* ================================================================== */
/* Neural decode of cells (Sec. III-A neural Gaussians, Sec. IV-A):    */
/* K Gaussians per cell from the cell feature f_n, the viewing distance */
/* delta_n and direction d_n through four MLPs F_sigma, F_c, F_s, F_q.  */
/* ================================================================== */
/*
 * The decoded scales, rotations and centres decide every Gaussian's pixel
 * box (an integer), so they are computed in binary32 in one fixed order that
 * the GPU follows too; opacity and colour only enter the continuous layer
 * and are activated in binary64.
 *
 * Weights: one float array holding, for the decoders d = 0 (opacity, a = 1),
 * 1 (colour, a = 3), 2 (scale ratio, a = 3), 3 (quaternion, a = 4) in this
 * order, W1[(F+4)][H] (input-major), b1[H], W2[H][K a], b2[K a]; output o of
 * decoder d belongs to member o / a, component o % a.
 * Input vector: (f_0 .. f_{F-1}, delta, d_x, d_y, d_z).
 */
static const int DEC_A[4] = {1, 3, 3, 4};

int64_t orc_decoder_size(int F, int H, int K) {
    int64_t n = 0;
    for (int d = 0; d < 4; d++) n += (int64_t)(F + 4) * H + H + (int64_t)H * K * DEC_A[d] + (int64_t)K * DEC_A[d];
    return n;
}

/* exp(x) in binary32 by the Cody-Waite reduction x = n ln2 + r (ln2 split
 * into an 8-significant-bit high part and the rest, so n * ln2_hi is exact)
 * and the degree-7 Taylor polynomial of e^r on |r| <= ln2 / 2, Horner form,
 * one rounding per operation; then scaled by 2^n. */
static float exp32_def(float x) {
    if (x > 88.0f) x = 88.0f;
    if (x < -88.0f) x = -88.0f;
    const float log2e = 1.44269504088896341f;
    const float ln2_hi = 0.693145751953125f, ln2_lo = 1.42860682030941723e-6f;
    float n = rintf(x * log2e);
    float r = (x - n * ln2_hi) - n * ln2_lo;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)n);
}

/* logistic sigmoid in binary32 on exp32_def */
static float sigmoid32_def(float y) { return 1.0f / (1.0f + exp32_def(-y)); }

void orc_exp32(int n, const float *x, float *out) {
    for (int i = 0; i < n; i++) out[i] = exp32_def(x[i]);
}

/* two-layer MLP of decoder d for one input vector, binary32 fixed order:
 * h_j = max(0, b1_j + sum_i x_i W1_ij) and y_o = b2_o + sum_j h_j W2_jo, each
 * sum accumulated by fused multiply-adds in ascending index order */
static void mlp32(const float *w, int I, int H, int O, const float *x, float *h, float *y) {
    const float *W1 = w, *b1 = W1 + (int64_t)I * H, *W2 = b1 + H, *b2 = W2 + (int64_t)H * O;
    for (int j = 0; j < H; j++) {
        float acc = b1[j];
        for (int i = 0; i < I; i++) acc = fmaf(x[i], W1[(int64_t)i * H + j], acc);
        h[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int o = 0; o < O; o++) {
        float acc = b2[o];
        for (int j = 0; j < H; j++) acc = fmaf(h[j], W2[(int64_t)j * O + o], acc);
        y[o] = acc;
    }
}

/*
 * Decode every cell (row-major [N][.] inputs): feat [N][F], offsets O^pos
 * [N*K][3] (components in [-1, 1]).  Outputs per Gaussian: mean, scale and
 * raw quaternion (binary32), opacity sigma = tanh(y) and colour sigmoid(y)
 * (binary64), and the raw decoder outputs y [N][sum K a] when raw != NULL.
 *   centre (eq. scaffold_offset, offsets in the cell frame):
 *       mu = x_n + R(Q_n) (O^pos * S_n)
 *   scale (eqs. nerual_scales, scale_res):
 *       r = max(0, min(sigmoid(y_s), 1 - |O^pos|)),  s = r * S_n
 */
int orc_decode(int N, int K, int F, int H, const float *cell_pos, const float *cell_scale, const float *cell_rot,
               const float *feat, const float *offs, const float *weights, const float *camv, float *means,
               float *scales, float *rots, double *opac, double *color, float *raw) {
    if (F < 1 || H < 1 || K < 1) return -1;
    cam_t k; cam_load(camv, &k);
    float o32[3] = {(float)k.od[0], (float)k.od[1], (float)k.od[2]};
    const int I = F + 4;
    int64_t off[4], ysz = 0, yoff[4];
    {
        int64_t acc = 0;
        for (int d = 0; d < 4; d++) {
            off[d] = acc;
            acc += (int64_t)I * H + H + (int64_t)H * K * DEC_A[d] + (int64_t)K * DEC_A[d];
            yoff[d] = ysz;
            ysz += (int64_t)K * DEC_A[d];
        }
    }
    int err = 0;
#pragma omp parallel
    {
        float *x = malloc(sizeof(float) * I), *h = malloc(sizeof(float) * H), *y = malloc(sizeof(float) * ysz);
        if (!x || !h || !y) err = 1;
#pragma omp for schedule(static)
        for (int n = 0; n < N; n++) {
            if (!x || !h || !y) continue;
            const float *p = cell_pos + 3 * n, *S = cell_scale + 3 * n;
            for (int i = 0; i < F; i++) x[i] = feat[(int64_t)n * F + i];
            float ex = p[0] - o32[0], ey = p[1] - o32[1], ez = p[2] - o32[2];
            float dist = sqrtf((ex * ex + ey * ey) + ez * ez);
            x[F] = dist;
            x[F + 1] = ex / dist; x[F + 2] = ey / dist; x[F + 3] = ez / dist;
            for (int d = 0; d < 4; d++) mlp32(weights + off[d], I, H, K * DEC_A[d], x, h, y + yoff[d]);
            if (raw) memcpy(raw + (int64_t)n * ysz, y, sizeof(float) * ysz);
            float R[9];
            quat_rot32(cell_rot + 4 * n, R);
            for (int kk = 0; kk < K; kk++) {
                int64_t g = (int64_t)n * K + kk;
                const float *O = offs + 3 * g;
                float u[3] = {O[0] * S[0], O[1] * S[1], O[2] * S[2]};
                for (int a = 0; a < 3; a++)
                    means[3 * g + a] = p[a] + ((R[3 * a] * u[0] + R[3 * a + 1] * u[1]) + R[3 * a + 2] * u[2]);
                float lim = 1.0f - sqrtf((O[0] * O[0] + O[1] * O[1]) + O[2] * O[2]);
                for (int a = 0; a < 3; a++) {
                    float r = sigmoid32_def(y[yoff[2] + 3 * kk + a]);
                    r = r < lim ? r : lim;
                    r = r > 0.0f ? r : 0.0f;
                    scales[3 * g + a] = r * S[a];
                }
                for (int a = 0; a < 4; a++) rots[4 * g + a] = y[yoff[3] + 4 * kk + a];
                opac[g] = tanh((double)y[yoff[0] + kk]);
                for (int c = 0; c < 3; c++) color[3 * g + c] = 1.0 / (1.0 + exp(-(double)y[yoff[1] + 3 * kk + c]));
            }
        }
        free(x); free(h); free(y);
    }
    return err ? -1 : 0;
}

/* FP64 continuous quantities of selected Gaussians, for the pins:
 * out[11*i] = u.x, u.y, cov.xx, cov.xy, cov.yy (no dilation), r, g, b,
 * and the conic of the dilated covariance. */
int orc_gauss_continuous(int n, const int32_t *idx, const float *means, const float *scales,
                         const float *rots, const float *opac, const float *sh, int sh_deg,
                         const float *camv, double delta, double *out) {
    cam_t k; cam_load(camv, &k);
    for (int i = 0; i < n; i++) {
        int g = idx[i];
        double u[2], cov[3];
        project64(&k, means + 3 * g, scales + 3 * g, rots + 4 * g, u, cov);
        g64_t G;
        gauss64(&k, g, means, scales, rots, opac, sh, sh_deg, delta, &G);
        double *o = out + 11 * i;
        o[0] = u[0]; o[1] = u[1]; o[2] = cov[0]; o[3] = cov[1]; o[4] = cov[2];
        o[5] = G.col[0]; o[6] = G.col[1]; o[7] = G.col[2];
        o[8] = G.con[0]; o[9] = G.con[1]; o[10] = G.con[2];
    }
    return 0;
}

/* v_n of selected cells (binary64) */
int orc_cell_v(int n, const int32_t *idx, const float *pos, const float *vsh, int vdeg, const float *camv,
               double *out) {
    cam_t k; cam_load(camv, &k);
    for (int i = 0; i < n; i++) out[i] = cell_v64(&k, idx[i], pos, vsh, vdeg);
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads later calls use (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
