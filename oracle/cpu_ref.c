/*
 * Plain FP64 CPU oracle of the accumulated-summation 2-D Gaussian rasteriser, in C with OpenMP.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load or call this library.  It shares no code, header or table with the GPU path.
 *
 * It computes the same functions as the NumPy oracle (oracle/ref.py), written again from the
 * paper, for inputs too large for NumPy loops and for timing on the host cores.  Build:
 *   gcc -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp -shared -fPIC cpu_ref.c -lm
 * -ffp-contract=off matters: the tile rule below must round every float64 operation on its own.
 *
 * Record: (mu_x, mu_y, l1, l2, l3, c0, c1, c2), pixel units, L = [[l1, 0], [l2, l3]],
 * Sigma = L L^T (Sec. 3.1, Eq. cholesky); colour c' weights exp(-sigma) (Sec. 3.2,
 * Eq. rasterization4).  Pixel (x, y) has centre (x + 0.5, y + 0.5) and d = p - mu.  A Gaussian
 * reaches every pixel of the 16x16 tiles its 3-sigma box touches and no other pixel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TILE 16
#define R_MAX 33554432.0 /* 2^25 */

typedef struct {
    double mx, my, l1, l2, l3, c[3];
    double i00, i01, i11; /* Sigma^{-1} */
    int64_t tx0, ty0, tx1, ty1, count;
} gauss_t;

static int is_active(const float *q) {
    for (int k = 0; k < 8; ++k)
        if (!isfinite(q[k])) return 0;
    double l1 = q[2], l2 = q[3], l3 = q[4];
    if (fabs(l1) < 0x1p-24 || fabs(l3) < 0x1p-24) return 0;
    if (fabs(l2) > 0x1p24 || fabs((double)q[0]) > 0x1p24 || fabs((double)q[1]) > 0x1p24) return 0;
    return 1;
}

/* r^2 >= 9 lambda_max(Sigma): with R = r^2, p = R - 9 s00, q = R - 9 s11, both p + q >= 0 and
 * p q >= 81 s01^2.  Fixed order of IEEE float64 operations, no contraction. */
static int covers(double r, double s00, double s01, double s11) {
    double R = r * r;
    double p = R - 9.0 * s00;
    double q = R - 9.0 * s11;
    return ((p + q) >= 0.0) && ((p * q) >= 81.0 * (s01 * s01));
}

/* Least integer r in [0, 2^25] with r >= 3 sqrt(lambda_max), 2^25 if none. */
static double radius(double s00, double s01, double s11) {
    double lam = 0.5 * (s00 + s11) + sqrt(0.25 * (s00 - s11) * (s00 - s11) + s01 * s01);
    double r = ceil(3.0 * sqrt(lam));
    if (!(r >= 0.0)) r = 0.0;
    if (r > R_MAX) r = R_MAX;
    while (r > 0.0 && covers(r - 1.0, s00, s01, s11)) r -= 1.0;
    while (r < R_MAX && !covers(r, s00, s01, s11)) r += 1.0;
    return r;
}

static void form(const float *q, int32_t H, int32_t W, gauss_t *g) {
    memset(g, 0, sizeof(*g));
    g->tx1 = g->ty1 = -1;
    if (!is_active(q)) return;
    g->mx = q[0]; g->my = q[1]; g->l1 = q[2]; g->l2 = q[3]; g->l3 = q[4];
    g->c[0] = q[5]; g->c[1] = q[6]; g->c[2] = q[7];
    double s00 = g->l1 * g->l1, s01 = g->l1 * g->l2, s11 = g->l2 * g->l2 + g->l3 * g->l3;
    double det = (g->l1 * g->l3) * (g->l1 * g->l3);
    g->i00 = s11 / det; g->i01 = -s01 / det; g->i11 = s00 / det;
    double r = radius(s00, s01, s11);
    double tw = (double)((W + TILE - 1) / TILE), th = (double)((H + TILE - 1) / TILE);
    double fx0 = floor((g->mx - r) / TILE), fx1 = floor((g->mx + r) / TILE);
    double fy0 = floor((g->my - r) / TILE), fy1 = floor((g->my + r) / TILE);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > tw - 1.0) fx1 = tw - 1.0;
    if (fy1 > th - 1.0) fy1 = th - 1.0;
    if (fx0 > fx1 || fy0 > fy1) return;
    g->tx0 = (int64_t)fx0; g->ty0 = (int64_t)fy0; g->tx1 = (int64_t)fx1; g->ty1 = (int64_t)fy1;
    g->count = (g->tx1 - g->tx0 + 1) * (g->ty1 - g->ty0 + 1);
}

static gauss_t *form_all(const float *params, int64_t n, int32_t H, int32_t W) {
    gauss_t *g = (gauss_t *)malloc(sizeof(gauss_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) form(params + 8 * i, H, W, g + i);
    return g;
}

/* exp(-sigma) with sigma = 1/2 d^T Sigma^{-1} d (Sec. 3.2, Eq. rasterization2). */
static inline double weight(const gauss_t *g, double px, double py, double *dx, double *dy) {
    *dx = px - g->mx;
    *dy = py - g->my;
    double s = 0.5 * (g->i00 * *dx * *dx + 2.0 * g->i01 * *dx * *dy + g->i11 * *dy * *dy);
    return exp(-s);
}

int64_t or_tile_rects(const float *params, int64_t n, int32_t H, int32_t W, int64_t *rect,
                      int64_t *count) {
    gauss_t *g = form_all(params, n, H, W);
    int64_t K = 0;
    for (int64_t i = 0; i < n; ++i) {
        rect[4 * i + 0] = g[i].count ? g[i].tx0 : 0;
        rect[4 * i + 1] = g[i].count ? g[i].ty0 : 0;
        rect[4 * i + 2] = g[i].count ? g[i].tx1 : -1;
        rect[4 * i + 3] = g[i].count ? g[i].ty1 : -1;
        count[i] = g[i].count;
        K += g[i].count;
    }
    free(g);
    return K;
}

/* Tile lists in CSR form: tile t (row-major) owns ids[start[t] .. start[t+1]), ascending. */
static int64_t build_lists(const gauss_t *g, int64_t n, int64_t T, int64_t tw, int64_t *start,
                           int64_t **ids_out) {
    memset(start, 0, sizeof(int64_t) * (size_t)(T + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t ty = g[i].ty0; ty <= g[i].ty1; ++ty)
            for (int64_t tx = g[i].tx0; tx <= g[i].tx1; ++tx) start[ty * tw + tx + 1]++;
    for (int64_t t = 0; t < T; ++t) start[t + 1] += start[t];
    int64_t K = start[T];
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    memcpy(fill, start, sizeof(int64_t) * (size_t)T);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t ty = g[i].ty0; ty <= g[i].ty1; ++ty)
            for (int64_t tx = g[i].tx0; tx <= g[i].tx1; ++tx) ids[fill[ty * tw + tx]++] = i;
    free(fill);
    *ids_out = ids;
    return K;
}

int64_t or_tile_lists(const float *params, int64_t n, int32_t H, int32_t W, int64_t *ranges,
                      int64_t *ids, int64_t ids_cap) {
    int64_t tw = (W + TILE - 1) / TILE, th = (H + TILE - 1) / TILE, T = tw * th;
    gauss_t *g = form_all(params, n, H, W);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    int64_t *lst = NULL;
    int64_t K = build_lists(g, n, T, tw, start, &lst);
    for (int64_t t = 0; t < T; ++t) {
        ranges[2 * t] = start[t];
        ranges[2 * t + 1] = start[t + 1];
    }
    if (ids && K <= ids_cap) memcpy(ids, lst, sizeof(int64_t) * (size_t)K);
    free(lst); free(start); free(g);
    return K;
}

/* Eq. rasterization4 over the tile support, tile by tile; img/absimg are [H][W][3] float64. */
static void render_lists(const gauss_t *g, const int64_t *start, const int64_t *ids, int32_t H,
                         int32_t W, double *img, double *absimg) {
    int64_t tw = (W + TILE - 1) / TILE, th = (H + TILE - 1) / TILE, T = tw * th;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < T; ++t) {
        int64_t tx = t % tw, ty = t / tw;
        for (int64_t y = ty * TILE; y < (ty + 1) * TILE && y < H; ++y)
            for (int64_t x = tx * TILE; x < (tx + 1) * TILE && x < W; ++x) {
                double acc[3] = {0, 0, 0}, aacc[3] = {0, 0, 0}, dx, dy;
                for (int64_t j = start[t]; j < start[t + 1]; ++j) {
                    const gauss_t *q = g + ids[j];
                    double e = weight(q, x + 0.5, y + 0.5, &dx, &dy);
                    for (int k = 0; k < 3; ++k) {
                        acc[k] += q->c[k] * e;
                        aacc[k] += fabs(q->c[k]) * e;
                    }
                }
                for (int k = 0; k < 3; ++k) {
                    img[(y * W + x) * 3 + k] = acc[k];
                    if (absimg) absimg[(y * W + x) * 3 + k] = aacc[k];
                }
            }
    }
}

void or_render_culled(const float *params, int64_t n, int32_t H, int32_t W, double *img,
                      double *absimg) {
    int64_t tw = (W + TILE - 1) / TILE, th = (H + TILE - 1) / TILE, T = tw * th;
    gauss_t *g = form_all(params, n, H, W);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    int64_t *ids = NULL;
    build_lists(g, n, T, tw, start, &ids);
    render_lists(g, start, ids, H, W, img, absimg);
    free(ids); free(start); free(g);
}

/* Selected pixels only (linear index y*W + x): every Gaussian is tested for tile membership. */
void or_render_pixels(const float *params, int64_t n, int32_t H, int32_t W, const int64_t *pix,
                      int64_t m, double *out, double *absout) {
    gauss_t *g = form_all(params, n, H, W);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t s = 0; s < m; ++s) {
        int64_t x = pix[s] % W, y = pix[s] / W, tx = x / TILE, ty = y / TILE;
        double acc[3] = {0, 0, 0}, aacc[3] = {0, 0, 0}, dx, dy;
        for (int64_t i = 0; i < n; ++i) {
            const gauss_t *q = g + i;
            if (!q->count || tx < q->tx0 || tx > q->tx1 || ty < q->ty0 || ty > q->ty1) continue;
            double e = weight(q, x + 0.5, y + 0.5, &dx, &dy);
            for (int k = 0; k < 3; ++k) {
                acc[k] += q->c[k] * e;
                aacc[k] += fabs(q->c[k]) * e;
            }
        }
        for (int k = 0; k < 3; ++k) {
            out[3 * s + k] = acc[k];
            if (absout) absout[3 * s + k] = aacc[k];
        }
    }
    free(g);
}

/* App. A for one Gaussian over its tile support; writes d[8] and |.| sums absd[8]. */
static void grad_one(const gauss_t *q, int32_t H, int32_t W, const float *G, double *d,
                     double *absd) {
    double acc[8] = {0}, aacc[8] = {0}, dx, dy;
    if (q->count) {
        int64_t x1 = (q->tx1 + 1) * TILE < W ? (q->tx1 + 1) * TILE : W;
        int64_t y1 = (q->ty1 + 1) * TILE < H ? (q->ty1 + 1) * TILE : H;
        for (int64_t y = q->ty0 * TILE; y < y1; ++y)
            for (int64_t x = q->tx0 * TILE; x < x1; ++x) {
                const float *gp = G + (y * W + x) * 3;
                double e = weight(q, x + 0.5, y + 0.5, &dx, &dy);
                double part[8];
                double gc = gp[0] * q->c[0] + gp[1] * q->c[1] + gp[2] * q->c[2];
                double dsig = -e * gc;                      /* dL/dsigma (App. A.1) */
                double vx = q->i00 * dx + q->i01 * dy;      /* Sigma^{-1} d */
                double vy = q->i01 * dx + q->i11 * dy;
                double g1 = dsig * (-0.5 * vx * vx), g2 = dsig * (-0.5 * vx * vy),
                       g3 = dsig * (-0.5 * vy * vy);        /* dL/dSigma */
                part[0] = -dsig * vx;                       /* dsigma/dmu = -Sigma^{-1} d */
                part[1] = -dsig * vy;
                part[2] = 2.0 * g1 * q->l1 + 2.0 * g2 * q->l2; /* App. A.2 */
                part[3] = 2.0 * g2 * q->l1 + 2.0 * g3 * q->l2;
                part[4] = 2.0 * g3 * q->l3;
                part[5] = gp[0] * e;
                part[6] = gp[1] * e;
                part[7] = gp[2] * e;
                for (int k = 0; k < 8; ++k) {
                    acc[k] += part[k];
                    aacc[k] += fabs(part[k]);
                }
            }
    }
    for (int k = 0; k < 8; ++k) {
        d[k] = acc[k];
        if (absd) absd[k] = aacc[k];
    }
}

void or_grads_culled(const float *params, int64_t n, int32_t H, int32_t W, const float *G,
                     double *d, double *absd) {
    gauss_t *g = form_all(params, n, H, W);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) grad_one(g + i, H, W, G, d + 8 * i, absd ? absd + 8 * i : NULL);
    free(g);
}

void or_grads_subset(const float *params, int64_t n, int32_t H, int32_t W, const float *G,
                     const int64_t *which, int64_t m, double *d, double *absd) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; ++s) {
        gauss_t q;
        (void)n;
        form(params + 8 * which[s], H, W, &q);
        grad_one(&q, H, W, G, d + 8 * s, absd ? absd + 8 * s : NULL);
    }
}

/* One fit step: render (culled), L2 loss (Sec. 3.4) with dL/dC = 2 (C - T) / (3 H W),
 * gradients (App. A), Adam with bias correction and the |l1|, |l3| >= l_min floor.
 * hp = {lr_mu, lr_l, lr_c, beta1, beta2, eps, l_min}.  params_in float32; params_out, m, v
 * float64 (m, v read and written).  Returns the loss before the update. */
double or_fit_step(const float *params_in, double *params_out, double *m, double *v,
                   const float *target, int64_t n, int32_t H, int32_t W, const double *hp,
                   int64_t step, double *image_out) {
    int64_t tw = (W + TILE - 1) / TILE, th = (H + TILE - 1) / TILE, T = tw * th;
    int64_t npx = (int64_t)H * W;
    gauss_t *g = form_all(params_in, n, H, W);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    int64_t *ids = NULL;
    build_lists(g, n, T, tw, start, &ids);
    double *img = image_out ? image_out : (double *)malloc(sizeof(double) * (size_t)npx * 3);
    render_lists(g, start, ids, H, W, img, NULL);
    double *Gd = (double *)malloc(sizeof(double) * (size_t)npx * 3);
    double loss = 0.0;
    for (int64_t i = 0; i < npx * 3; ++i) {
        double r = img[i] - (double)target[i];
        loss += r * r;
        Gd[i] = 2.0 * r / (double)(npx * 3);
    }
    loss /= (double)(npx * 3);
    double *dp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 8);
    /* same as grad_one, with the float64 dL/dC of the loss */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        const gauss_t *q = g + i;
        double acc[8] = {0}, dx, dy;
        if (q->count) {
            int64_t x1 = (q->tx1 + 1) * TILE < W ? (q->tx1 + 1) * TILE : W;
            int64_t y1 = (q->ty1 + 1) * TILE < H ? (q->ty1 + 1) * TILE : H;
            for (int64_t y = q->ty0 * TILE; y < y1; ++y)
                for (int64_t x = q->tx0 * TILE; x < x1; ++x) {
                    const double *gp = Gd + (y * W + x) * 3;
                    double e = weight(q, x + 0.5, y + 0.5, &dx, &dy);
                    double gc = gp[0] * q->c[0] + gp[1] * q->c[1] + gp[2] * q->c[2];
                    double dsig = -e * gc;
                    double vx = q->i00 * dx + q->i01 * dy, vy = q->i01 * dx + q->i11 * dy;
                    double g1 = dsig * (-0.5 * vx * vx), g2 = dsig * (-0.5 * vx * vy),
                           g3 = dsig * (-0.5 * vy * vy);
                    acc[0] += -dsig * vx;
                    acc[1] += -dsig * vy;
                    acc[2] += 2.0 * g1 * q->l1 + 2.0 * g2 * q->l2;
                    acc[3] += 2.0 * g2 * q->l1 + 2.0 * g3 * q->l2;
                    acc[4] += 2.0 * g3 * q->l3;
                    acc[5] += gp[0] * e;
                    acc[6] += gp[1] * e;
                    acc[7] += gp[2] * e;
                }
        }
        for (int k = 0; k < 8; ++k) dp[8 * i + k] = acc[k];
    }
    double b1 = hp[3], b2 = hp[4], eps = hp[5], lmin = hp[6];
    double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 8; ++k) {
            double lr = k < 2 ? hp[0] : (k < 5 ? hp[1] : hp[2]);
            double gr = dp[8 * i + k];
            double mm = b1 * m[8 * i + k] + (1.0 - b1) * gr;
            double vv = b2 * v[8 * i + k] + (1.0 - b2) * gr * gr;
            m[8 * i + k] = mm;
            v[8 * i + k] = vv;
            double p = (double)params_in[8 * i + k] - lr * (mm / bc1) / (sqrt(vv / bc2) + eps);
            if ((k == 2 || k == 4) && lmin > 0.0 && fabs(p) < lmin) p = copysign(lmin, p);
            params_out[8 * i + k] = p;
        }
    free(Gd); free(dp);
    if (!image_out) free(img);
    free(ids); free(start); free(g);
    return loss;
}

int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
