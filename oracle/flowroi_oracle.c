/*
 * FlowRoI flow -> RoI-mask hot path: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library. The product path
 * (the HIP library) shares no code with it and never calls it.
 *
 * What it computes (FlowRoI, Method: "Optical flow extraction" and "Region of
 * Interest extraction"): dense two-frame Farneback optical flow between a
 * frame pair, the flow magnitude compared with a threshold, and a binary
 * dilation of the result into the RoI mask. The paper names the Farneback
 * estimator but fixes none of its constants; the estimator is the two-frame
 * polynomial-expansion method (G. Farneback, "Two-Frame Motion Estimation
 * Based on Polynomial Expansion", SCIA 2003):
 *
 *   - every frame is fitted locally by f(x) ~ x^T A x + b^T x + c in the
 *     weighted least-squares sense (Gaussian applicability);
 *   - a displacement d turns b into b - 2 A d, so each pixel gives a linear
 *     equation A d = db; the equations are pooled over a window and solved;
 *   - a coarse-to-fine pyramid and a few iterations with the previous
 *     estimate as prior displacement make it work for large motion.
 *
 * Conventions (readings where the paper is silent):
 *   - images are row-major h x w; x is the column, y the row;
 *   - flow is interleaved (dx, dy) per pixel and points from prev to next:
 *     next(x + d) ~ prev(x);
 *   - every stencil and every warp replicates the border pixel;
 *   - pyramid level l+1 = 5x5 binomial ([1 4 6 4 1]/16 in each axis) blur of
 *     level l, sampled at the even pixels; size ceil(n / 2);
 *   - the pooled 2x2 system G d = h is regularised as
 *     d = adj(G) h / max(det G, eps * (tr G)^2), and d = 0 where tr G = 0;
 *   - the mask is [|d| > tau] (strict), dilated with a square or disc of
 *     radius r, pixels outside the image counting as 0.
 *
 * Everything is computed in double, directly from the definitions, with no
 * blocking, running sums or reordering. OpenMP (if enabled) only splits the
 * outer row loops; it does not change any arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Pyramid                                                                   */
/* ------------------------------------------------------------------------ */

/* One pyramid step: dst(i, j) = sum_{u,v} k(u) k(v) src(2i + u, 2j + v) with
 * k = [1 4 6 4 1] / 16 (binomial, Burt-Adelson), replicate border.
 * dst is ceil(h/2) x ceil(w/2). */
void orc_pyr_down(const double *src, int h, int w, double *dst)
{
    static const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h2; ++i)
        for (int j = 0; j < w2; ++j) {
            double acc = 0.0;
            for (int u = -2; u <= 2; ++u)
                for (int v = -2; v <= 2; ++v) {
                    const int yy = clampi(2 * i + u, 0, h - 1);
                    const int xx = clampi(2 * j + v, 0, w - 1);
                    acc += k[u + 2] * k[v + 2] * src[(size_t)yy * w + xx];
                }
            dst[(size_t)i * w2 + j] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Polynomial expansion (Farneback 2003, section 2)                          */
/* ------------------------------------------------------------------------ */

/* Invert an n x n matrix (row-major) by Gauss-Jordan elimination with partial
 * pivoting. Returns 0 on success, -1 if singular. */
static int invert(double *m, double *inv, int n)
{
    double a[6][12];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            a[i][j] = j < n ? m[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
        if (a[p][c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = a[p][j];
                a[p][j] = a[c][j];
                a[c][j] = t;
            }
        const double piv = a[c][c];
        for (int j = 0; j < 2 * n; ++j) a[c][j] /= piv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) inv[i * n + j] = a[i][n + j];
    return 0;
}

/* Basis of the local quadratic model at offset (x = column, y = row):
 * {1, x, y, x^2, y^2, x y}. */
static void basis(double x, double y, double *b)
{
    b[0] = 1.0;
    b[1] = x;
    b[2] = y;
    b[3] = x * x;
    b[4] = y * y;
    b[5] = x * y;
}

/* Weighted least-squares fit of the quadratic model over the (2n+1)^2
 * neighbourhood of every pixel, applicability a(u, v) = g(u) g(v) with
 * g(t) = exp(-t^2 / (2 sigma^2)), replicate border.
 *
 * out holds 5 planes of h*w doubles, in this order:
 *   [0] rx  = b_x      [1] ry = b_y
 *   [2] rxx = A_xx     [3] ryy = A_yy     [4] rxy = coefficient of x*y,
 * so that A = [[rxx, rxy/2], [rxy/2, ryy]] and b = (rx, ry).
 * The constant term c is not kept (nothing downstream uses it). */
int orc_poly_expand(const double *img, int h, int w, int n, double sigma, double *out)
{
    if (n < 1 || n > 8 || !(sigma > 0)) return ORC_EINVAL;
    const int side = 2 * n + 1;
    double *wgt = (double *)malloc(sizeof(double) * side * side);
    if (!wgt) return ORC_ENOMEM;
    double gram[36] = {0}, ginv[36];
    for (int u = -n; u <= n; ++u)
        for (int v = -n; v <= n; ++v) {
            const double a = exp(-(double)(u * u) / (2 * sigma * sigma)) *
                             exp(-(double)(v * v) / (2 * sigma * sigma));
            wgt[(u + n) * side + (v + n)] = a;
            double b[6];
            basis((double)v, (double)u, b); /* u = row offset (y), v = column offset (x) */
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 6; ++c) gram[r * 6 + c] += a * b[r] * b[c];
        }
    if (invert(gram, ginv, 6) != 0) {
        free(wgt);
        return ORC_EINVAL;
    }
    const size_t plane = (size_t)h * w;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            double rhs[6] = {0};
            for (int u = -n; u <= n; ++u)
                for (int v = -n; v <= n; ++v) {
                    const double f = img[(size_t)clampi(i + u, 0, h - 1) * w + clampi(j + v, 0, w - 1)];
                    const double a = wgt[(u + n) * side + (v + n)];
                    double b[6];
                    basis((double)v, (double)u, b);
                    for (int r = 0; r < 6; ++r) rhs[r] += a * b[r] * f;
                }
            double coef[6];
            for (int r = 0; r < 6; ++r) {
                double s = 0.0;
                for (int c = 0; c < 6; ++c) s += ginv[r * 6 + c] * rhs[c];
                coef[r] = s;
            }
            const size_t p = (size_t)i * w + j;
            out[0 * plane + p] = coef[1];
            out[1 * plane + p] = coef[2];
            out[2 * plane + p] = coef[3];
            out[3 * plane + p] = coef[4];
            out[4 * plane + p] = coef[5];
        }
    free(wgt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sampling                                                                  */
/* ------------------------------------------------------------------------ */

/* Bilinear sample of an h x w plane at (x, y) = (column, row), the point
 * first clamped to [0, w-1] x [0, h-1]. */
double orc_bilinear(const double *p, int h, int w, double x, double y)
{
    if (x < 0) x = 0;
    if (x > w - 1) x = w - 1;
    if (y < 0) y = 0;
    if (y > h - 1) y = h - 1;
    const int x0 = (int)floor(x), y0 = (int)floor(y);
    const int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
    const double fx = x - x0, fy = y - y0;
    const double p00 = p[(size_t)y0 * w + x0], p01 = p[(size_t)y0 * w + x1];
    const double p10 = p[(size_t)y1 * w + x0], p11 = p[(size_t)y1 * w + x1];
    return (1 - fy) * ((1 - fx) * p00 + fx * p01) + fy * ((1 - fx) * p10 + fx * p11);
}

/* Flow of pyramid level l from level l+1 (hc x wc): pixel (i, j) of the finer
 * level sits at (j/2, i/2) on the coarser grid (the coarse grid keeps the
 * even fine pixels); displacements double. */
void orc_flow_upsample(const double *coarse, int hc, int wc, double *fine, int h, int w)
{
    const size_t pc = (size_t)hc * wc;
    double *cx = (double *)malloc(sizeof(double) * pc), *cy = (double *)malloc(sizeof(double) * pc);
    for (size_t q = 0; q < pc; ++q) {
        cx[q] = coarse[2 * q];
        cy[q] = coarse[2 * q + 1];
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            const size_t p = (size_t)i * w + j;
            fine[2 * p] = 2.0 * orc_bilinear(cx, hc, wc, j / 2.0, i / 2.0);
            fine[2 * p + 1] = 2.0 * orc_bilinear(cy, hc, wc, j / 2.0, i / 2.0);
        }
    free(cx);
    free(cy);
}

/* ------------------------------------------------------------------------ */
/* One displacement update (Farneback 2003, sections 3-4)                    */
/* ------------------------------------------------------------------------ */

/* Per-pixel normal-equation terms for the current prior flow.
 * r1, r2: expansions (5 planes, layout of orc_poly_expand) of prev and next.
 * flow:   prior displacement d~ (interleaved dx, dy).
 * gh:     5 output planes G11, G12, G22, h1, h2 with G = A^T A, h = A^T db,
 *         A  = (A1(x) + A2(x + d~)) / 2,
 *         db = -(b2(x + d~) - b1(x)) / 2 + A d~,
 *         next's coefficients sampled bilinearly at x + d~. */
void orc_update_terms(const double *r1, const double *r2, const double *flow, int h, int w, double *gh)
{
    const size_t plane = (size_t)h * w;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            const size_t p = (size_t)i * w + j;
            const double dx = flow[2 * p], dy = flow[2 * p + 1];
            const double xs = j + dx, ys = i + dy;
            double c2[5];
            for (int k = 0; k < 5; ++k) c2[k] = orc_bilinear(r2 + k * plane, h, w, xs, ys);
            const double A1[2][2] = {{r1[2 * plane + p], r1[4 * plane + p] / 2},
                                     {r1[4 * plane + p] / 2, r1[3 * plane + p]}};
            const double A2[2][2] = {{c2[2], c2[4] / 2}, {c2[4] / 2, c2[3]}};
            const double b1[2] = {r1[0 * plane + p], r1[1 * plane + p]};
            const double b2[2] = {c2[0], c2[1]};
            const double dt[2] = {dx, dy};
            double A[2][2], db[2];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) A[r][c] = 0.5 * (A1[r][c] + A2[r][c]);
            for (int r = 0; r < 2; ++r) db[r] = -0.5 * (b2[r] - b1[r]) + A[r][0] * dt[0] + A[r][1] * dt[1];
            double G[2][2], hv[2];
            for (int r = 0; r < 2; ++r) {
                for (int c = 0; c < 2; ++c) G[r][c] = A[0][r] * A[0][c] + A[1][r] * A[1][c];
                hv[r] = A[0][r] * db[0] + A[1][r] * db[1];
            }
            gh[0 * plane + p] = G[0][0];
            gh[1 * plane + p] = G[0][1];
            gh[2 * plane + p] = G[1][1];
            gh[3 * plane + p] = hv[0];
            gh[4 * plane + p] = hv[1];
        }
}

/* Window aggregation: out(i, j) = sum over the winsize x winsize square
 * centred on (i, j) of in, replicate border. nplanes planes of h*w. */
void orc_box_sum(const double *in, int nplanes, int h, int w, int winsize, double *out)
{
    const int r = winsize / 2;
    const size_t plane = (size_t)h * w;
    for (int k = 0; k < nplanes; ++k) {
        const double *src = in + k * plane;
        double *dst = out + k * plane;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j) {
                double s = 0.0;
                for (int u = -r; u <= r; ++u)
                    for (int v = -r; v <= r; ++v)
                        s += src[(size_t)clampi(i + u, 0, h - 1) * w + clampi(j + v, 0, w - 1)];
                dst[(size_t)i * w + j] = s;
            }
    }
}

/* Regularised 2x2 solve of the pooled system at every pixel.
 * gh: 5 planes G11, G12, G22, h1, h2 (already window-summed). */
void orc_solve(const double *gh, int h, int w, double eps, double *flow)
{
    const size_t plane = (size_t)h * w;
    for (size_t p = 0; p < plane; ++p) {
        const double g11 = gh[p], g12 = gh[plane + p], g22 = gh[2 * plane + p];
        const double h1 = gh[3 * plane + p], h2 = gh[4 * plane + p];
        const double tr = g11 + g22;
        if (tr == 0.0) {
            flow[2 * p] = 0.0;
            flow[2 * p + 1] = 0.0;
            continue;
        }
        const double det = g11 * g22 - g12 * g12;
        const double den = det > eps * tr * tr ? det : eps * tr * tr;
        /* adj(G) = [[g22, -g12], [-g12, g11]] */
        flow[2 * p] = (g22 * h1 - g12 * h2) / den;
        flow[2 * p + 1] = (g11 * h2 - g12 * h1) / den;
    }
}

/* ------------------------------------------------------------------------ */
/* Coarse-to-fine flow                                                       */
/* ------------------------------------------------------------------------ */

static int level_dim(int n, int l)
{
    for (int k = 0; k < l; ++k) n = (n + 1) / 2;
    return n;
}

/* Dense flow prev -> next.
 * init (nullable): initial flow at full resolution; at the coarsest level L-1
 * pixel (i, j) takes init at (min(2^(L-1) i, h-1), min(2^(L-1) j, w-1))
 * divided by 2^(L-1). Without init the coarsest level starts at zero.
 * flow: h*w*2 output. */
int orc_flow(const double *prev, const double *next, int h, int w, int levels, int winsize,
             int iterations, int poly_n, double poly_sigma, double eps, const double *init, double *flow)
{
    if (levels < 1 || levels > 16 || winsize < 1 || (winsize % 2) == 0 || iterations < 1) return ORC_EINVAL;
    double *pyr1[16] = {0}, *pyr2[16] = {0}, *r1[16] = {0}, *r2[16] = {0};
    int hh[16], ww[16];
    int rc = ORC_OK;
    for (int l = 0; l < levels; ++l) {
        hh[l] = level_dim(h, l);
        ww[l] = level_dim(w, l);
        const size_t pl = (size_t)hh[l] * ww[l];
        pyr1[l] = (double *)malloc(sizeof(double) * pl);
        pyr2[l] = (double *)malloc(sizeof(double) * pl);
        r1[l] = (double *)malloc(sizeof(double) * pl * 5);
        r2[l] = (double *)malloc(sizeof(double) * pl * 5);
        if (!pyr1[l] || !pyr2[l] || !r1[l] || !r2[l]) {
            rc = ORC_ENOMEM;
            goto done;
        }
    }
    memcpy(pyr1[0], prev, sizeof(double) * (size_t)h * w);
    memcpy(pyr2[0], next, sizeof(double) * (size_t)h * w);
    for (int l = 1; l < levels; ++l) {
        orc_pyr_down(pyr1[l - 1], hh[l - 1], ww[l - 1], pyr1[l]);
        orc_pyr_down(pyr2[l - 1], hh[l - 1], ww[l - 1], pyr2[l]);
    }
    for (int l = 0; l < levels; ++l) {
        if ((rc = orc_poly_expand(pyr1[l], hh[l], ww[l], poly_n / 2, poly_sigma, r1[l])) != ORC_OK) goto done;
        if ((rc = orc_poly_expand(pyr2[l], hh[l], ww[l], poly_n / 2, poly_sigma, r2[l])) != ORC_OK) goto done;
    }
    {
        double *cur = NULL;
        int hc = 0, wc = 0;
        for (int l = levels - 1; l >= 0; --l) {
            const int H = hh[l], W = ww[l];
            const size_t pl = (size_t)H * W;
            double *d = (double *)calloc(pl * 2, sizeof(double));
            double *gh = (double *)malloc(sizeof(double) * pl * 5);
            double *ghs = (double *)malloc(sizeof(double) * pl * 5);
            if (!d || !gh || !ghs) {
                free(d);
                free(gh);
                free(ghs);
                free(cur);
                rc = ORC_ENOMEM;
                goto done;
            }
            if (l == levels - 1) {
                if (init) {
                    const int s = 1 << l;
                    for (int i = 0; i < H; ++i)
                        for (int j = 0; j < W; ++j) {
                            const size_t q = (size_t)clampi(s * i, 0, h - 1) * w + clampi(s * j, 0, w - 1);
                            d[2 * ((size_t)i * W + j)] = init[2 * q] / s;
                            d[2 * ((size_t)i * W + j) + 1] = init[2 * q + 1] / s;
                        }
                }
            } else {
                orc_flow_upsample(cur, hc, wc, d, H, W);
            }
            for (int it = 0; it < iterations; ++it) {
                orc_update_terms(r1[l], r2[l], d, H, W, gh);
                orc_box_sum(gh, 5, H, W, winsize, ghs);
                orc_solve(ghs, H, W, eps, d);
            }
            free(gh);
            free(ghs);
            free(cur);
            cur = d;
            hc = H;
            wc = W;
        }
        memcpy(flow, cur, sizeof(double) * 2 * (size_t)h * w);
        free(cur);
    }
done:
    for (int l = 0; l < levels; ++l) {
        free(pyr1[l]);
        free(pyr2[l]);
        free(r1[l]);
        free(r2[l]);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Threshold and dilation                                                    */
/* ------------------------------------------------------------------------ */

/* Squared magnitude dx^2 + dy^2 of n flow vectors. */
void orc_magnitude2(const double *flow, size_t n, double *m2)
{
    for (size_t p = 0; p < n; ++p) m2[p] = flow[2 * p] * flow[2 * p] + flow[2 * p + 1] * flow[2 * p + 1];
}

/* Absolute threshold: pre = [|d| > tau], tested as |d|^2 > tau^2. */
void orc_threshold_abs(const double *flow, size_t n, double tau, uint8_t *pre)
{
    for (size_t p = 0; p < n; ++p) {
        const double m2 = flow[2 * p] * flow[2 * p] + flow[2 * p + 1] * flow[2 * p + 1];
        pre[p] = m2 > tau * tau ? 1 : 0;
    }
}

static int cmp_desc(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Quantile threshold ("RoI threshold" q in (0, 1): keep the top q fraction).
 * k = floor(q n); tau^2 = the (k+1)-th largest |d|^2; pre = [|d|^2 > tau^2].
 * At most k pixels are kept, fewer where values tie at tau^2.
 * Returns tau^2 through *tau2. */
int orc_threshold_top(const double *flow, size_t n, double q, uint8_t *pre, double *tau2)
{
    if (!(q > 0 && q < 1) || n == 0) return ORC_EINVAL;
    double *m2 = (double *)malloc(sizeof(double) * n), *srt = (double *)malloc(sizeof(double) * n);
    if (!m2 || !srt) {
        free(m2);
        free(srt);
        return ORC_ENOMEM;
    }
    orc_magnitude2(flow, n, m2);
    memcpy(srt, m2, sizeof(double) * n);
    qsort(srt, n, sizeof(double), cmp_desc);
    const size_t k = (size_t)floor(q * (double)n);
    const double t = srt[k];
    for (size_t p = 0; p < n; ++p) pre[p] = m2[p] > t ? 1 : 0;
    if (tau2) *tau2 = t;
    free(m2);
    free(srt);
    return ORC_OK;
}

/* Binary dilation: mask(i, j) = OR over offsets (u, v) of the structuring
 * element of pre(i + u, j + v), pixels outside the image counting as 0.
 * shape 0: square |u|, |v| <= r; shape 1: disc u^2 + v^2 <= r^2. */
int orc_dilate(const uint8_t *pre, int h, int w, int r, int shape, uint8_t *mask)
{
    if (r < 0 || (shape != 0 && shape != 1)) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            uint8_t m = 0;
            for (int u = -r; u <= r && !m; ++u)
                for (int v = -r; v <= r && !m; ++v) {
                    if (shape == 1 && u * u + v * v > r * r) continue;
                    const int yy = i + u, xx = j + v;
                    if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
                    if (pre[(size_t)yy * w + xx]) m = 1;
                }
            mask[(size_t)i * w + j] = m;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Denoising pre-stage (FlowRoI Method, Optical flow extraction: median then  */
/* bilateral filtering before the flow)                                      */
/* ------------------------------------------------------------------------ */

static int cmp_asc(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Median over the (2 mr + 1)^2 square around each pixel, replicate border. */
void orc_median(const double *img, int h, int w, int mr, double *out)
{
    const int side = 2 * mr + 1, n = side * side;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i) {
        double buf[81];
        for (int j = 0; j < w; ++j) {
            int k = 0;
            for (int u = -mr; u <= mr; ++u)
                for (int v = -mr; v <= mr; ++v) buf[k++] = img[(size_t)clampi(i + u, 0, h - 1) * w + clampi(j + v, 0, w - 1)];
            qsort(buf, n, sizeof(double), cmp_asc);
            out[(size_t)i * w + j] = buf[n / 2];
        }
    }
}

/* Bilateral filter over the (2 br + 1)^2 square, replicate border:
 * out(p) = sum_q ws(q - p) wr(I(q) - I(p)) I(q) / sum_q ws wr with
 * ws(t) = exp(-|t|^2 / (2 ss^2)) and wr(e) = exp(-e^2 / (2 sr^2)). */
void orc_bilateral(const double *img, int h, int w, int br, double ss, double sr, double *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            const double c = img[(size_t)i * w + j];
            double num = 0.0, den = 0.0;
            for (int u = -br; u <= br; ++u)
                for (int v = -br; v <= br; ++v) {
                    const double q = img[(size_t)clampi(i + u, 0, h - 1) * w + clampi(j + v, 0, w - 1)];
                    const double wt = exp(-(double)(u * u + v * v) / (2 * ss * ss)) * exp(-(q - c) * (q - c) / (2 * sr * sr));
                    num += wt * q;
                    den += wt;
                }
            out[(size_t)i * w + j] = num / den;
        }
}

/* Median (radius mr, skipped when 0) then bilateral (radius br, skipped
 * when 0). */
int orc_denoise(const double *img, int h, int w, int mr, int br, double ss, double sr, double *out)
{
    if (mr < 0 || mr > 4 || br < 0 || (br > 0 && !(ss > 0 && sr > 0))) return ORC_EINVAL;
    const size_t n = (size_t)h * w;
    double *tmp = (double *)malloc(sizeof(double) * n);
    if (!tmp) return ORC_ENOMEM;
    if (mr > 0) orc_median(img, h, w, mr, tmp);
    else memcpy(tmp, img, sizeof(double) * n);
    if (br > 0) orc_bilateral(tmp, h, w, br, ss, sr, out);
    else memcpy(out, tmp, sizeof(double) * n);
    free(tmp);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The paper's RoI rule (Region of Interest extraction): motion saliency from */
/* flow magnitude and its spatial gradient, normalisation, quantile          */
/* threshold, opening and closing, removal of small connected components.    */
/* ------------------------------------------------------------------------ */

/* Saliency: M = |d|; G = |grad M| by central differences with replicated
 * edges; S = wt M / max M + (1 - wt) G / max G (a term whose maximum is 0
 * contributes 0); output S / max S (0 where max S = 0). */
void orc_saliency(const double *flow, int h, int w, double wt, double *sal)
{
    const size_t n = (size_t)h * w;
    double *M = (double *)malloc(sizeof(double) * n), *G = (double *)malloc(sizeof(double) * n);
    double mM = 0.0, mG = 0.0, mS = 0.0;
    for (size_t p = 0; p < n; ++p) {
        M[p] = sqrt(flow[2 * p] * flow[2 * p] + flow[2 * p + 1] * flow[2 * p + 1]);
        if (M[p] > mM) mM = M[p];
    }
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            const double gx = 0.5 * (M[(size_t)i * w + clampi(j + 1, 0, w - 1)] - M[(size_t)i * w + clampi(j - 1, 0, w - 1)]);
            const double gy = 0.5 * (M[(size_t)clampi(i + 1, 0, h - 1) * w + j] - M[(size_t)clampi(i - 1, 0, h - 1) * w + j]);
            G[(size_t)i * w + j] = sqrt(gx * gx + gy * gy);
            if (G[(size_t)i * w + j] > mG) mG = G[(size_t)i * w + j];
        }
    for (size_t p = 0; p < n; ++p) {
        const double a = mM > 0 ? M[p] / mM : 0.0, b = mG > 0 ? G[p] / mG : 0.0;
        sal[p] = wt * a + (1.0 - wt) * b;
        if (sal[p] > mS) mS = sal[p];
    }
    for (size_t p = 0; p < n; ++p) sal[p] = mS > 0 ? sal[p] / mS : 0.0;
    free(M);
    free(G);
}

/* Binary erosion (erode = 1) or dilation (erode = 0) by the (2r+1)^2 square,
 * over the part of the square inside the frame. */
static void morph_square(const uint8_t *in, int h, int w, int r, int erode, uint8_t *out)
{
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            uint8_t v = erode ? 1 : 0;
            for (int u = -r; u <= r; ++u)
                for (int q = -r; q <= r; ++q) {
                    const int y = i + u, x = j + q;
                    if (y < 0 || y >= h || x < 0 || x >= w) continue;
                    if (erode && !in[(size_t)y * w + x]) v = 0;
                    if (!erode && in[(size_t)y * w + x]) v = 1;
                }
            out[(size_t)i * w + j] = v;
        }
}

/* Opening (erode, dilate) then closing (dilate, erode), square of radius r. */
void orc_open_close(const uint8_t *pre, int h, int w, int r, uint8_t *out)
{
    const size_t n = (size_t)h * w;
    uint8_t *a = (uint8_t *)malloc(n), *b = (uint8_t *)malloc(n);
    morph_square(pre, h, w, r, 1, a);
    morph_square(a, h, w, r, 0, b);
    morph_square(b, h, w, r, 0, a);
    morph_square(a, h, w, r, 1, out);
    free(a);
    free(b);
}

/* Keep the 8-connected components of `mask` whose area is >= min_area.
 * Labels by depth-first flood fill. */
void orc_cc_filter(const uint8_t *mask, int h, int w, int min_area, uint8_t *out)
{
    const size_t n = (size_t)h * w;
    int *lab = (int *)malloc(sizeof(int) * n);
    size_t *stack = (size_t *)malloc(sizeof(size_t) * n);
    size_t *members = (size_t *)malloc(sizeof(size_t) * n);
    for (size_t p = 0; p < n; ++p) lab[p] = -1;
    memset(out, 0, n);
    for (size_t s0 = 0; s0 < n; ++s0) {
        if (!mask[s0] || lab[s0] >= 0) continue;
        size_t top = 0, cnt = 0;
        stack[top++] = s0;
        lab[s0] = 1;
        while (top) {
            const size_t p = stack[--top];
            members[cnt++] = p;
            const int i = (int)(p / w), j = (int)(p % w);
            for (int u = -1; u <= 1; ++u)
                for (int v = -1; v <= 1; ++v) {
                    const int y = i + u, x = j + v;
                    if (y < 0 || y >= h || x < 0 || x >= w) continue;
                    const size_t q = (size_t)y * w + x;
                    if (mask[q] && lab[q] < 0) {
                        lab[q] = 1;
                        stack[top++] = q;
                    }
                }
        }
        if ((int64_t)cnt >= min_area)
            for (size_t k = 0; k < cnt; ++k) out[members[k]] = 1;
    }
    free(lab);
    free(stack);
    free(members);
}

/* ------------------------------------------------------------------------ */
/* Whole path                                                                */
/* ------------------------------------------------------------------------ */

/* flow (h*w*2) and mask (h*w) from a frame pair given as doubles.
 * thresh_mode 0: |d| > thresh (pixels); 1: top-`thresh` fraction.
 * tau2_out (nullable) receives the squared threshold actually used. */
int orc_roi_mask(const double *prev, const double *next, int h, int w, int levels, int winsize,
                 int iterations, int poly_n, double poly_sigma, double eps, const double *init,
                 int thresh_mode, double thresh, int dilate_radius, int se_shape, double *flow,
                 uint8_t *mask, double *tau2_out)
{
    int rc = orc_flow(prev, next, h, w, levels, winsize, iterations, poly_n, poly_sigma, eps, init, flow);
    if (rc != ORC_OK) return rc;
    const size_t n = (size_t)h * w;
    uint8_t *pre = (uint8_t *)malloc(n);
    if (!pre) return ORC_ENOMEM;
    if (thresh_mode == 0) {
        orc_threshold_abs(flow, n, thresh, pre);
        if (tau2_out) *tau2_out = thresh * thresh;
    } else if (thresh_mode == 1) {
        rc = orc_threshold_top(flow, n, thresh, pre, tau2_out);
    } else {
        rc = ORC_EINVAL;
    }
    if (rc == ORC_OK) rc = orc_dilate(pre, h, w, dilate_radius, se_shape, mask);
    free(pre);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
