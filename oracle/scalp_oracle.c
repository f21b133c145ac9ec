/*
 * scalp_oracle.c -- plain CPU oracle for the SCALP clustering path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path
 * (the HIP library) never calls, links or includes anything from here, and
 * this file includes nothing from the product path.
 *
 * What it computes, following the paper
 *   "SCALP: Superpixels with Contour Adherence using Linear Path"
 *   (Giraud, Ta, Papadakis; ICPR 2018, arXiv 1903.07149):
 *
 *   grid            Sec. II-A: regular grid of blocks of side r = sqrt(N/k).
 *   w map           Eq. (2): summand 1 - exp(-C(q)^2 / sigma^2).
 *   linear path     Sec. II-B: the Bresenham pixels from p to the barycenter.
 *   distance D      Eqs. (1)-(3): path colour distance x contour weight
 *                   + spatial distance * m^2 / r^2.
 *   assignment      Algorithm 1 (SCALP method), the inner loops: keep the
 *                   strictly smaller D.
 *   update          Algorithm 1, cluster update: mean Lab and mean position.
 *   projection      Sec. II-D Remark, Eq. (4): when the rounded barycenter is
 *                   not in its superpixel, use the nearest member pixel.
 *   soft mode       an extension, not in the paper: softmax over the same
 *                   distances, soft barycenters, and the exact FP64 gradient.
 *
 * Readings taken where the paper is silent (each is listed with its reason
 * in the design notes of the repository):
 *   - grid:  nx = max(1, lround(W/r)), ny = max(1, lround(H/r)); the cell of
 *            pixel (x, y) is (floor(y*ny/H), floor(x*nx/W)); r uses the
 *            requested k.
 *   - candidates: the 3x3 grid-neighbour cells of the pixel's own cell, in
 *            row-major order (ascending k); strict '<' keeps the first of
 *            equal distances, as in Algorithm 1 with k ascending.
 *   - path:  q_i = p + sgn(d) * floor((2 i |d| + n) / (2 n)) per axis,
 *            i = 0..n, n = max(|dx|, |dy|), from p to the rounded barycenter
 *            c = floor(X_k + 0.5): nearest pixel to the segment on every
 *            major-axis step, ties toward c.  Both ends are included, so
 *            |P| = n + 1 and p's own colour term is counted in Eq. (1).
 *   - spatial term uses the barycenter X_k itself (Sec. II-D Remark: the
 *            projected X_k* serves only the path).
 *   - hard-mode arithmetic is FP32 in a fixed order with no contraction;
 *            the means of the update are FP64 sums in raster order rounded
 *            once to FP32 ("plain" mode) or 2^-24 fixed-point integer sums
 *            ("fixed" mode, an order-free rounding of the same mean).
 *   - projection: "contained" means label(round(X_k)) == k; the argmin of
 *            Eq. (4) is over FP32 squared distances, ties to the lowest
 *            raster index; an empty superpixel keeps centre and endpoint.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fexcess-precision=standard
 *        -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ */
/* Grid (Sec. II-A: blocks of size r, r = sqrt(N/k))                   */
/* ------------------------------------------------------------------ */

double orc_grid_r(int W, int H, int k) {
    return sqrt((double)W * (double)H / (double)k);
}

/* Returns K' = nx * ny, or -1 on invalid input. */
int orc_grid(int W, int H, int k, int *nx, int *ny) {
    if (W <= 0 || H <= 0 || k < 1 || (long)k > (long)W * H) return -1;
    double r = orc_grid_r(W, H, k);
    long gx = lround((double)W / r), gy = lround((double)H / r);
    if (gx < 1) gx = 1;
    if (gy < 1) gy = 1;
    if (gx > W) gx = W;
    if (gy > H) gy = H;
    *nx = (int)gx;
    *ny = (int)gy;
    return (int)(gx * gy);
}

/* Eq. (3) spatial weight m^2 / r^2 and the default gamma = 2r (Sec. III-A.3). */
float orc_spatial_weight(int W, int H, int k, float m) {
    double r = orc_grid_r(W, H, k);
    return (float)(((double)m * (double)m) / (r * r));
}

float orc_default_gamma(int W, int H, int k) {
    return (float)(2.0 * orc_grid_r(W, H, k));
}

static int cell_row(int y, int H, int ny) { return (int)(((long)y * ny) / H); }
static int cell_col(int x, int W, int nx) { return (int)(((long)x * nx) / W); }

/* ------------------------------------------------------------------ */
/* Contour weight summand of Eq. (2)                                   */
/* ------------------------------------------------------------------ */

void orc_wmap(const float *contour, long n, float sigma, float *w) {
    double s2 = (double)sigma * (double)sigma;
    for (long i = 0; i < n; i++) {
        double c = (double)contour[i];
        w[i] = (float)(1.0 - exp(-(c * c) / s2));
    }
}

/* ------------------------------------------------------------------ */
/* Linear path (Sec. II-B), closed form, random access by step i       */
/* ------------------------------------------------------------------ */

static int path_offset(long i, long n, int d) {
    if (n == 0) return 0;
    long ad = d < 0 ? -(long)d : (long)d;
    long off = (2 * i * ad + n) / (2 * n);
    return d < 0 ? (int)-off : (int)off;
}

/* Writes the n+1 path pixels from (x, y) to (cx, cy); returns n+1. */
int orc_path(int x, int y, int cx, int cy, int *qx, int *qy) {
    int dx = cx - x, dy = cy - y;
    int n = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    for (int i = 0; i <= n; i++) {
        qx[i] = x + path_offset(i, n, dx);
        qy[i] = y + path_offset(i, n, dy);
    }
    return n + 1;
}

/* ------------------------------------------------------------------ */
/* Distance D(p, C_k), Eqs. (1)-(3), FP32 in a fixed order             */
/* ------------------------------------------------------------------ */

typedef struct {
    int W, H;
    const float *lab;   /* [H][W][3] */
    const float *w;     /* [H][W]    */
    float lambda, gamma, spw;
} hard_ctx;

static float colour_dist(const float *f, const float *ck) {
    float dl = f[0] - ck[0];
    float da = f[1] - ck[1];
    float db = f[2] - ck[2];
    return (dl * dl + da * da) + db * db;
}

/* centre = {l, a, b, x, y}; (cx, cy) = endpoint of the path. */
static float hard_distance(const hard_ctx *c, int x, int y, const float *centre,
                           int cx, int cy, int *samples, float *A_out, float *B_out) {
    int dx = cx - x, dy = cy - y;
    int n = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    float sc = 0.0f, sw = 0.0f;
    for (int i = 0; i <= n; i++) {
        int qx = x + path_offset(i, n, dx);
        int qy = y + path_offset(i, n, dy);
        long q = (long)qy * c->W + qx;
        sc = sc + colour_dist(c->lab + 3 * q, centre);
        sw = sw + c->w[q];
    }
    if (samples) *samples += n + 1;
    float dcp = colour_dist(c->lab + 3 * ((long)y * c->W + x), centre);
    float np = (float)(n + 1);
    float oml = 1.0f - c->lambda;
    float A = c->lambda * dcp + oml * (sc / np);         /* Eq. (1) */
    float B = 1.0f + c->gamma * (sw / np);               /* Eq. (2) */
    float ex = (float)x - centre[3];
    float ey = (float)y - centre[4];
    float ds = ex * ex + ey * ey;                        /* d_s, Sec. II-A */
    if (A_out) *A_out = A;
    if (B_out) *B_out = B;
    return A * B + ds * c->spw;                          /* Eq. (3) */
}

/* D and its factors A (Eq. (1)) and B (Eq. (2)), FP32; used by the soft
 * oracle's FP32-distance mode. */
float orc_distance_ab(int W, int H, const float *lab, const float *w, float lambda, float gamma,
                      float spw, int x, int y, const float *centre, int cx, int cy,
                      float *A_out, float *B_out, int *np1) {
    hard_ctx c = {W, H, lab, w, lambda, gamma, spw};
    int samples = 0;
    float D = hard_distance(&c, x, y, centre, cx, cy, &samples, A_out, B_out);
    *np1 = samples;
    return D;
}

float orc_distance(int W, int H, const float *lab, const float *w,
                   float lambda, float gamma, float spw,
                   int x, int y, const float *centre, int cx, int cy) {
    hard_ctx c = {W, H, lab, w, lambda, gamma, spw};
    return hard_distance(&c, x, y, centre, cx, cy, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------ */
/* Assignment (Algorithm 1, inner loops), 3x3 grid-neighbour candidates */
/* ------------------------------------------------------------------ */

void orc_assign(int W, int H, int nx, int ny, const float *lab, const float *w,
                const float *centres, const int *endpoints,
                float lambda, float gamma, float spw,
                int *labels, float *best_out, long *samples_out) {
    hard_ctx c = {W, H, lab, w, lambda, gamma, spw};
    long total = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(+:total)
    for (int y = 0; y < H; y++) {
        int ci = cell_row(y, H, ny);
        for (int x = 0; x < W; x++) {
            int cj = cell_col(x, W, nx);
            float best = INFINITY;
            int bestk = -1, samples = 0;
            for (int di = -1; di <= 1; di++) {
                for (int dj = -1; dj <= 1; dj++) {
                    int ii = ci + di, jj = cj + dj;
                    if (ii < 0 || ii >= ny || jj < 0 || jj >= nx) continue;
                    int k = ii * nx + jj;
                    float D = hard_distance(&c, x, y, centres + 5 * (long)k,
                                            endpoints[2 * k], endpoints[2 * k + 1],
                                            &samples, NULL, NULL);
                    if (D < best) { best = D; bestk = k; }
                }
            }
            if (bestk < 0) bestk = ci * nx + cj;   /* only with non-finite input */
            labels[(long)y * W + x] = bestk;
            if (best_out) best_out[(long)y * W + x] = best;
            total += samples;
        }
    }
    if (samples_out) *samples_out = total;
}

/* ------------------------------------------------------------------ */
/* Assignment, cluster-centric form of Algorithm 1                      */
/* ------------------------------------------------------------------ */

/* Half-width of the (2r+1) x (2r+1) window of Algorithm 1, r rounded to a
 * whole number of pixels. */
int orc_window_radius(int W, int H, int k) {
    return (int)floor(orc_grid_r(W, H, k) + 0.5);
}

/* The window form of the candidate rule (Algorithm 1): cluster k is a
 * candidate of pixel p when p lies in k's window, the square of half-width R
 * centred on k's barycenter rounded to a pixel (clamped into the image).
 * Each pixel takes the candidate with the smallest D(p, C_k) of Eq. (3)
 * (path to k's endpoint), the smallest k among equal distances; a pixel that
 * no window contains keeps the label it had (labels is in/out).  best_out
 * receives that smallest D (+infinity where no window contains the pixel).
 * Per image row, the clusters whose window spans the row are listed first in
 * ascending k; each pixel of the row then tests the column range of each. */
void orc_assign_window(int W, int H, int K, int R, const float *lab, const float *w,
                       const float *centres, const int *endpoints,
                       float lambda, float gamma, float spw, int *labels, float *best_out) {
    hard_ctx c = {W, H, lab, w, lambda, gamma, spw};
    int *wx = malloc(sizeof(int) * (size_t)K), *wy = malloc(sizeof(int) * (size_t)K);
    for (int k = 0; k < K; k++) {
        int ex = (int)floorf(centres[5 * (long)k + 3] + 0.5f);
        int ey = (int)floorf(centres[5 * (long)k + 4] + 0.5f);
        wx[k] = ex < 0 ? 0 : (ex > W - 1 ? W - 1 : ex);
        wy[k] = ey < 0 ? 0 : (ey > H - 1 ? H - 1 : ey);
    }
    #pragma omp parallel
    {
        int *rowk = malloc(sizeof(int) * (size_t)K);
        #pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; y++) {
            int nk = 0;
            for (int k = 0; k < K; k++)
                if (abs(y - wy[k]) <= R) rowk[nk++] = k;
            for (int x = 0; x < W; x++) {
                float best = INFINITY;
                int bestk = -1;
                for (int i = 0; i < nk; i++) {
                    int k = rowk[i];
                    if (abs(x - wx[k]) > R) continue;
                    float D = hard_distance(&c, x, y, centres + 5 * (long)k, endpoints[2 * k],
                                            endpoints[2 * k + 1], NULL, NULL, NULL);
                    if (D < best) {       /* ascending k: an equal D keeps the first */
                        best = D;
                        bestk = k;
                    }
                }
                long p = (long)y * W + x;
                if (bestk >= 0) labels[p] = bestk;
                if (best_out) best_out[p] = best;
            }
        }
        free(rowk);
    }
    free(wx);
    free(wy);
}

/* ------------------------------------------------------------------ */
/* Update (Algorithm 1): mean Lab and barycenter of each superpixel    */
/* ------------------------------------------------------------------ */

#define ORC_MEAN_PLAIN 0
#define ORC_MEAN_FIXED 1
#define ORC_FIX_SCALE 16777216.0    /* 2^24 */

/* counts[k] = |S_k|.  Non-empty superpixels get their mean colour and
 * barycenter; empty ones keep the centre they had.  Labels outside [0, K)
 * are ignored. */
void orc_update(int W, int H, int K, const float *lab, const int *labels,
                int mode, float *centres, int *counts) {
    long N = (long)W * H;
    double *sum = calloc((size_t)K * 3, sizeof(double));
    long long *fix = calloc((size_t)K * 3, sizeof(long long));
    long long *sx = calloc((size_t)K, sizeof(long long));
    long long *sy = calloc((size_t)K, sizeof(long long));
    long *cnt = calloc((size_t)K, sizeof(long));
    for (long p = 0; p < N; p++) {
        int k = labels[p];
        if (k < 0 || k >= K) continue;
        cnt[k] += 1;
        sx[k] += p % W;
        sy[k] += p / W;
        for (int ch = 0; ch < 3; ch++) {
            float v = lab[3 * p + ch];
            sum[3 * (long)k + ch] += (double)v;
            fix[3 * (long)k + ch] += llrintf(v * (float)ORC_FIX_SCALE);
        }
    }
    for (int k = 0; k < K; k++) {
        counts[k] = (int)cnt[k];
        if (cnt[k] == 0) continue;
        double n = (double)cnt[k];
        for (int ch = 0; ch < 3; ch++) {
            double mean = mode == ORC_MEAN_FIXED
                ? ((double)fix[3 * (long)k + ch] / n) * (1.0 / ORC_FIX_SCALE)
                : sum[3 * (long)k + ch] / n;
            centres[5 * (long)k + ch] = (float)mean;
        }
        centres[5 * (long)k + 3] = (float)((double)sx[k] / n);
        centres[5 * (long)k + 4] = (float)((double)sy[k] / n);
    }
    free(sum); free(fix); free(sx); free(sy); free(cnt);
}

/* ------------------------------------------------------------------ */
/* Projection (Sec. II-D Remark, Eq. (4))                              */
/* ------------------------------------------------------------------ */

static int round_coord(float v, int hi) {
    int e = (int)floorf(v + 0.5f);
    if (e < 0) e = 0;
    if (e > hi) e = hi;
    return e;
}

void orc_round_endpoints(int W, int H, int K, const float *centres, int *endpoints) {
    for (int k = 0; k < K; k++) {
        endpoints[2 * k] = round_coord(centres[5 * k + 3], W - 1);
        endpoints[2 * k + 1] = round_coord(centres[5 * k + 4], H - 1);
    }
}

/* Returns the number of projected (moved) endpoints. */
int orc_project(int W, int H, int K, const int *labels, const float *centres,
                const int *counts, int *endpoints) {
    int moved = 0;
    for (int k = 0; k < K; k++) {
        if (counts[k] == 0) continue;
        int ex = round_coord(centres[5 * k + 3], W - 1);
        int ey = round_coord(centres[5 * k + 4], H - 1);
        if (labels[(long)ey * W + ex] == k) {
            endpoints[2 * k] = ex;
            endpoints[2 * k + 1] = ey;
            continue;
        }
        float best = INFINITY;
        long bestp = -1;
        for (long p = 0; p < (long)W * H; p++) {
            if (labels[p] != k) continue;
            float dx = (float)(p % W) - centres[5 * k + 3];
            float dy = (float)(p / W) - centres[5 * k + 4];
            float d = dx * dx + dy * dy;
            if (d < best) { best = d; bestp = p; }
        }
        endpoints[2 * k] = (int)(bestp % W);
        endpoints[2 * k + 1] = (int)(bestp / W);
        moved++;
    }
    return moved;
}

/* ------------------------------------------------------------------ */
/* Initialisation (Algorithm 1: clusters from a regular grid)          */
/* ------------------------------------------------------------------ */

void orc_init_grid(int W, int H, int nx, int ny, const float *lab, int mode,
                   float *centres, int *endpoints, int *labels) {
    int K = nx * ny;
    int *counts = malloc(sizeof(int) * (size_t)K);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            labels[(long)y * W + x] = cell_row(y, H, ny) * nx + cell_col(x, W, nx);
    memset(centres, 0, sizeof(float) * 5 * (size_t)K);
    orc_update(W, H, K, lab, labels, mode, centres, counts);
    orc_round_endpoints(W, H, K, centres, endpoints);
    free(counts);
}

/* ------------------------------------------------------------------ */
/* Whole run: init, then `iters` x (assign, update, project)           */
/* ------------------------------------------------------------------ */

long orc_run_window(int W, int H, int k, const float *lab, const float *contour,
                    float m, float lambda, float sigma, float gamma, int iters,
                    int project, int mode, float *centres, int *endpoints, int *labels,
                    int *counts);

long orc_run(int W, int H, int k, const float *lab, const float *contour,
             float m, float lambda, float sigma, float gamma, int iters,
             int project, int mode, float *centres, int *endpoints, int *labels,
             int *counts) {
    int nx, ny;
    int K = orc_grid(W, H, k, &nx, &ny);
    if (K < 0) return -1;
    long N = (long)W * H;
    float *w = malloc(sizeof(float) * (size_t)N);
    orc_wmap(contour, N, sigma, w);
    float spw = orc_spatial_weight(W, H, k, m);
    if (gamma < 0.0f) gamma = orc_default_gamma(W, H, k);
    orc_init_grid(W, H, nx, ny, lab, mode, centres, endpoints, labels);
    long samples = 0;
    for (int it = 0; it < iters; it++) {
        long s = 0;
        orc_assign(W, H, nx, ny, lab, w, centres, endpoints, lambda, gamma, spw,
                   labels, NULL, &s);
        samples += s;
        orc_update(W, H, K, lab, labels, mode, centres, counts);
        if (project)
            orc_project(W, H, K, labels, centres, counts, endpoints);
        else
            orc_round_endpoints(W, H, K, centres, endpoints);
    }
    free(w);
    return samples;
}

/* The same run with the window assignment of Algorithm 1. */
long orc_run_window(int W, int H, int k, const float *lab, const float *contour,
                    float m, float lambda, float sigma, float gamma, int iters,
                    int project, int mode, float *centres, int *endpoints, int *labels,
                    int *counts) {
    int nx, ny;
    int K = orc_grid(W, H, k, &nx, &ny);
    if (K < 0) return -1;
    long N = (long)W * H;
    float *w = malloc(sizeof(float) * (size_t)N);
    orc_wmap(contour, N, sigma, w);
    float spw = orc_spatial_weight(W, H, k, m);
    if (gamma < 0.0f) gamma = orc_default_gamma(W, H, k);
    int R = orc_window_radius(W, H, k);
    orc_init_grid(W, H, nx, ny, lab, mode, centres, endpoints, labels);
    for (int it = 0; it < iters; it++) {
        orc_assign_window(W, H, K, R, lab, w, centres, endpoints, lambda, gamma, spw, labels,
                          NULL);
        orc_update(W, H, K, lab, labels, mode, centres, counts);
        if (project)
            orc_project(W, H, K, labels, centres, counts, endpoints);
        else
            orc_round_endpoints(W, H, K, centres, endpoints);
    }
    free(w);
    return 0;
}

void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
