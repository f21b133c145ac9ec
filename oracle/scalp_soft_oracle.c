/*
 * scalp_soft_oracle.c -- FP64 CPU oracle for soft (differentiable) SCALP.
 *
 * TEST INFRASTRUCTURE ONLY (see scalp_oracle.c).
 *
 * Soft SCALP is an extension of the paper's method, not part of it.  It
 * keeps the distance D of Eqs. (1)-(3) over the same 3x3 grid-neighbour
 * candidates as the hard assignment of Algorithm 1, and replaces the argmin
 * and the hard update by
 *     Q_pj   = exp(-(D_pj - min_j D_pj) / T) / sum_j exp(-(D_pj - min_j D_pj) / T)
 *     Z_k    = sum_{(p,j) -> k} Q_pj
 *     f_k    = sum Q_pj f_p / Z_k,   X_k = sum Q_pj X_p / Z_k   (Z_k = 0: keep)
 * starting from Theta_0 = cell means of the Lab features and cell
 * barycenters.  Path endpoints are the rounded barycenters floor(X_k + 0.5)
 * with no projection (Eq. (4) needs hard membership); they are piecewise
 * constant in X_k, so they carry no gradient.  Slots j = (di+1)*3 + (dj+1)
 * index the 3x3 neighbourhood; slots outside the grid have Q = 0.
 *
 * A superpixel whose soft mass Z_k is below 1e-6 (a millionth of a pixel)
 * counts as empty and keeps its centre, as an empty superpixel does in the
 * hard update: its soft mean would be decided by weights that FP32 cannot
 * represent, and dTheta/dQ = (f - Theta)/Z would be unbounded.
 *
 * Two precisions:
 *   d32 = 0  everything in FP64.  This is the mode whose gradient is checked
 *            against central finite differences of its own forward.
 *   d32 = 1  the precision contract of the FP32 path: D, A and B are the hard
 *            oracle's FP32 distance (same operation order), the softmax and
 *            the update sums are FP64, and Q and Theta are rounded to FP32
 *            where they are produced (endpoints are floorf(x + 0.5f) of the
 *            FP32 barycenter); the backward is the FP64 chain rule at those
 *            values.  The GPU path is compared with this mode.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

int orc_grid(int W, int H, int k, int *nx, int *ny);
double orc_grid_r(int W, int H, int k);
float orc_spatial_weight(int W, int H, int k, float m);
float orc_default_gamma(int W, int H, int k);
void orc_wmap(const float *contour, long n, float sigma, float *w);
float orc_distance_ab(int W, int H, const float *lab, const float *w, float lambda, float gamma,
                      float spw, int x, int y, const float *centre, int cx, int cy,
                      float *A_out, float *B_out, int *np1);

#define SOFT_Z_MIN 1e-6

typedef struct {
    int W, H, nx, ny, K;
    const float *lab;      /* [H][W][3] */
    const double *w;       /* [H][W]    */
    double lambda, gamma, spw, T;
    int d32;               /* FP32-distance mode (see header) */
    const float *w32;      /* [H][W], FP32 w map (d32 mode) */
    float lambda32, gamma32, spw32;
} soft_ctx;

/* FP64 value as produced in the active precision (FP32 rounding in d32 mode). */
static double as_out(const soft_ctx *c, double v) { return c->d32 ? (double)(float)v : v; }

static int s_path_offset(long i, long n, int d) {
    if (n == 0) return 0;
    long ad = d < 0 ? -(long)d : (long)d;
    long off = (2 * i * ad + n) / (2 * n);
    return d < 0 ? (int)-off : (int)off;
}

static int s_round(double v, int hi, int d32) {
    int e = d32 ? (int)floorf((float)v + 0.5f) : (int)floor(v + 0.5);
    if (e < 0) e = 0;
    if (e > hi) e = hi;
    return e;
}

static int slot_cluster(const soft_ctx *c, int x, int y, int j) {
    int ci = (int)(((long)y * c->ny) / c->H), cj = (int)(((long)x * c->nx) / c->W);
    int ii = ci + j / 3 - 1, jj = cj + j % 3 - 1;
    if (ii < 0 || ii >= c->ny || jj < 0 || jj >= c->nx) return -1;
    return ii * c->nx + jj;
}

static double dc64(const float *f, const double *ck) {
    double dl = (double)f[0] - ck[0], da = (double)f[1] - ck[1], db = (double)f[2] - ck[2];
    return dl * dl + da * da + db * db;
}

/* D(p, C_k) of Eq. (3) in FP64; also returns the two factors A (Eq. (1))
 * and B (Eq. (2)) and the path length n+1. */
static double soft_distance(const soft_ctx *c, int x, int y, const double *th,
                            int cx, int cy, double *A, double *B, int *np1) {
    if (c->d32) {
        float centre[5] = {(float)th[0], (float)th[1], (float)th[2], (float)th[3], (float)th[4]};
        float a32, b32;
        float D = orc_distance_ab(c->W, c->H, c->lab, c->w32, c->lambda32, c->gamma32, c->spw32,
                                  x, y, centre, cx, cy, &a32, &b32, np1);
        *A = a32;
        *B = b32;
        return D;
    }
    int dx = cx - x, dy = cy - y;
    int n = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    double sc = 0.0, sw = 0.0;
    for (int i = 0; i <= n; i++) {
        long q = (long)(y + s_path_offset(i, n, dy)) * c->W + (x + s_path_offset(i, n, dx));
        sc += dc64(c->lab + 3 * q, th);
        sw += c->w[q];
    }
    double np = (double)(n + 1);
    double dcp = dc64(c->lab + 3 * ((long)y * c->W + x), th);
    *A = c->lambda * dcp + (1.0 - c->lambda) * sc / np;
    *B = 1.0 + c->gamma * sw / np;
    *np1 = n + 1;
    double ex = (double)x - th[3], ey = (double)y - th[4];
    return (*A) * (*B) + (ex * ex + ey * ey) * c->spw;
}

static void soft_init(const soft_ctx *c, double *th0) {
    double *cnt = calloc((size_t)c->K, sizeof(double));
    memset(th0, 0, sizeof(double) * 5 * (size_t)c->K);
    for (int y = 0; y < c->H; y++)
        for (int x = 0; x < c->W; x++) {
            int k = slot_cluster(c, x, y, 4);
            const float *f = c->lab + 3 * ((long)y * c->W + x);
            th0[5 * k + 0] += f[0];
            th0[5 * k + 1] += f[1];
            th0[5 * k + 2] += f[2];
            th0[5 * k + 3] += x;
            th0[5 * k + 4] += y;
            cnt[k] += 1.0;
        }
    for (int k = 0; k < c->K; k++)
        for (int e = 0; e < 5; e++) th0[5 * k + e] = as_out(c, th0[5 * k + e] / cnt[k]);
    free(cnt);
}

/* One soft iteration: Q from theta_prev, then theta_next and Z. */
static void soft_step(const soft_ctx *c, const double *th_prev, double *q, double *th_next,
                      double *z) {
    int K = c->K;
    int *ex = malloc(sizeof(int) * 2 * (size_t)K);
    for (int k = 0; k < K; k++) {
        ex[2 * k] = s_round(th_prev[5 * k + 3], c->W - 1, c->d32);
        ex[2 * k + 1] = s_round(th_prev[5 * k + 4], c->H - 1, c->d32);
    }
    double *acc = calloc((size_t)K * 5, sizeof(double));
    memset(z, 0, sizeof(double) * (size_t)K);
    for (int y = 0; y < c->H; y++)
        for (int x = 0; x < c->W; x++) {
            double D[9], mn = INFINITY, A, B, s = 0.0;
            int np1;
            long p = (long)y * c->W + x;
            for (int j = 0; j < 9; j++) {
                int k = slot_cluster(c, x, y, j);
                D[j] = INFINITY;
                if (k < 0) continue;
                D[j] = soft_distance(c, x, y, th_prev + 5 * k, ex[2 * k], ex[2 * k + 1],
                                     &A, &B, &np1);
                if (D[j] < mn) mn = D[j];
            }
            for (int j = 0; j < 9; j++) {
                double e = slot_cluster(c, x, y, j) < 0 ? 0.0 : exp(-(D[j] - mn) / c->T);
                q[9 * p + j] = e;
                s += e;
            }
            const float *f = c->lab + 3 * p;
            for (int j = 0; j < 9; j++) {
                q[9 * p + j] = as_out(c, q[9 * p + j] / s);
                int k = slot_cluster(c, x, y, j);
                if (k < 0) continue;
                double Q = q[9 * p + j];
                z[k] += Q;
                acc[5 * k + 0] += Q * f[0];
                acc[5 * k + 1] += Q * f[1];
                acc[5 * k + 2] += Q * f[2];
                acc[5 * k + 3] += Q * x;
                acc[5 * k + 4] += Q * y;
            }
        }
    for (int k = 0; k < K; k++)
        for (int e = 0; e < 5; e++)
            th_next[5 * k + e] = z[k] >= SOFT_Z_MIN ? as_out(c, acc[5 * k + e] / z[k])
                                                     : th_prev[5 * k + e];
    free(acc);
    free(ex);
}

static int soft_setup(soft_ctx *c, int W, int H, int k, const float *lab, const float *contour,
                      double m, double lambda, double sigma, double gamma, double T, int d32,
                      double **wbuf, float **w32buf) {
    int nx, ny;
    int K = orc_grid(W, H, k, &nx, &ny);
    if (K < 0 || T <= 0.0 || sigma <= 0.0) return -1;
    double r = orc_grid_r(W, H, k);
    long N = (long)W * H;
    double *w = malloc(sizeof(double) * (size_t)N);
    for (long i = 0; i < N; i++) {
        double cq = contour[i];
        w[i] = 1.0 - exp(-(cq * cq) / (sigma * sigma));
    }
    c->W = W; c->H = H; c->nx = nx; c->ny = ny; c->K = K;
    c->lab = lab; c->w = w;
    c->lambda = lambda;
    c->gamma = gamma < 0.0 ? 2.0 * r : gamma;
    c->spw = m * m / (r * r);
    c->T = T;
    c->d32 = d32;
    float *w32 = malloc(sizeof(float) * (size_t)N);
    orc_wmap(contour, N, (float)sigma, w32);
    c->w32 = w32;
    c->lambda32 = (float)lambda;
    c->gamma32 = gamma < 0.0 ? orc_default_gamma(W, H, k) : (float)gamma;
    c->spw32 = orc_spatial_weight(W, H, k, (float)m);
    *wbuf = w;
    *w32buf = w32;
    return K;
}

/* theta: [iters+1][B][K][5]; q: [iters][B][H][W][9]; z: [iters][B][K]. */
int orc_soft_forward(int Bn, int W, int H, int k, const float *lab, const float *contour,
                     double m, double lambda, double sigma, double gamma, double T, int iters,
                     int d32, double *theta, double *q, double *z) {
    long N = (long)W * H;
    for (int b = 0; b < Bn; b++) {
        soft_ctx c;
        double *w;
        float *w32;
        int K = soft_setup(&c, W, H, k, lab + 3 * N * b, contour + N * b, m, lambda, sigma,
                           gamma, T, d32, &w, &w32);
        if (K < 0) return -1;
        soft_init(&c, theta + 5L * K * b);
        for (int t = 0; t < iters; t++) {
            const double *prev = theta + 5L * K * ((long)t * Bn + b);
            double *next = theta + 5L * K * ((long)(t + 1) * Bn + b);
            soft_step(&c, prev, q + 9 * N * ((long)t * Bn + b), next, z + (long)K * ((long)t * Bn + b));
        }
        free(w);
        free(w32);
    }
    return 0;
}

/* Gradient of L = <gq, Q_T> + <gtheta, Theta_T> w.r.t. the Lab features and
 * the contour map.  gq: [B][H][W][9]; gtheta: [B][K][5]; glab: [B][H][W][3];
 * gcontour: [B][H][W]. */
int orc_soft_backward(int Bn, int W, int H, int k, const float *lab, const float *contour,
                      double m, double lambda, double sigma, double gamma, double T, int iters,
                      int d32, const double *gq_in, const double *gtheta_in,
                      double *glab, double *gcontour) {
    long N = (long)W * H;
    for (int b = 0; b < Bn; b++) {
        soft_ctx c;
        double *w;
        float *w32;
        int K = soft_setup(&c, W, H, k, lab + 3 * N * b, contour + N * b, m, lambda, sigma,
                           gamma, T, d32, &w, &w32);
        if (K < 0) return -1;
        const float *f = c.lab;
        /* forward, keeping every iterate */
        double *th = malloc(sizeof(double) * 5 * (size_t)K * (size_t)(iters + 1));
        double *qq = malloc(sizeof(double) * 9 * (size_t)N * (size_t)(iters > 0 ? iters : 1));
        double *zz = malloc(sizeof(double) * (size_t)K * (size_t)(iters > 0 ? iters : 1));
        soft_init(&c, th);
        for (int t = 0; t < iters; t++)
            soft_step(&c, th + 5L * K * t, qq + 9 * N * t, th + 5L * K * (t + 1), zz + (long)K * t);

        double *gf = calloc((size_t)N * 3, sizeof(double));
        double *gw = calloc((size_t)N, sizeof(double));
        double *gth = malloc(sizeof(double) * 5 * (size_t)K);
        double *gth_prev = malloc(sizeof(double) * 5 * (size_t)K);
        double *gQ = malloc(sizeof(double) * 9 * (size_t)N);
        memcpy(gth, gtheta_in + 5L * K * b, sizeof(double) * 5 * (size_t)K);
        memcpy(gQ, gq_in + 9 * N * b, sizeof(double) * 9 * (size_t)N);
        int *ex = malloc(sizeof(int) * 2 * (size_t)K);

        for (int t = iters - 1; t >= 0; t--) {
            const double *thp = th + 5L * K * t;        /* Theta_{t}   (input of step t) */
            const double *thn = th + 5L * K * (t + 1);  /* Theta_{t+1} (output)          */
            const double *Q = qq + 9 * N * t;
            const double *Z = zz + (long)K * t;
            if (t != iters - 1) memset(gQ, 0, sizeof(double) * 9 * (size_t)N);
            /* soft update backward: theta_next = sum Q feat / Z */
            memset(gth_prev, 0, sizeof(double) * 5 * (size_t)K);
            for (int kk = 0; kk < K; kk++)
                if (!(Z[kk] >= SOFT_Z_MIN))
                    for (int e = 0; e < 5; e++) gth_prev[5 * kk + e] += gth[5 * kk + e];
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) {
                    long p = (long)y * W + x;
                    double feat[5] = {f[3 * p], f[3 * p + 1], f[3 * p + 2], (double)x, (double)y};
                    for (int j = 0; j < 9; j++) {
                        int kk = slot_cluster(&c, x, y, j);
                        if (kk < 0 || !(Z[kk] >= SOFT_Z_MIN)) continue;
                        double s = 0.0;
                        for (int e = 0; e < 5; e++)
                            s += gth[5 * kk + e] * (feat[e] - thn[5 * kk + e]);
                        gQ[9 * p + j] += s / Z[kk];
                        for (int e = 0; e < 3; e++)
                            gf[3 * p + e] += gth[5 * kk + e] * Q[9 * p + j] / Z[kk];
                    }
                }
            /* softmax backward and path backward */
            for (int kk = 0; kk < K; kk++) {
                ex[2 * kk] = s_round(thp[5 * kk + 3], W - 1, c.d32);
                ex[2 * kk + 1] = s_round(thp[5 * kk + 4], H - 1, c.d32);
            }
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) {
                    long p = (long)y * W + x;
                    double dot = 0.0;
                    for (int j = 0; j < 9; j++) dot += Q[9 * p + j] * gQ[9 * p + j];
                    for (int j = 0; j < 9; j++) {
                        int kk = slot_cluster(&c, x, y, j);
                        if (kk < 0) continue;
                        double g = -(1.0 / T) * Q[9 * p + j] * (gQ[9 * p + j] - dot);
                        if (g == 0.0) continue;
                        const double *ck = thp + 5 * kk;
                        double A, Bw;
                        int np1;
                        soft_distance(&c, x, y, ck, ex[2 * kk], ex[2 * kk + 1], &A, &Bw, &np1);
                        double np = (double)np1;
                        int cx = ex[2 * kk], cy = ex[2 * kk + 1];
                        int ddx = cx - x, ddy = cy - y;
                        int n = np1 - 1;
                        double gk[3] = {0.0, 0.0, 0.0};
                        for (int e = 0; e < 3; e++) {
                            double dpe = 2.0 * ((double)f[3 * p + e] - ck[e]);
                            gf[3 * p + e] += g * Bw * lambda * dpe;
                            gk[e] -= g * Bw * lambda * dpe;
                        }
                        for (int i = 0; i <= n; i++) {
                            long qix = (long)(y + s_path_offset(i, n, ddy)) * W +
                                       (x + s_path_offset(i, n, ddx));
                            for (int e = 0; e < 3; e++) {
                                double dqe = 2.0 * ((double)f[3 * qix + e] - ck[e]);
                                gf[3 * qix + e] += g * Bw * (1.0 - lambda) / np * dqe;
                                gk[e] -= g * Bw * (1.0 - lambda) / np * dqe;
                            }
                            gw[qix] += g * A * c.gamma / np;
                        }
                        for (int e = 0; e < 3; e++) gth_prev[5 * kk + e] += gk[e];
                        gth_prev[5 * kk + 3] += -2.0 * g * c.spw * ((double)x - ck[3]);
                        gth_prev[5 * kk + 4] += -2.0 * g * c.spw * ((double)y - ck[4]);
                    }
                }
            memcpy(gth, gth_prev, sizeof(double) * 5 * (size_t)K);
        }
        /* Theta_0 = cell means of the features */
        {
            double *cnt = calloc((size_t)K, sizeof(double));
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) cnt[slot_cluster(&c, x, y, 4)] += 1.0;
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) {
                    long p = (long)y * W + x;
                    int kk = slot_cluster(&c, x, y, 4);
                    for (int e = 0; e < 3; e++) gf[3 * p + e] += gth[5 * kk + e] / cnt[kk];
                }
            free(cnt);
        }
        for (long p = 0; p < N; p++) {
            for (int e = 0; e < 3; e++) glab[3 * (N * b + p) + e] = gf[3 * p + e];
            double cq = contour[N * b + p];
            double s2 = sigma * sigma;
            gcontour[N * b + p] = gw[p] * (2.0 * cq / s2) * exp(-(cq * cq) / s2);
        }
        free(th); free(qq); free(zz); free(gf); free(gw); free(gth); free(gth_prev);
        free(gQ); free(ex); free(w); free(w32);
    }
    return 0;
}
