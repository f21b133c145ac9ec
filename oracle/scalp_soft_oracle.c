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

/* ------------------------------------------------------------------ */
/* Backward                                                             */
/* ------------------------------------------------------------------ */

/* Rounding to FP32 of every intermediate result of the backward (the r32
 * option): a second, FP32 evaluation of the same chain rule, which the
 * error bound below must cover. */
static double R(int r32, double v) { return r32 ? (double)(float)v : v; }

/* Error bound of an FP32 evaluation of the backward (test infrastructure).
 * First-order running error analysis (Wilkinson; Higham, Accuracy and
 * Stability of Numerical Algorithms, ch. 3) with u = 2^-24: a quantity x of
 * the chain rule carries a bound E(x) (in units of u) on how far an FP32
 * evaluation of it can be from the exact value at the reference's inputs:
 *   z = x * y           E(z) = |x| E(y) + |y| E(x) + |z|        (one rounding)
 *   z = x - y           E(z) = E(x) + E(y) + |z|
 *   s = t_1 + ... + t_n E(s) = sum E(t_i) + (n - 1) sum |t_i|  (any order or
 *                       tree of FP32 additions, as with float atomics)
 * with a few more roundings allowed per formula for the way an FP32 path may
 * group it.  Forward values that the FP32 path produces itself are leaves
 * with their own error: Q and Theta within one FP32 ulp of this oracle's
 * (E = 2|Q|, 2|Theta|), Z rounded from an FP64 sum of such Q (3|Z|), the
 * factor A of Eq. (1) evaluated in FP32 on both sides from a Theta one ulp
 * apart (2 (n + 8) A for the two evaluations of a path of n steps, plus the
 * first-order effect of the Theta difference), the factor B of Eq. (2)
 * bit-identical (no Theta in it once the endpoints agree).
 * Two readings keep the bound from compounding over iterations (an
 * absolute-value chain through the softmax and update backward grows by
 * 10^3-10^4 per iteration): dL/dTheta is taken to be summed in FP64 from
 * FP32 partial sums no longer than one path, so it enters the iteration below
 * with E = (longest path to the superpixel + B_LOCAL + 16) sum |terms|, each
 * term counted at its local depth rather than with the bound of the dL/dD it
 * came from (one level).  Everything within an iteration, and the
 * accumulation of the outputs, is bounded in full.
 * Separately, Md bounds (absolutely) what leaving out every slot with
 * Q < 2^-24 changes: such a slot's dL/dD enters Md whole and propagates
 * linearly through the full chain (a slot within one ulp of the cut counts
 * as left out; with the qcut option, which leaves those slots out here too,
 * only the slots within one ulp of the cut enter Md).  An FP32 evaluation then errs by at most u E + Md per
 * element, to first order.
 * Per accumulated element: se = sum of term bounds, sa = sum of |terms|,
 * n = number of terms, md = sum of term Md. */
typedef struct { double *se, *sa, *n, *md; } bacc;

static int bacc_alloc(bacc *a, size_t len) {
    a->se = calloc(len, sizeof(double));
    a->sa = calloc(len, sizeof(double));
    a->n = calloc(len, sizeof(double));
    a->md = calloc(len, sizeof(double));
    return a->se && a->sa && a->n && a->md;
}
static void bacc_free(bacc *a) { free(a->se); free(a->sa); free(a->n); free(a->md); }
static void bacc_zero(bacc *a, size_t len) {
    memset(a->se, 0, len * sizeof(double));
    memset(a->sa, 0, len * sizeof(double));
    memset(a->n, 0, len * sizeof(double));
    memset(a->md, 0, len * sizeof(double));
}
/* adds the term t, whose own bound is e and dropped bound md */
static void bacc_add(bacc *a, long i, double t, double e, double md) {
    a->se[i] += e;
    a->sa[i] += fabs(t);
    a->n[i] += 1.0;
    a->md[i] += md;
}
/* E of the accumulated sum */
static double bacc_e(const bacc *a, long i) {
    return a->se[i] + (a->n[i] > 1.0 ? (a->n[i] - 1.0) * a->sa[i] : 0.0);
}

#define B_DQ 2.0     /* Q: one FP32 ulp */
#define B_DTH 2.0    /* Theta: one FP32 ulp */
#define B_DZ 3.0     /* Z: FP64 sum of such Q, rounded to FP32 */
#define B_QCUT 0x1p-24
#define B_LOCAL 40.0  /* roundings of one term of dL/dTheta (its g, path factors, difference) */

/* Gradient of L = <gq, Q_T> + <gtheta, Theta_T> w.r.t. the Lab features and
 * the contour map.  gq: [B][H][W][9]; gtheta: [B][K][5]; glab: [B][H][W][3];
 * gcontour: [B][H][W].
 * Options (test infrastructure; 0 and NULL give the plain FP64 chain rule):
 *   qcut   leave out every slot whose Q is below 2^-24;
 *   r32    round every intermediate result to FP32;
 *   bnd    if not NULL, four arrays receive the error bound of an FP32
 *          evaluation (see bacc above): E and Md of glab ([B][H][W][3]
 *          each), then of gcontour ([B][H][W] each). */
int orc_soft_backward_ex(int Bn, int W, int H, int k, const float *lab, const float *contour,
                         double m, double lambda, double sigma, double gamma, double T,
                         int iters, int d32, const double *gq_in, const double *gtheta_in,
                         double *glab, double *gcontour, int qcut, int r32, double **bnd) {
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
        for (long i = 0; i < 5L * K; i++) gth[i] = R(r32, gtheta_in[5L * K * b + i]);
        for (long i = 0; i < 9 * N; i++) gQ[i] = R(r32, gq_in[9 * N * b + i]);
        int *ex = malloc(sizeof(int) * 2 * (size_t)K);
        /* the bound: per-element accumulators, and the finished dL/dTheta
         * of the iteration below (its E and Md) */
        bacc bf = {0}, bw = {0}, bq = {0}, bp = {0};
        double *eth = NULL, *mdth = NULL, *ge = NULL, *gmd = NULL, *plen = NULL;
        if (bnd) {
            if (!bacc_alloc(&bf, 3 * (size_t)N) || !bacc_alloc(&bw, (size_t)N) ||
                !bacc_alloc(&bq, 9 * (size_t)N) || !bacc_alloc(&bp, 5 * (size_t)K))
                return -2;
            eth = calloc(5 * (size_t)K, sizeof(double));
            mdth = calloc(5 * (size_t)K, sizeof(double));
            ge = malloc(sizeof(double) * 9);
            gmd = malloc(sizeof(double) * 9);
            plen = calloc((size_t)K, sizeof(double));
            for (long i = 0; i < 9 * N; i++) bacc_add(&bq, i, gQ[i], 0.0, 0.0);
        }

        for (int t = iters - 1; t >= 0; t--) {
            const double *thp = th + 5L * K * t;        /* Theta_{t}   (input of step t) */
            const double *thn = th + 5L * K * (t + 1);  /* Theta_{t+1} (output)          */
            const double *Q = qq + 9 * N * t;
            const double *Z = zz + (long)K * t;
            if (t != iters - 1) {
                memset(gQ, 0, sizeof(double) * 9 * (size_t)N);
                if (bnd) bacc_zero(&bq, 9 * (size_t)N);
            }
            /* soft update backward: theta_next = sum Q feat / Z */
            memset(gth_prev, 0, sizeof(double) * 5 * (size_t)K);
            if (bnd) {
                bacc_zero(&bp, 5 * (size_t)K);
                memset(plen, 0, sizeof(double) * (size_t)K);
            }
            for (int kk = 0; kk < K; kk++)
                if (!(Z[kk] >= SOFT_Z_MIN))
                    for (int e = 0; e < 5; e++) {
                        gth_prev[5 * kk + e] += gth[5 * kk + e];
                        if (bnd) bacc_add(&bp, 5 * kk + e, gth[5 * kk + e], eth[5 * kk + e],
                                          mdth[5 * kk + e]);
                    }
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) {
                    long p = (long)y * W + x;
                    double feat[5] = {f[3 * p], f[3 * p + 1], f[3 * p + 2], (double)x, (double)y};
                    for (int j = 0; j < 9; j++) {
                        int kk = slot_cluster(&c, x, y, j);
                        if (kk < 0 || !(Z[kk] >= SOFT_Z_MIN)) continue;
                        double Zk = R(r32, Z[kk]);
                        double s = 0.0;
                        for (int e = 0; e < 5; e++)
                            s = R(r32, s + R(r32, gth[5 * kk + e] *
                                                  R(r32, feat[e] - thn[5 * kk + e])));
                        double tau = R(r32, s / Zk);
                        gQ[9 * p + j] = R(r32, gQ[9 * p + j] + tau);
                        for (int e = 0; e < 3; e++)
                            gf[3 * p + e] = R(r32, gf[3 * p + e] +
                                                   R(r32, R(r32, gth[5 * kk + e] * Q[9 * p + j]) / Zk));
                        if (bnd) {
                            /* tau = sum_e gth_e (feat_e - thn_e) / Z: an FP32 path may
                             * form u = gth / Z, then u . feat - u . thn, so its
                             * roundings are counted on |u| (|feat| + |thn|) */
                            double z = Z[kk], ez = B_DZ * z, et = 0.0, mt = 0.0, cancel = 0.0;
                            for (int e = 0; e < 5; e++) {
                                double d = feat[e] - thn[5 * kk + e], g0 = gth[5 * kk + e];
                                et += fabs(d) * (eth[5 * kk + e] / z + fabs(g0) * ez / (z * z)) +
                                      fabs(g0) / z * B_DTH * fabs(thn[5 * kk + e]);
                                cancel += fabs(g0) / z * (fabs(feat[e]) + fabs(thn[5 * kk + e]));
                                mt += mdth[5 * kk + e] * fabs(d) / z;
                            }
                            et += 12.0 * cancel;
                            bacc_add(&bq, 9 * p + j, s / z, et, mt);
                            for (int e = 0; e < 3; e++) {
                                double g0 = gth[5 * kk + e], qv = Q[9 * p + j];
                                double tv = g0 * qv / z;
                                bacc_add(&bf, 3 * p + e, tv,
                                         qv / z * eth[5 * kk + e] + fabs(g0) / z * B_DQ * qv +
                                             fabs(tv) / z * ez + 3.0 * fabs(tv),
                                         mdth[5 * kk + e] * qv / z);
                            }
                        }
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
                    for (int j = 0; j < 9; j++)
                        dot = R(r32, dot + R(r32, Q[9 * p + j] * gQ[9 * p + j]));
                    if (bnd) {
                        /* E and Md of dot = sum_j Q_j G_j, then of every
                         * g_j = -(1/T) Q_j (G_j - dot) */
                        double edot = 0.0, sdot = 0.0, mddot = 0.0;
                        for (int j = 0; j < 9; j++) {
                            double qj = Q[9 * p + j], G = gQ[9 * p + j];
                            edot += qj * bacc_e(&bq, 9 * p + j) + fabs(G) * B_DQ * qj + qj * fabs(G);
                            sdot += qj * fabs(G);
                            mddot += qj * bq.md[9 * p + j];
                        }
                        edot += 8.0 * sdot;
                        for (int j = 0; j < 9; j++) {
                            double qj = Q[9 * p + j], dl = gQ[9 * p + j] - dot;
                            double gv = qj * dl / T;
                            double edl = bacc_e(&bq, 9 * p + j) + edot + fabs(dl);
                            ge[j] = (qj * edl + fabs(dl) * B_DQ * qj) / T + 3.0 * fabs(gv);
                            gmd[j] = qj * (bq.md[9 * p + j] + mddot) / T;
                            /* left out by one side only: below the cut (with qcut,
                             * only within one ulp of it, where the two sides'
                             * Q may fall on different sides) */
                            if (qj <= B_QCUT * (1.0 + 0x1p-22) &&
                                (!qcut || qj >= B_QCUT * (1.0 - 0x1p-22)))
                                gmd[j] += fabs(gv);
                        }
                    }
                    for (int j = 0; j < 9; j++) {
                        int kk = slot_cluster(&c, x, y, j);
                        if (kk < 0) continue;
                        double g = R(r32, -R(r32, R(r32, 1.0 / T) * Q[9 * p + j]) *
                                              R(r32, gQ[9 * p + j] - dot));
                        if (qcut && Q[9 * p + j] < B_QCUT) g = 0.0;
                        if (g == 0.0 && !(bnd && (ge[j] > 0.0 || gmd[j] > 0.0))) continue;
                        const double *ck = thp + 5 * kk;
                        double A, Bw;
                        int np1;
                        soft_distance(&c, x, y, ck, ex[2 * kk], ex[2 * kk + 1], &A, &Bw, &np1);
                        double np = (double)np1;
                        int cx = ex[2 * kk], cy = ex[2 * kk + 1];
                        int ddx = cx - x, ddy = cy - y;
                        int n = np1 - 1;
                        double gk[3] = {0.0, 0.0, 0.0};
                        double cfp = R(r32, R(r32, g * Bw) * lambda);          /* at p */
                        double cfq = R(r32, R(r32, R(r32, g * Bw) * (1.0 - lambda)) / np);
                        double cwq = R(r32, R(r32, R(r32, g * A) * c.gamma) / np);
                        for (int e = 0; e < 3; e++) {
                            double dpe = R(r32, 2.0 * R(r32, (double)f[3 * p + e] - ck[e]));
                            double v = R(r32, cfp * dpe);
                            gf[3 * p + e] = R(r32, gf[3 * p + e] + v);
                            gk[e] = R(r32, gk[e] - v);
                        }
                        /* the bound's factors (the reference value g is the plain
                         * one, also where qcut left it out) */
                        double gv = 0.0, eg = 0.0, mdg = 0.0, eA = 0.0, ecf = 0.0, mdcf = 0.0;
                        double cfv = 0.0, cwv = 0.0, ecw = 0.0, mdcw = 0.0;
                        if (bnd) {
                            if (np > plen[kk]) plen[kk] = np;
                            gv = -(Q[9 * p + j] * (gQ[9 * p + j] - dot)) / T;
                            eg = ge[j];
                            mdg = gmd[j];
                            /* A: two FP32 evaluations (2 (n + 8) A) and the effect of
                             * Theta one ulp away, sum_e 2 |Theta_e| |dA/dTheta_e| */
                            double sp[3] = {0.0, 0.0, 0.0}, sq[3] = {0.0, 0.0, 0.0};
                            for (int e = 0; e < 3; e++) sp[e] = fabs((double)f[3 * p + e] - ck[e]);
                            for (int i = 0; i <= n; i++) {
                                long qix = (long)(y + s_path_offset(i, n, ddy)) * W +
                                           (x + s_path_offset(i, n, ddx));
                                for (int e = 0; e < 3; e++)
                                    sq[e] += fabs((double)f[3 * qix + e] - ck[e]);
                            }
                            eA = 2.0 * (n + 8) * A;
                            for (int e = 0; e < 3; e++)
                                eA += B_DTH * fabs(ck[e]) * 2.0 *
                                      (lambda * sp[e] + (1.0 - lambda) * sq[e] / np);
                            double lfv = 2.0 * gv * Bw * lambda;
                            double elf = 2.0 * Bw * lambda * eg + 3.0 * fabs(lfv);
                            double mdlf = 2.0 * Bw * lambda * mdg;
                            cfv = 2.0 * gv * Bw * (1.0 - lambda) / np;
                            ecf = 2.0 * Bw * (1.0 - lambda) / np * eg + 5.0 * fabs(cfv);
                            mdcf = 2.0 * Bw * (1.0 - lambda) / np * mdg;
                            cwv = gv * A * c.gamma / np;
                            ecw = A * c.gamma / np * eg + fabs(gv) * c.gamma / np * eA +
                                  6.0 * fabs(cwv);
                            mdcw = A * c.gamma / np * mdg;
                            for (int e = 0; e < 3; e++) {
                                double d = (double)f[3 * p + e] - ck[e], tv = lfv * d;
                                double et = fabs(d) * elf +
                                            fabs(lfv) * (B_DTH * fabs(ck[e]) + fabs(d)) + fabs(tv);
                                bacc_add(&bf, 3 * p + e, tv, et, fabs(d) * mdlf);
                                bacc_add(&bp, 5 * kk + e, tv, et, fabs(d) * mdlf);
                            }
                        }
                        for (int i = 0; i <= n; i++) {
                            long qix = (long)(y + s_path_offset(i, n, ddy)) * W +
                                       (x + s_path_offset(i, n, ddx));
                            for (int e = 0; e < 3; e++) {
                                double dqe = R(r32, 2.0 * R(r32, (double)f[3 * qix + e] - ck[e]));
                                double v = R(r32, cfq * dqe);
                                gf[3 * qix + e] = R(r32, gf[3 * qix + e] + v);
                                gk[e] = R(r32, gk[e] - v);
                                if (bnd) {
                                    double d = (double)f[3 * qix + e] - ck[e], tv = cfv * d;
                                    double et = fabs(d) * ecf +
                                                fabs(cfv) * (B_DTH * fabs(ck[e]) + fabs(d)) +
                                                fabs(tv);
                                    bacc_add(&bf, 3 * qix + e, tv, et, fabs(d) * mdcf);
                                    bacc_add(&bp, 5 * kk + e, tv, et, fabs(d) * mdcf);
                                }
                            }
                            gw[qix] = R(r32, gw[qix] + cwq);
                            if (bnd) bacc_add(&bw, qix, cwv, ecw, mdcw);
                        }
                        for (int e = 0; e < 3; e++)
                            gth_prev[5 * kk + e] = R(r32, gth_prev[5 * kk + e] + gk[e]);
                        double dxk = R(r32, (double)x - ck[3]), dyk = R(r32, (double)y - ck[4]);
                        gth_prev[5 * kk + 3] = R(r32, gth_prev[5 * kk + 3] +
                                                          R(r32, R(r32, -2.0 * g * c.spw) * dxk));
                        gth_prev[5 * kk + 4] = R(r32, gth_prev[5 * kk + 4] +
                                                          R(r32, R(r32, -2.0 * g * c.spw) * dyk));
                        if (bnd)
                            for (int e = 3; e < 5; e++) {
                                double d = (e == 3 ? (double)x : (double)y) - ck[e];
                                double tv = -2.0 * gv * c.spw * d;
                                double et = 2.0 * c.spw * fabs(d) * eg +
                                            2.0 * fabs(gv) * c.spw * (B_DTH * fabs(ck[e]) + fabs(d)) +
                                            5.0 * fabs(tv);
                                bacc_add(&bp, 5 * kk + e, tv, et, 2.0 * c.spw * fabs(d) * mdg);
                            }
                    }
                }
            memcpy(gth, gth_prev, sizeof(double) * 5 * (size_t)K);
            if (bnd)
                for (long i = 0; i < 5L * K; i++) {
                    /* one level: the summation bound of dL/dTheta itself, its
                     * terms counted at their local depth */
                    eth[i] = (plen[i / 5] + B_LOCAL + 16.0) * bp.sa[i];
                    mdth[i] = bp.md[i];
                }
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
                    for (int e = 0; e < 3; e++) {
                        gf[3 * p + e] = R(r32, gf[3 * p + e] + R(r32, gth[5 * kk + e] / cnt[kk]));
                        if (bnd) {
                            double tv = gth[5 * kk + e] / cnt[kk];
                            bacc_add(&bf, 3 * p + e, tv, eth[5 * kk + e] / cnt[kk] + fabs(tv),
                                     mdth[5 * kk + e] / cnt[kk]);
                        }
                    }
                }
            free(cnt);
        }
        for (long p = 0; p < N; p++) {
            for (int e = 0; e < 3; e++) glab[3 * (N * b + p) + e] = gf[3 * p + e];
            double cq = contour[N * b + p];
            double s2 = sigma * sigma;
            double fac = (2.0 * cq / s2) * exp(-(cq * cq) / s2);
            gcontour[N * b + p] = R(r32, gw[p] * (2.0 * cq / s2) * exp(-(cq * cq) / s2));
            if (bnd) {
                for (int e = 0; e < 3; e++) {
                    long o = 3 * (N * b + p) + e;
                    bnd[0][o] = bacc_e(&bf, 3 * p + e) + fabs(gf[3 * p + e]);
                    bnd[1][o] = bf.md[3 * p + e];
                }
                bnd[2][N * b + p] = fabs(fac) * bacc_e(&bw, p) + 2.0 * fabs(gw[p] * fac);
                bnd[3][N * b + p] = fabs(fac) * bw.md[p];
            }
        }
        if (bnd) {
            bacc_free(&bf); bacc_free(&bw); bacc_free(&bq); bacc_free(&bp);
            free(eth); free(mdth); free(ge); free(gmd); free(plen);
        }
        free(th); free(qq); free(zz); free(gf); free(gw); free(gth); free(gth_prev);
        free(gQ); free(ex); free(w); free(w32);
    }
    return 0;
}

/* The plain FP64 chain rule (no cut, no FP32 rounding, no bound). */
int orc_soft_backward(int Bn, int W, int H, int k, const float *lab, const float *contour,
                      double m, double lambda, double sigma, double gamma, double T, int iters,
                      int d32, const double *gq_in, const double *gtheta_in,
                      double *glab, double *gcontour) {
    return orc_soft_backward_ex(Bn, W, H, k, lab, contour, m, lambda, sigma, gamma, T, iters, d32,
                                gq_in, gtheta_in, glab, gcontour, 0, 0, NULL);
}
