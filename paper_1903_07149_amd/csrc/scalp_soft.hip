// scalp_soft.hip -- soft (differentiable) SCALP on gfx950.
//
// An extension of the paper's method: the distance D of Eqs. (1)-(3) over the
// same 3x3 grid-neighbour candidates as Algorithm 1, a softmax with
// temperature T over the candidates instead of the argmin, and soft
// barycenters instead of the hard update.  Paths go to the rounded
// barycenter floor(X_k + 0.5) (no Eq. (4) projection, which needs hard
// membership); the rounding is piecewise constant, so it carries no gradient.
//
// Forward, per iteration:
//   k_soft_assign  workgroup per (image, cell, slice), one pixel per lane:
//                  per-candidate LDS tables of (colour distance, w) and
//                  per-lane path walks as in the hard kernel; writes D and
//                  the factors A (Eq. (1)) and B (Eq. (2)).
//   k_soft_softmax FP64 softmax of -D/T over the 9 slots, written as Q.
//   k_soft_update  workgroup per (image, superpixel): gathers Q over the 3x3
//                  cell block in a fixed order (FP64 partial sums, tree
//                  reduction): deterministic, no atomics.
// Backward, per iteration in reverse:
//   k_soft_bwd_update  thread per pixel: soft-update and softmax backward,
//                      giving dL/dD for the 9 slots.
//   k_soft_bwd_path    workgroup per (image, cell): every (pixel, slot) with a
//                      nonzero dL/dD re-walks its path (samples are recomputed,
//                      never stored), adding the path's two per-sample weights
//                      into LDS tiles; a fold over the tiles then forms dL/df,
//                      dL/dw and the candidates' centre gradients (FP64), which
//                      leave the workgroup as atomics (not bit-reproducible).
#include <algorithm>

#include "scalp_device.h"

namespace scalp {
namespace {

using namespace dev;

struct SoftImg {
    int W, H, nx, ny, K, B;
    int spl;    // work items (slices) per cell of the path kernels
    long long N;
    float spw, gamma, lambda, inv_t;
    double temp;
    int prune;   // 1: skip the walks of slots whose softmax weight is provably 0
};

// A superpixel whose soft mass is below a millionth of a pixel counts as
// empty and keeps its centre (as an empty one does in the hard update).
constexpr double kZMin = 1e-6;

// Softmax weight below which a slot's path terms are left out of the backward.
constexpr float kQMin = 0x1p-24f;

struct SoftCand {
    int k;
    float l, a, b, x, y;
    int cx, cy;
    float dcc, wc;
    int tx0, ty0, tw, th;       // forward: table origin, row pitch, rows; tw == 0: not staged
    int rpp;                    // rows per pass of the column-wise fill (WG / tw, 0 when tw > WG)
    unsigned mag;               // ceil(2^24 / tw): lane tid's first row is tid * mag >> 24
};

struct SoftShared {
    SoftCand cand[9];
};

// Candidates of cell (ci, cj) from theta [K][5]; endpoint = rounded barycenter.
__device__ __forceinline__ void load_candidates(const SoftImg& s, int ci, int cj,
                                                const float* __restrict__ theta,
                                                const float4* __restrict__ img, SoftShared& sh) {
    const int tid = threadIdx.x;
    if (tid < 9) {
        SoftCand c;
        const int ii = ci + tid / 3 - 1, jj = cj + tid % 3 - 1;
        if (ii >= 0 && ii < s.ny && jj >= 0 && jj < s.nx) {
            const int k = ii * s.nx + jj;
            const float* ck = theta + 5LL * k;
            c.k = k;
            c.l = ck[0]; c.a = ck[1]; c.b = ck[2]; c.x = ck[3]; c.y = ck[4];
            c.cx = round_coord(c.x, s.W - 1);
            c.cy = round_coord(c.y, s.H - 1);
            const float4 fc = img[(long long)c.cy * s.W + c.cx];
            c.dcc = colour_dist(fc, c.l, c.a, c.b);
            c.wc = fc.w;
        } else {
            c.k = -1;
            c.l = c.a = c.b = c.x = c.y = 0.0f;
            c.cx = c.cy = 0;
            c.dcc = c.wc = 0.0f;
        }
        sh.cand[tid] = c;
    }
}

// ------------------------------------------------------------------ forward

template <int WG>
__global__ __launch_bounds__(WG) void k_soft_init(SoftImg s, const float4* __restrict__ packed,
                                                  float* __restrict__ theta0) {
    __shared__ double red[6][WG];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / s.K, k = blockIdx.x - b * s.K;
    const int ci = k / s.nx, cj = k - ci * s.nx;
    const int x0 = cell_lo(cj, s.W, s.nx), x1 = cell_lo(cj + 1, s.W, s.nx);
    const int y0 = cell_lo(ci, s.H, s.ny), y1 = cell_lo(ci + 1, s.H, s.ny);
    const float4* img = packed + (long long)b * s.N;
    const int cw = x1 - x0, P = cw * (y1 - y0);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int t = tid; t < P; t += WG) {
        const int r = t / cw;
        const int x = x0 + (t - r * cw), y = y0 + r;
        const float4 f = img[(long long)y * s.W + x];
        acc[0] += f.x; acc[1] += f.y; acc[2] += f.z; acc[3] += x; acc[4] += y; acc[5] += 1.0;
    }
    for (int v = 0; v < 6; ++v) red[v][tid] = acc[v];
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int v = 0; v < 6; ++v) red[v][tid] += red[v][tid + h];
        __syncthreads();
    }
    if (tid < 5) theta0[(5LL * b) * s.K + 5LL * k + tid] = (float)(red[tid][0] / red[5][0]);
}

// One workgroup per (image, cell, slice) work item, one pixel per lane, as
// in the hard assignment: a cell with more pixels than the workgroup has
// lanes is cut into spl slices of whole 64-pixel chunks.  Candidates are
// taken one at a time: the workgroup writes a table of (d_c(q, k), w_q) over
// the rectangle spanned by the item's pixels and the candidate's endpoint
// (two tables alternate, one barrier per candidate), and every lane walks
// its pixel's path over it, two adds per sample; a rectangle beyond the
// budget walks from global memory.  Same FP32 operations, same order.
template <int WG>
__global__ __launch_bounds__(WG) void k_soft_assign(SoftImg s, const float4* __restrict__ packed,
                                                    const float* __restrict__ theta_prev,
                                                    float* __restrict__ q, float* __restrict__ fa,
                                                    float* __restrict__ fb, int cap) {
    extern __shared__ float4 lds_dyn[];
    float2* tabs = reinterpret_cast<float2*>(lds_dyn);          // two tables of cap entries
    __shared__ SoftShared sh;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int bc = item / s.spl, slice = item - bc * s.spl;
    const int b = bc / s.K, cell = bc - b * s.K;
    const int tid = threadIdx.x;
    const int W = s.W, H = s.H;
    const int ci = cell / s.nx, cj = cell - ci * s.nx;
    const int x0 = cell_lo(cj, W, s.nx), x1 = cell_lo(cj + 1, W, s.nx);
    const int y0 = cell_lo(ci, H, s.ny), y1 = cell_lo(ci + 1, H, s.ny);
    const int cw = x1 - x0, ch = y1 - y0, P = cw * ch;
    const int chunks = (P + 63) >> 6;
    const int t0 = 64 * (int)((long long)chunks * slice / s.spl);
    const int t1 = min(P, 64 * (int)((long long)chunks * (slice + 1) / s.spl));
    if (t1 <= t0) return;                                       // uniform: an empty slice
    // columns of the item's pixels: the 8-column strips its range touches
    int ix0 = x0, ix1 = x1;
    if (s.spl > 1) {
        ix0 = x0 + 8 * strip_of(t0, cw, ch);
        ix1 = min(x1, x0 + 8 * strip_of(t1 - 1, cw, ch) + 8);
    }
    const float4* __restrict__ img = packed + (long long)b * s.N;
    load_candidates(s, ci, cj, theta_prev + 5LL * s.K * b, img, sh);
    if (tid < 9) {                                              // the thread that loaded it
        SoftCand& c = sh.cand[tid];
        c.tw = 0;
        c.tx0 = c.ty0 = c.th = 0;
        c.rpp = 0;
        c.mag = 0u;
        if (c.k >= 0) {
            const int tx0 = min(ix0, c.cx), ty0 = min(y0, c.cy);
            const int rwid = max(ix1, c.cx + 1) - tx0, th = max(y1, c.cy + 1) - ty0;
            const int tw = rwid + (24 - rwid % 16) % 16;        // pitch: 8 (mod 16) entries
            if ((long long)tw * th <= cap) {
                c.tx0 = tx0; c.ty0 = ty0; c.tw = tw; c.th = th;
                c.rpp = WG / tw;
                c.mag = (0x1000000u + (unsigned)tw - 1u) / (unsigned)tw;
            }
        }
    }
    const bool mine = tid < t1 - t0;
    int x = 0, y = 0;
    if (mine) {
        cell_pixel(t0 + tid, cw, ch, x, y);
        x += x0;
        y += y0;
    }
    const int p = y * W + x;
    __syncthreads();
    const float lambda = s.lambda, oml = 1.0f - lambda;
    const long long base = 9LL * s.N * b + p;
    int buf = 0;
    // Exact pruning: D >= LB = fl(fl(lambda dcp) + fl(ds spw)) (the hard
    // kernel's bound), and the softmax gives a slot Q = 0 exactly when
    // (D - Dmin) / T > 110 in FP64; Dmin <= best, the smallest D computed so
    // far, and both FP64 steps are monotone, so a slot with
    // (LB - best) / T > 110 gets Q = 0 whatever its walk would give: its D is
    // written as +inf (the softmax maps it to 0) and its saved factors are not
    // written (the backward reads them only where dL/dD, a multiple of Q, is
    // not 0; slots outside the grid likewise).
    // The own cell is visited first, then the edge neighbours, then the
    // corners; each slot is written separately, so the order changes nothing.
    const float4 fown = mine ? img[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float best = INFINITY;
    constexpr unsigned long long kOrder = 0x862075314ULL;   // slots 4, 1, 3, 5, 7, 0, 2, 6, 8
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
        const int j = (int)((kOrder >> (4 * t)) & 15ULL);
        const int k = sh.cand[j].k;
        const long long o = base + (long long)j * s.N;
        if (k < 0) continue;                                    // uniform
        const float l = sh.cand[j].l, a = sh.cand[j].a, bb = sh.cand[j].b;
        const int cx = sh.cand[j].cx, cy = sh.cand[j].cy;
        const int tx0 = sh.cand[j].tx0, ty0 = sh.cand[j].ty0, tw = sh.cand[j].tw;
        const bool staged = tw > 0;
        float2* tab = tabs + (buf ? cap : 0);
        if (staged) {                                           // uniform
            const int rpp = sh.cand[j].rpp;
            if (rpp > 0)                                        // uniform
                fill_table_cols<WG>(tab, img, W, tx0, ty0, tw, sh.cand[j].th, rpp,
                                    sh.cand[j].mag, l, a, bb);
            else
                fill_table<WG>(tab, img, W, tx0, ty0, tw, tw * sh.cand[j].th, l, a, bb);
            __syncthreads();
            buf ^= 1;
        }
        if (!mine) continue;
        const float dcc = sh.cand[j].dcc, wc = sh.cand[j].wc;
        const float ccx = sh.cand[j].x, ccy = sh.cand[j].y;
        const float ex = (float)x - ccx, ey = (float)y - ccy;
        const float ds = ex * ex + ey * ey;
        const float lb = lambda * colour_dist(fown, l, a, bb) + ds * s.spw;
        if (s.prune && ((double)lb - (double)best) / s.temp > 110.0) {
            q[o] = INFINITY;
            continue;
        }
        const int dx = cx - x, dy = cy - y;
        const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
        const int n = adx > ady ? adx : ady;
        const double inv = path_recip(n);
        float dcp, sc, sw;
        if (staged) {
            const int lidx = (y - ty0) * tw + (x - tx0);
            const float2 e0 = tab[lidx];
            dcp = e0.x;
            sc = dcp;
            sw = e0.y;
            walk_table(tab, lidx, tw, dx, dy, sc, sw);
        } else {
            const float4 fp = img[p];
            dcp = colour_dist(fp, l, a, bb);
            sc = dcp;
            sw = fp.w;
            walk_path(img, p, 1, W, dx, dy, l, a, bb, sc, sw);
        }
        if (n > 0) {
            sc = sc + dcc;
            sw = sw + wc;
        }
        float qc, qw;
        div_path_len(sc, sw, n, inv, qc, qw);
        const float A = lambda * dcp + oml * qc;
        const float Bw = 1.0f + s.gamma * qw;
        const float D = A * Bw + ds * s.spw;
        best = fminf(best, D);
        // D goes to the Q buffer (k_soft_softmax turns it into Q); A and B
        // go straight to the saved factors
        q[o] = D;
        fa[o] = A;
        fb[o] = Bw;
    }
}

// Per-pixel soft kernels run a 3D grid: image in z, rows strided over y,
// 256-column segments in x (no per-pixel division to recover coordinates).
#define SOFT_FOR_PIXELS(s)                                                   \
    const int b = blockIdx.z;                                                \
    const int x = blockIdx.x * 256 + threadIdx.x;                            \
    for (int y = blockIdx.y; y < (s).H; y += gridDim.y)                      \
        if (x < (s).W)

// Q_pj = softmax_j(-D_pj / T) in FP64 over the slots inside the grid, rounded
// once to FP32 (the FP32 distances differ by far more than FP32's exponent
// range allows at small T).  In place over the D values.  A separate kernel
// so that the FP64 exponentials do not raise the register count of the path
// walk.
__global__ __launch_bounds__(256) void k_soft_softmax(SoftImg s, float* __restrict__ q) {
    SOFT_FOR_PIXELS(s) {
        const long long p = (long long)y * s.W + x;
        const int ci = cell_of(y, s.ny, s.H), cj = cell_of(x, s.nx, s.W);
        const long long base = 9LL * s.N * b + p;
        float D[9];
        bool ok[9];
        float dmin = INFINITY;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int ii = ci + j / 3 - 1, jj = cj + j % 3 - 1;
            ok[j] = ii >= 0 && ii < s.ny && jj >= 0 && jj < s.nx;
            D[j] = ok[j] ? q[base + (long long)j * s.N] : INFINITY;
            dmin = fminf(dmin, D[j]);
        }
        // a slot with (D - Dmin) / T > 110 has exp < 2^-158: added to the sum
        // (at least 1, the minimum's term) it changes nothing in FP64, and its
        // Q rounds to 0 in FP32, so neither the exponential nor the quotient
        // is computed (same results, most slots at low T)
        double e[9], sum = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const double t = ((double)D[j] - (double)dmin) / s.temp;
            e[j] = ok[j] && t <= 110.0 ? exp(-t) : 0.0;
            sum += e[j];
        }
#pragma unroll
        for (int j = 0; j < 9; ++j)
            q[base + (long long)j * s.N] = e[j] == 0.0 ? 0.0f : (float)(e[j] / sum);
    }
}

template <int WG>
__device__ __forceinline__ void block_sum6(double (&v)[6], double (*red)[WG]) {
    const int tid = threadIdx.x;
    for (int i = 0; i < 6; ++i) red[i][tid] = v[i];
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int i = 0; i < 6; ++i) red[i][tid] += red[i][tid + h];
        __syncthreads();
    }
    for (int i = 0; i < 6; ++i) v[i] = red[i][0];
}

// Soft update of superpixel k: Z = sum Q, f_k = sum Q f / Z, X_k = sum Q X / Z
// over the pixels of the 3x3 cell block around k, each read through the slot
// under which it sees k.
template <int WG>
__global__ __launch_bounds__(WG) void k_soft_update(SoftImg s, const float* __restrict__ q,
                                                    const float4* __restrict__ packed,
                                                    const float* __restrict__ theta_prev,
                                                    float* __restrict__ theta_next,
                                                    double* __restrict__ z) {
    __shared__ double red[6][WG];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / s.K, k = blockIdx.x - b * s.K;
    const int ci = k / s.nx, cj = k - ci * s.nx;
    const int X0 = cell_lo(max(cj - 1, 0), s.W, s.nx), X1 = cell_lo(min(cj + 2, s.nx), s.W, s.nx);
    const int Y0 = cell_lo(max(ci - 1, 0), s.H, s.ny), Y1 = cell_lo(min(ci + 2, s.ny), s.H, s.ny);
    const int bw = X1 - X0, area = bw * (Y1 - Y0);
    const float4* img = packed + (long long)b * s.N;
    const float* qb = q + 9LL * s.N * b;
    // the block's inner cell boundaries: a pixel's cell row is ci - 1 + (y >= yb1)
    // + (y >= yb2), likewise for columns
    const int yb1 = cell_lo(ci, s.H, s.ny), yb2 = cell_lo(ci + 1, s.H, s.ny);
    const int xb1 = cell_lo(cj, s.W, s.nx), xb2 = cell_lo(cj + 1, s.W, s.nx);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    // element e = r * bw + c; lanes step by WG elements = (dr rows, dc columns)
    const int dr = WG / bw, dc = WG - dr * bw;
    int r = tid / bw, c = tid - r * bw;
    // kU elements per trip (e, e + WG, ...: the thread's order is unchanged),
    // their Q loads issued first; a texel is read only where its Q is not 0
    // (at low T most slots underflow to 0, and 0 * f adds exactly nothing)
    constexpr int kU = 4;
    for (int e = tid; e < area; e += kU * WG) {
        int xs[kU], ys[kU];
        long long ps[kU];
        double Qs[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            xs[u] = X0 + c;
            ys[u] = Y0 + r;
            c += dc;
            const bool wrap = c >= bw;
            c -= wrap ? bw : 0;
            r += dr + (wrap ? 1 : 0);
            const int di = (ys[u] >= yb1 ? 1 : 0) + (ys[u] >= yb2 ? 1 : 0);
            const int dj = (xs[u] >= xb1 ? 1 : 0) + (xs[u] >= xb2 ? 1 : 0);
            const int j = (2 - di) * 3 + (2 - dj);  // the pixel's slot that points at k
            ps[u] = (long long)ys[u] * s.W + xs[u];
            Qs[u] = e + u * WG < area ? (double)qb[(long long)j * s.N + ps[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (Qs[u] == 0.0) continue;
            const double Q = Qs[u];
            const float4 f = img[ps[u]];
            acc[0] += Q;
            acc[1] += Q * f.x;
            acc[2] += Q * f.y;
            acc[3] += Q * f.z;
            acc[4] += Q * xs[u];
            acc[5] += Q * ys[u];
        }
    }
    block_sum6<WG>(acc, red);
    if (tid < 5) {
        const long long o = 5LL * s.K * b + 5LL * k + tid;
        theta_next[o] = acc[0] >= kZMin ? (float)(acc[tid + 1] / acc[0]) : theta_prev[o];
    }
    if (tid == 0) z[(long long)s.K * b + k] = acc[0];
}

// ------------------------------------------------------------------ backward

// Per superpixel, what the soft-update backward needs of it, in two float4:
// u = dL/dTheta_k / Z_k (5 values) and v = u . Theta_k, all zero when Z_k is
// below kZMin (such a superpixel kept its centre and passes no gradient to
// Q or f).
__global__ void k_soft_bwd_cand(SoftImg s, const double* __restrict__ z,
                                const float* __restrict__ theta, const double* __restrict__ gth,
                                float4* __restrict__ cand) {
    const long long total = (long long)s.B * s.K;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        float u[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float v = 0.0f;
        const double Zd = z[i];
        if (Zd >= kZMin) {
            for (int c = 0; c < 5; ++c) {
                u[c] = (float)(gth[5 * i + c] / Zd);
                v += u[c] * theta[5 * i + c];
            }
        }
        cand[2 * i] = make_float4(u[0], u[1], u[2], u[3]);
        cand[2 * i + 1] = make_float4(u[4], v, 0.0f, 0.0f);
    }
}

// Soft-update backward (theta_t = sum Q feat / Z) and softmax backward:
// gd[j] = dL/dD_pj (0 where Q_pj < kQMin).  gf += dL/df_p through the update.
// With u, v of k_soft_bwd_cand: dL/dQ_pk += u . feat_p - v and
// dL/df_p += Q_pk u[0..2].
__global__ __launch_bounds__(256) void k_soft_bwd_update(SoftImg s, int first,
                                                         const float* __restrict__ q,
                                                         const float4* __restrict__ cand,
                                                         const float4* __restrict__ packed,
                                                         const float* __restrict__ gq_in,
                                                         float* __restrict__ gd,
                                                         unsigned short* __restrict__ gmask,
                                                         float4* __restrict__ gf) {
    SOFT_FOR_PIXELS(s) {
        const long long p = (long long)y * s.W + x;
        const long long i = (long long)b * s.N + p;
        const int ci = cell_of(y, s.ny, s.H), cj = cell_of(x, s.nx, s.W);
        const float4 f = packed[i];
        const float fx = (float)x, fy = (float)y;
        const long long qb = 9LL * s.N * b + p;
        const float4* cb = cand + 2LL * s.K * b;
        float Q[9], G[9];
        float gfl = 0.0f, gfa = 0.0f, gfb = 0.0f, dot = 0.0f;
#pragma unroll
        for (int j = 0; j < 9; ++j) Q[j] = q[qb + (long long)j * s.N];
        // a slot with Q_pj = 0 adds nothing to the softmax dot product, to
        // dL/df or to dL/dD (Q_pj < 2^-24): its dL/dQ and candidate terms
        // are not loaded
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int ii = ci + j / 3 - 1, jj = cj + j % 3 - 1;
            G[j] = 0.0f;
            if (ii < 0 || ii >= s.ny || jj < 0 || jj >= s.nx || Q[j] == 0.0f) continue;
            if (first) G[j] = gq_in[qb + (long long)j * s.N];
            const int k = ii * s.nx + jj;
            const float4 u = cb[2 * k], u4v = cb[2 * k + 1];
            G[j] += (((u.x * f.x + u.y * f.y) + (u.z * f.z + u.w * fx)) + u4v.x * fy) - u4v.y;
            gfl += u.x * Q[j];
            gfa += u.y * Q[j];
            gfb += u.z * Q[j];
            dot += Q[j] * G[j];
        }
        // A slot's whole path contribution is proportional to Q_pj; below
        // FP32's unit roundoff (2^-24) it is dropped, and the path pass skips
        // the slot (at low T most pixels have one slot above it).  Only the
        // nonzero dL/dD are stored; bit j of the pixel's mask says which.
        unsigned m = 0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const float g = Q[j] < kQMin ? 0.0f : -s.inv_t * Q[j] * (G[j] - dot);
            if (g != 0.0f) {
                gd[qb + (long long)j * s.N] = g;
                m |= 1u << j;
            }
        }
        gmask[i] = (unsigned short)m;
        float4 o = gf[i];
        o.x += gfl;
        o.y += gfa;
        o.z += gfb;
        gf[i] = o;
    }
}

// dL/dTheta_{t-1} starts as the pass-through of superpixels whose soft mass
// was zero (they kept their previous centre) and receives the path terms.
__global__ void k_soft_bwd_pass(SoftImg s, const double* __restrict__ z,
                                const double* __restrict__ gth, double* __restrict__ gth_prev) {
    const long long total = 5LL * s.B * s.K;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x)
        gth_prev[i] = z[i / 5] >= kZMin ? 0.0 : gth[i];
}

// Per wave, a list of (pixel, slot) pairs whose dL/dD is not zero, listed
// chunk by chunk and slot by slot, walked in whole rounds of 64 whenever the
// next slot would overflow its kBwdBatch entries (the rest carried over);
// per slot, seven FP64 sums (the centre gradient's five components, the
// endpoint's two weights) in kBwdCopies copies.
constexpr int kBwdBatch = 192;
constexpr int kBwdCopies = 8;
// Texels per thread and trip of the fold.
constexpr int kFold = 2;

// Where the backward path pass of one work item keeps its tiles: per slot,
// the box [bx0, bx1) x [by0, by1) of the pixels whose path to the slot it
// walks, grown to contain the slot's endpoint, and the offset (in doubles)
// of the slot's FP64 weight tile over that box (-1: the slot's paths scatter
// to global memory instead); one FP32 tile of dL/dw over the union of the
// staged boxes follows the weight tiles.
struct BwdLayout {
    int bx0[9], bx1[9], by0[9], by1[9];
    int has[9];
    int soff[9];
    int ux0, uy0, uw, uh;
    int woff;      // in floats
};

// One workgroup per (image, cell).  Every (pixel, slot) whose dL/dD is not
// zero (at low T about one per pixel) re-walks its path.  Along a path to
// candidate k every sample q receives the same two weights,
//   dL/df_q += cf (f_q - f_k)   with cf = dL/dD * B (1 - lambda) 2 / |P|
//   dL/dw_q += cw               with cw = dL/dD * A gamma / |P|
// (and p itself dL/dD * B lambda 2 (f_p - f_k)), so the walk only adds cf
// into an FP64 tile S_k(q) of the slot (p's lambda term included) and cw
// into the FP32 tile of dL/dw: two LDS atomics per sample and no texel read.
// A fold over the union of the slots' boxes then forms, per texel,
// dL/df_q = sum_k S_k(q) (f_q - f_k) from one texel load, and the centre
// gradient of each candidate, -sum_q S_k(q) (f_q - f_k), in FP64.  The
// spatial part of the centre gradient and the endpoint's weights (every path
// to k ends there) are summed per slot and added once.  A first pass over
// the slot masks of dL/dD sizes the boxes.  Slots whose tiles do not fit the
// budget walk their paths from global memory instead, reading the texels and
// scattering the four gradient floats with float atomics.  The centre
// gradients are summed in FP64 (no FP32 partial sum longer than one path);
// dL/dTheta leaves as FP64 atomics, dL/df and dL/dw as float atomics (not
// bit-reproducible).  At least 4 waves per SIMD (at most 128 VGPRs): two 512-lane
// workgroups per CU, as the LDS budget allows.
template <int WG>
__global__ __launch_bounds__(WG, 4) void k_soft_bwd_path(SoftImg s, const float4* __restrict__ packed,
                                                      const float* __restrict__ theta_prev,
                                                      const float* __restrict__ fa,
                                                      const float* __restrict__ fb,
                                                      const float* __restrict__ gd,
                                                      const unsigned short* __restrict__ gmask,
                                                      float4* __restrict__ gf,
                                                      double* __restrict__ gth_prev, int cap_bytes) {
    extern __shared__ double bwd_dyn[];
    __shared__ SoftShared sh;
    __shared__ BwdLayout bl;
    __shared__ int wl_t[WG / 64][kBwdBatch];              // pixel (see wl_xy) in the cell
    __shared__ unsigned char wl_j[WG / 64][kBwdBatch];    // slot
    __shared__ float wl_g[WG / 64][kBwdBatch];            // dL/dD
    __shared__ double bins[9][7][kBwdCopies];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int b = item / s.K, cell = item - b * s.K;
    const int tid = threadIdx.x;
    const int W = s.W, H = s.H;
    const int ci = cell / s.nx, cj = cell - ci * s.nx;
    const int x0 = cell_lo(cj, W, s.nx), x1 = cell_lo(cj + 1, W, s.nx);
    const int y0 = cell_lo(ci, H, s.ny), y1 = cell_lo(ci + 1, H, s.ny);
    const float4* __restrict__ img = packed + (long long)b * s.N;
    float4* __restrict__ gimg = gf + (long long)b * s.N;
    // the candidates' centres (this pass needs no endpoint texel) are loaded
    // here and stored after the first pass, which does not use them; the
    // slots' boxes start empty and take the endpoint in the layout step
    float cl = 0.0f, ca = 0.0f, cb = 0.0f, cxf = 0.0f, cyf = 0.0f;
    int ck = -1;
    if (tid < 9) {
        const int ii = ci + tid / 3 - 1, jj = cj + tid % 3 - 1;
        if (ii >= 0 && ii < s.ny && jj >= 0 && jj < s.nx) {
            ck = ii * s.nx + jj;
            const float* c5 = theta_prev + 5LL * s.K * b + 5LL * ck;
            cl = c5[0]; ca = c5[1]; cb = c5[2]; cxf = c5[3]; cyf = c5[4];
        }
        bl.bx0[tid] = INT_MAX;
        bl.bx1[tid] = INT_MIN;
        bl.by0[tid] = INT_MAX;
        bl.by1[tid] = INT_MIN;
        bl.has[tid] = 0;
    }
    for (int t = tid; t < 9 * 7 * kBwdCopies; t += WG) (&bins[0][0][0])[t] = 0.0;
    __syncthreads();
    const int cw = x1 - x0, ch = y1 - y0, P = cw * ch;
    const int lane = tid & 63, wave = tid >> 6;
    const int cp = lane & (kBwdCopies - 1);
    const long long base = 9LL * s.N * b;
    // list entries hold the pixel's offsets in the cell as two 16-bit
    // halves when they fit, else its index in the cell's pixel order
    const bool wl_xy = cw < 65536 && ch < 65536;
    // pass 1: the box of each slot's walked pixels (a chunk's box per chunk
    // with any nonzero dL/dD in the slot)
    for (int chunk = wave; chunk * 64 < P; chunk += WG / 64) {
        const int t = chunk * 64 + lane;
        const bool valid = t < P;
        int px = 0, py = 0;
        if (valid) {
            cell_pixel(t, cw, ch, px, py);
            px += x0;
            py += y0;
        }
        int mnx = valid ? px : 0x7fffffff, mxx = valid ? px : -1;
        int mny = valid ? py : 0x7fffffff, mxy = valid ? py : -1;
        for (int o = 32; o > 0; o >>= 1) {
            mnx = min(mnx, __shfl_xor(mnx, o, 64));
            mxx = max(mxx, __shfl_xor(mxx, o, 64));
            mny = min(mny, __shfl_xor(mny, o, 64));
            mxy = max(mxy, __shfl_xor(mxy, o, 64));
        }
        const unsigned msk = valid ? gmask[(long long)b * s.N + (long long)py * W + px] : 0u;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            if (__ballot((msk >> j) & 1u) != 0ULL && lane == 0) {
                atomicMin(&bl.bx0[j], mnx);
                atomicMax(&bl.bx1[j], mxx + 1);
                atomicMin(&bl.by0[j], mny);
                atomicMax(&bl.by1[j], mxy + 1);
                bl.has[j] = 1;
            }
        }
    }
    if (tid < 9) {
        SoftCand c;
        c.k = ck;
        c.l = cl; c.a = ca; c.b = cb; c.x = cxf; c.y = cyf;
        c.cx = ck >= 0 ? round_coord(cxf, W - 1) : 0;
        c.cy = ck >= 0 ? round_coord(cyf, H - 1) : 0;
        c.dcc = c.wc = 0.0f;   // not used by this pass
        sh.cand[tid] = c;
    }
    __syncthreads();
    // tile layout: slots in the order own cell, edges, corners, while they fit
    if (tid == 0) {
        constexpr unsigned long long kOrder = 0x862075314ULL;
        int used = 0;                                           // bytes of weight tiles
        int ux0 = 0x7fffffff, uy0 = 0x7fffffff, ux1 = -1, uy1 = -1;
        for (int t = 0; t < 9; ++t) {
            const int j = (int)((kOrder >> (4 * t)) & 15ULL);
            bl.soff[j] = -1;
            if (sh.cand[j].k < 0 || !bl.has[j]) continue;
            // every path of the slot ends at its endpoint
            bl.bx0[j] = min(bl.bx0[j], sh.cand[j].cx);
            bl.bx1[j] = max(bl.bx1[j], sh.cand[j].cx + 1);
            bl.by0[j] = min(bl.by0[j], sh.cand[j].cy);
            bl.by1[j] = max(bl.by1[j], sh.cand[j].cy + 1);
            const int bw = bl.bx1[j] - bl.bx0[j], bh = bl.by1[j] - bl.by0[j];
            const long long sb = 8LL * bw * bh;
            const int nx0 = min(ux0, bl.bx0[j]), nx1 = max(ux1, bl.bx1[j]);
            const int ny0 = min(uy0, bl.by0[j]), ny1 = max(uy1, bl.by1[j]);
            const long long ub = 4LL * (nx1 - nx0) * (ny1 - ny0);
            if (used + sb + ub <= cap_bytes) {
                bl.soff[j] = used / 8;
                used += (int)sb;
                ux0 = nx0; ux1 = nx1; uy0 = ny0; uy1 = ny1;
            }
        }
        if (ux1 < 0) ux0 = ux1 = uy0 = uy1 = 0;
        bl.ux0 = ux0; bl.uy0 = uy0; bl.uw = ux1 - ux0; bl.uh = uy1 - uy0;
        bl.woff = used / 4;
    }
    __syncthreads();
    float* wtile = reinterpret_cast<float*>(bwd_dyn) + bl.woff;
    const int ux0 = bl.ux0, uy0 = bl.uy0, uw = bl.uw, uh = bl.uh;
    {
        const int words = bl.woff + uw * uh;
        float* z = reinterpret_cast<float*>(bwd_dyn);
        for (int e = tid; e < words; e += WG) z[e] = 0.0f;
    }
    __syncthreads();
    const float lambda = s.lambda, oml = 1.0f - lambda;
    // walks listed pair i of this wave (the lanes of a wave call it together)
    auto walk_pair = [&](int i) {
        const int jj = wl_j[wave][i];
        const float gj = wl_g[wave][i];
        int x, y;
        if (wl_xy) {
            x = wl_t[wave][i] & 0xffff;
            y = wl_t[wave][i] >> 16;
        } else {
            cell_pixel(wl_t[wave][i], cw, ch, x, y);
        }
        x += x0;
        y += y0;
        const int p = y * W + x;
        const SoftCand c = sh.cand[jj];
        const long long o = base + (long long)jj * s.N + p;
        const float A = fa[o], Bw = fb[o];
        const int dx = c.cx - x, dy = c.cy - y;
        const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
        const int n = adx > ady ? adx : ady;
        const float inv_np = 1.0f / (float)(n + 1);
        const float cf = 2.0f * gj * Bw * oml * inv_np;  // per sample, times (f_q - f_k)
        const float cw_ = gj * A * s.gamma * inv_np;     // per sample: dL/dw_q
        const float lf = 2.0f * gj * Bw * lambda;        // lambda term of p
        atomicAdd(&bins[jj][3][cp], (double)(-2.0f * gj * s.spw * ((float)x - c.x)));
        atomicAdd(&bins[jj][4][cp], (double)(-2.0f * gj * s.spw * ((float)y - c.y)));
        const bool xmaj = adx >= ady;
        const int so = bl.soff[jj];
        if (so >= 0) {                                   // staged
            // samples i = 0 .. n-1 (p itself first); the endpoint i = n is
            // added once per slot
            const int sbx0 = bl.bx0[jj], sby0 = bl.by0[jj], sp = bl.bx1[jj] - sbx0;
            double* st = bwd_dyn + so;
            const int stx = dx < 0 ? -1 : 1;
            const int sys = dy < 0 ? -sp : sp, syw = dy < 0 ? -uw : uw;
            const int smaj_s = xmaj ? stx : sys, sdiag_s = smaj_s + (xmaj ? sys : stx);
            const int smaj_w = xmaj ? stx : syw, sdiag_w = smaj_w + (xmaj ? syw : stx);
            int ls = (y - sby0) * sp + (x - sbx0);
            int lw = (y - uy0) * uw + (x - ux0);
            const double cfd = (double)cf;
            if (n > 0) {
                atomicAdd(&st[ls], cfd + (double)lf);
                atomicAdd(&wtile[lw], cw_);
                const unsigned F = step_increment(xmaj ? ady : adx, n);
                unsigned acc = 0x80000000u;
                for (int i = 1; i < n; ++i) {
                    const bool cr = __builtin_add_overflow(acc, F, &acc);
                    ls += cr ? sdiag_s : smaj_s;
                    lw += cr ? sdiag_w : smaj_w;
                    atomicAdd(&st[ls], cfd);
                    atomicAdd(&wtile[lw], cw_);
                }
            } else {
                atomicAdd(&st[ls], (double)lf);
            }
            atomicAdd(&bins[jj][5][cp], cfd);
            atomicAdd(&bins[jj][6][cp], (double)cw_);
        } else {                                         // scatter to global memory
            float gk[3] = {0.0f, 0.0f, 0.0f};
            const float4 fp = img[p];
            const float dl = fp.x - c.l, da = fp.y - c.a, db = fp.z - c.b;
            gk[0] -= lf * dl;
            gk[1] -= lf * da;
            gk[2] -= lf * db;
            const int am = xmaj ? ady : adx;
            const int two_n = 2 * n, inc = 2 * am;
            int rem = n;
            const int stx = dx < 0 ? -1 : 1, sty = dy < 0 ? -W : W;
            const int smaj = xmaj ? stx : sty;
            const int sdiag = smaj + (xmaj ? sty : stx);
            int gi = p;
            unsafeAtomicAdd(&gimg[gi].x, lf * dl);
            unsafeAtomicAdd(&gimg[gi].y, lf * da);
            unsafeAtomicAdd(&gimg[gi].z, lf * db);
            for (int i = 0; i <= n; ++i) {
                if (i > 0) {
                    rem += inc;
                    const bool st_ = rem >= two_n;
                    rem -= st_ ? two_n : 0;
                    gi += st_ ? sdiag : smaj;
                }
                const float4 fq = img[gi];
                const float el = cf * (fq.x - c.l), ea = cf * (fq.y - c.a),
                            eb = cf * (fq.z - c.b);
                unsafeAtomicAdd(&gimg[gi].x, el);
                unsafeAtomicAdd(&gimg[gi].y, ea);
                unsafeAtomicAdd(&gimg[gi].z, eb);
                unsafeAtomicAdd(&gimg[gi].w, cw_);
                gk[0] -= el;
                gk[1] -= ea;
                gk[2] -= eb;
            }
#pragma unroll
            for (int v = 0; v < 3; ++v) atomicAdd(&bins[jj][v][cp], (double)gk[v]);
        }
    };
    // walks pairs [0, upto) of the list, 64 per round; then the list's LDS
    // may be rewritten (a wave's LDS accesses stay in order; the fences keep
    // the compiler from moving them across)
    auto walk_list = [&](int upto) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = lane; i - lane < upto; i += 64)            // uniform trip count
            if (i < upto) walk_pair(i);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // pass 2: list the nonzero pairs and walk them
    int nb = 0;                        // pairs listed and not walked yet (uniform over the wave)
    for (int chunk = wave; chunk * 64 < P; chunk += WG / 64) {
        const int t = chunk * 64 + lane;
        const bool valid = t < P;
        int px = 0, py = 0;
        if (valid) {
            cell_pixel(t, cw, ch, px, py);
            px += x0;
            py += y0;
        }
        const unsigned msk = valid ? gmask[(long long)b * s.N + (long long)py * W + px] : 0u;
        float g[9];
#pragma unroll
        for (int j = 0; j < 9; ++j)
            g[j] = (msk >> j) & 1u ? gd[base + (long long)j * s.N + (long long)py * W + px] : 0.0f;
        const int tag = wl_xy ? (px - x0) | ((py - y0) << 16) : t;
#pragma unroll 1
        for (int jn = 0; jn < 9; ++jn) {                        // uniform
            float gj = 0.0f;
#pragma unroll
            for (int j = 0; j < 9; ++j) gj = j == jn ? g[j] : gj;
            const unsigned long long m = __ballot(gj != 0.0f);
            const int cnt = __popcll(m);
            if (nb + cnt > kBwdBatch) {                         // uniform: make room
                // walk the whole rounds, move the rest (< 64 pairs) to the front
                const int full = nb & ~63;
                walk_list(full);
                const int left = nb - full;
                int lt = 0, lj = 0;
                float lg = 0.0f;
                if (lane < left) {
                    lt = wl_t[wave][full + lane];
                    lj = wl_j[wave][full + lane];
                    lg = wl_g[wave][full + lane];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < left) {
                    wl_t[wave][lane] = lt;
                    wl_j[wave][lane] = (unsigned char)lj;
                    wl_g[wave][lane] = lg;
                }
                nb = left;
            }
            if (gj != 0.0f) {
                const int at = nb + (int)__builtin_amdgcn_mbcnt_hi(
                                       (unsigned)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                wl_t[wave][at] = tag;
                wl_j[wave][at] = (unsigned char)jn;
                wl_g[wave][at] = gj;
            }
            nb += cnt;
        }
    }
    walk_list(nb);
    __syncthreads();
    // the endpoint's weights, once per staged slot (one writer per weight
    // tile entry; two candidates may round to the same endpoint pixel, so
    // the shared dL/dw tile takes an atomic)
    if (tid < 9 && bl.soff[tid] >= 0) {
        const SoftCand c = sh.cand[tid];
        double vc = 0.0, vw = 0.0;
        for (int k = 0; k < kBwdCopies; ++k) {
            vc += bins[tid][5][k];
            vw += bins[tid][6][k];
        }
        const int sp = bl.bx1[tid] - bl.bx0[tid];
        bwd_dyn[bl.soff[tid] + (c.cy - bl.by0[tid]) * sp + (c.cx - bl.bx0[tid])] += vc;
        atomicAdd(&wtile[(c.cy - uy0) * uw + (c.cx - ux0)], (float)vw);
    }
    __syncthreads();
    // fold over the union box, kFold texels per thread and trip with their
    // texel loads issued first: dL/df_q = sum_k S_k(q) (f_q - f_k) (FP64, one
    // rounding) and dL/dw_q; the centre gradients -sum_q S_k(q) (f_q - f_k)
    // go to the FP64 slot sums term by term
    {
        const int area = uw * uh;
        const int dr = uw > 0 ? WG / uw : 0, dc = uw > 0 ? WG - dr * uw : 0;
        int r = uw > 0 ? tid / uw : 0, c = tid - r * uw;
        for (int e0 = tid; e0 < area; e0 += kFold * WG) {
            int xs[kFold], ys[kFold];
            float4 fs[kFold];
#pragma unroll
            for (int u = 0; u < kFold; ++u) {
                xs[u] = ux0 + c;
                ys[u] = uy0 + r;
                if (e0 + u * WG < area) fs[u] = img[(long long)ys[u] * W + xs[u]];
                c += dc;
                const bool wrap = c >= uw;
                c -= wrap ? uw : 0;
                r += dr + (wrap ? 1 : 0);
            }
#pragma unroll
            for (int u = 0; u < kFold; ++u) {
                const int e = e0 + u * WG;
                if (e >= area) break;
                const int x = xs[u], y = ys[u];
                const float4 f = fs[u];
                const float wv = wtile[e];
                double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    const int so = bl.soff[j];
                    if (so < 0) continue;
                    if (x < bl.bx0[j] || x >= bl.bx1[j] || y < bl.by0[j] || y >= bl.by1[j])
                        continue;
                    const double sv = bwd_dyn[so + (y - bl.by0[j]) * (bl.bx1[j] - bl.bx0[j]) +
                                              (x - bl.bx0[j])];
                    if (sv == 0.0) continue;
                    const double el = sv * (double)(f.x - sh.cand[j].l);
                    const double ea = sv * (double)(f.y - sh.cand[j].a);
                    const double eb = sv * (double)(f.z - sh.cand[j].b);
                    ax += el;
                    ay += ea;
                    az += eb;
                    atomicAdd(&bins[j][0][cp], -el);
                    atomicAdd(&bins[j][1][cp], -ea);
                    atomicAdd(&bins[j][2][cp], -eb);
                }
                if (ax != 0.0 || ay != 0.0 || az != 0.0 || wv != 0.0f) {
                    float4* d = &gimg[(long long)y * W + x];
                    unsafeAtomicAdd(&d->x, (float)ax);
                    unsafeAtomicAdd(&d->y, (float)ay);
                    unsafeAtomicAdd(&d->z, (float)az);
                    unsafeAtomicAdd(&d->w, wv);
                }
            }
        }
    }
    __syncthreads();
    // the centre gradients
    if (tid < 9) {
        const SoftCand c = sh.cand[tid];
        if (c.k >= 0) {
            for (int q = 0; q < 5; ++q) {
                double a = 0.0;
                for (int k = 0; k < kBwdCopies; ++k) a += bins[tid][q][k];
                if (a != 0.0) unsafeAtomicAdd(&gth_prev[5LL * s.K * b + 5LL * c.k + q], a);
            }
        }
    }
}

// Theta_0 = cell means: dL/df_p += dL/dTheta_0 / |cell|; then the outputs:
// dL/dlab = dL/df and dL/dC = dL/dw * 2C/sigma^2 exp(-C^2/sigma^2).
__global__ __launch_bounds__(256) void k_soft_bwd_finish(SoftImg s, const float4* __restrict__ gf,
                                                         const double* __restrict__ gth0,
                                                         const float* __restrict__ contour,
                                                         float sigma, float* __restrict__ glab,
                                                         float* __restrict__ gcon) {
    const double s2 = (double)sigma * (double)sigma;
    SOFT_FOR_PIXELS(s) {
        const long long p = (long long)y * s.W + x;
        const long long i = (long long)b * s.N + p;
        const int ci = cell_of(y, s.ny, s.H), cj = cell_of(x, s.nx, s.W);
        const int cnt = (cell_lo(cj + 1, s.W, s.nx) - cell_lo(cj, s.W, s.nx)) *
                        (cell_lo(ci + 1, s.H, s.ny) - cell_lo(ci, s.H, s.ny));
        const double* g0 = gth0 + 5LL * s.K * b + 5LL * (ci * s.nx + cj);
        const float4 v = gf[i];
        glab[3 * i] = v.x + (float)(g0[0] / cnt);
        glab[3 * i + 1] = v.y + (float)(g0[1] / cnt);
        glab[3 * i + 2] = v.z + (float)(g0[2] / cnt);
        const double c = contour[i];
        gcon[i] = (float)((double)v.w * (2.0 * c / s2) * exp(-(c * c) / s2));
    }
}

__global__ void k_widen_f32(const float* __restrict__ src, double* __restrict__ dst, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

constexpr int kSoftWG = 256;
constexpr int kSoftBwdWG = 512;
// Tile budget of the backward path pass in bytes (FP64 weight tiles plus the
// FP32 dL/dw tile): with its ~18 KiB of static LDS (the waves' pair lists,
// the slot sums, the layout, the candidates) two 512-lane workgroups still
// fit in a CU's 160 KiB.  Slots beyond it scatter to global memory instead.
constexpr int kBwdLdsBytes = 60 * 1024;

unsigned grid_for(long long n) {
    return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65536));
}

}  // namespace

SoftGeom soft_geom(int W, int H, int nx, int ny, int B, float spw, float gamma, float lambda,
                   float temperature, int wg, int prune) {
    SoftGeom g;
    g.W = W; g.H = H; g.nx = nx; g.ny = ny; g.B = B; g.wg = wg;
    g.spw = spw; g.gamma = gamma; g.lambda = lambda; g.temperature = temperature;
    g.prune = prune;
    return g;
}

// Grid of the per-pixel soft kernels: about 4096 blocks over all images.
static dim3 pixel_grid(const SoftImg& s) {
    const int bx = (s.W + 255) / 256;
    const int by = std::max(1, std::min(s.H, 4096 / std::max(1, bx * s.B)));
    return dim3((unsigned)bx, (unsigned)std::min(by, 65535), (unsigned)s.B);
}

int soft_slices(int W, int H, int nx, int ny, int wg) {
    const long long cw = (W + nx - 1) / nx, ch = (H + ny - 1) / ny;
    const long long chunks = (cw * ch + 63) / 64, per = wg / 64;
    return (int)std::max<long long>(1, (chunks + per - 1) / per);
}

static SoftImg to_img(const SoftGeom& g) {
    SoftImg s;
    s.W = g.W; s.H = g.H; s.nx = g.nx; s.ny = g.ny; s.K = g.nx * g.ny; s.B = g.B;
    s.N = (long long)g.W * g.H;
    s.spl = soft_slices(g.W, g.H, g.nx, g.ny, g.wg);
    s.spw = g.spw; s.gamma = g.gamma; s.lambda = g.lambda; s.inv_t = 1.0f / g.temperature;
    s.temp = (double)g.temperature;
    s.prune = g.prune;
    return s;
}

void lift_soft_lds_limits() {
    const size_t cap = 160 * 1024 - sizeof(SoftShared) - 64;
    for (const void* k : {reinterpret_cast<const void*>(k_soft_assign<256>),
                          reinterpret_cast<const void*>(k_soft_assign<512>),
                          reinterpret_cast<const void*>(k_soft_assign<1024>)}) {
        static_cast<void>(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)cap));
        static_cast<void>(hipGetLastError());
    }
    static_cast<void>(hipFuncSetAttribute(
        reinterpret_cast<const void*>(k_soft_bwd_path<kSoftBwdWG>),
        hipFuncAttributeMaxDynamicSharedMemorySize, kBwdLdsBytes));
    static_cast<void>(hipGetLastError());
}

int launch_soft_init(const SoftGeom& g, const float4* packed, float* theta0, hipStream_t st) {
    const SoftImg s = to_img(g);
    hipLaunchKernelGGL(k_soft_init<kSoftWG>, dim3(s.B * s.K), dim3(kSoftWG), 0, st, s, packed,
                       theta0);
    return hipGetLastError();
}

template <int WG>
static int soft_assign_t(const SoftImg& s, const float4* packed, const float* theta_prev, float* q,
                         float* fa, float* fb, int cap, hipStream_t st) {
    hipLaunchKernelGGL(k_soft_assign<WG>, dim3(s.B * s.K * s.spl), dim3(WG), (size_t)cap * sizeof(float4),
                       st, s, packed, theta_prev, q, fa, fb, cap);
    return hipGetLastError();
}

int launch_soft_assign(const SoftGeom& g, const float4* packed, const float* theta_prev, float* q,
                       float* fa, float* fb, int cap, hipStream_t st) {
    const SoftImg s = to_img(g);
    int e;
    if (g.wg == 1024) e = soft_assign_t<1024>(s, packed, theta_prev, q, fa, fb, cap, st);
    else if (g.wg == 512) e = soft_assign_t<512>(s, packed, theta_prev, q, fa, fb, cap, st);
    else e = soft_assign_t<256>(s, packed, theta_prev, q, fa, fb, cap, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_softmax, pixel_grid(s), dim3(256), 0, st, s, q);
    return hipGetLastError();
}

int launch_soft_update(const SoftGeom& g, const float* q, const float4* packed,
                       const float* theta_prev, float* theta_next, double* z, hipStream_t st) {
    const SoftImg s = to_img(g);
    hipLaunchKernelGGL(k_soft_update<kSoftWG>, dim3(s.B * s.K), dim3(kSoftWG), 0, st, s, q, packed,
                       theta_prev, theta_next, z);
    return hipGetLastError();
}

int launch_soft_bwd_update(const SoftGeom& g, int first, const float* q, const double* z,
                           const float* theta, const float4* packed, const double* gth,
                           const float* gq_in, float* gd, unsigned short* gmask, float4* gf,
                           float4* cand, hipStream_t st) {
    const SoftImg s = to_img(g);
    hipLaunchKernelGGL(k_soft_bwd_cand, dim3(grid_for((long long)s.B * s.K)), dim3(256), 0, st, s,
                       z, theta, gth, cand);
    hipLaunchKernelGGL(k_soft_bwd_update, pixel_grid(s), dim3(256), 0, st, s, first, q, cand,
                       packed, gq_in, gd, gmask, gf);
    return hipGetLastError();
}

int launch_soft_bwd_pass(const SoftGeom& g, const double* z, const double* gth, double* gth_prev,
                         hipStream_t st) {
    const SoftImg s = to_img(g);
    hipLaunchKernelGGL(k_soft_bwd_pass, dim3(grid_for(5LL * s.B * s.K)), dim3(256), 0, st, s, z,
                       gth, gth_prev);
    return hipGetLastError();
}

template <int WG>
static int soft_bwd_path_t(const SoftImg& s, const float4* packed, const float* theta_prev,
                           const float* fa, const float* fb, const float* gd,
                           const unsigned short* gmask, float4* gf, double* gth_prev,
                           int cap_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_soft_bwd_path<WG>, dim3(s.B * s.K), dim3(WG), (size_t)cap_bytes, st, s,
                       packed, theta_prev, fa, fb, gd, gmask, gf, gth_prev, cap_bytes);
    return hipGetLastError();
}

int launch_soft_bwd_path(const SoftGeom& g, const float4* packed, const float* theta_prev,
                         const float* fa, const float* fb, const float* gd,
                         const unsigned short* gmask, float4* gf, double* gth_prev,
                         int cap_bytes, hipStream_t st) {
    // one shape for the backward pass whatever the assignment's (512 lanes;
    // a cell's work is split over its 64-pixel chunks, one wave each)
    return soft_bwd_path_t<kSoftBwdWG>(to_img(g), packed, theta_prev, fa, fb, gd, gmask, gf,
                                       gth_prev, std::min(cap_bytes, kBwdLdsBytes) & ~7, st);
}

int launch_soft_bwd_finish(const SoftGeom& g, const float4* gf, const double* gth0,
                           const float* contour, float sigma, float* glab, float* gcon,
                           hipStream_t st) {
    const SoftImg s = to_img(g);
    hipLaunchKernelGGL(k_soft_bwd_finish, pixel_grid(s), dim3(256), 0, st, s, gf, gth0,
                       contour, sigma, glab, gcon);
    return hipGetLastError();
}

int launch_widen_f32(const float* src, double* dst, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_widen_f32, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace scalp
