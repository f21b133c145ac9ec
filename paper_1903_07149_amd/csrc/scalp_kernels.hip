// scalp_kernels.hip -- HIP kernels (gfx950) of the SCALP clustering path.
//
//   k_prepare         packs (l, a, b, w) with w = 1 - exp(-C^2/sigma^2), the
//                     summand of Eq. (2), evaluated in FP64 and rounded once.
//   k_init_cells      Algorithm 1 initialisation: labels = grid cell, per-cell
//                     integer sums (Sec. II-A regular grid).
//   k_assign*         Algorithm 1 assignment: one workgroup per (cell, slice)
//                     work item, one pixel per lane.  For each of the <= 9
//                     candidates in turn the workgroup writes an LDS table of
//                     (colour distance, w) over the rectangle of the item and
//                     the candidate's endpoint; every lane then walks the
//                     discrete line (Sec. II-B) from its pixel to the endpoint
//                     over the table, accumulating Eq. (1)'s colour term and
//                     Eq. (2)'s contour term in a fixed FP32 order, forms D of
//                     Eq. (3) and keeps the first strict minimum.  A lane
//                     skips the walk of a candidate whose exact lower bound
//                     on D (colour at the pixel and spatial term only) cannot
//                     win, which leaves the labels unchanged.  With ACCUM
//                     the update's sums are fused in: each pixel can only
//                     choose among the cell's 9 candidates, so they reduce
//                     into 9 LDS bins and leave the workgroup as at most 54
//                     integer atomics.
//   k_finalize*       Algorithm 1 update: means from the integer sums, the
//                     rounded barycenter, and the membership test of the
//                     Sec. II-D Remark; clusters that fail it are queued.
//   k_project*        Eq. (4): nearest member pixel of each queued cluster.
//
// All FP32 arithmetic of the distance is written operation by operation and
// compiled with -ffp-contract=off, so it matches the plain CPU definition
// bit for bit.
#include <algorithm>

#include "scalp_device.h"

namespace scalp {
namespace {

using namespace dev;


struct Cand {
    int k;            // superpixel index within the image, -1 outside the grid
    float l, a, b, x, y;
    int cx, cy;       // path endpoint
    float dcc, wc;    // colour distance and w of the endpoint sample
    int tx0, ty0, tw, th;   // its LDS table: origin, row pitch, rows; tw == 0: paths read global memory
    int rpp;                // rows per pass of the column-wise fill (WG / tw, 0 when tw > WG)
    unsigned mag;           // ceil(2^24 / tw): lane tid's first row is tid * mag >> 24
};

// Copies of the update bins: the lanes of a wave mostly pick the same
// candidate, and 64-bit LDS atomics on one word serialise, so lane t adds to
// copy (t ^ (t >> 3)) mod kBinCopies: every row and every column of the
// wave's 8x8 pixel block spreads over all copies, and at most 8 lanes of a
// wave share one word.
constexpr int kBinCopies = 8;

// Per work item: the candidates and the update bins, [slot * 6 + sum][copy].
struct CellShared {
    Cand cand[9];
    int box[9][4];    // voted tables: per slot, min x, min y, max x, max y of the waves that walk it
    unsigned long long bins[9 * 6][kBinCopies];
};

// Work item (cell, slice): pixels [t0, t1) of the cell in cell_pixel order,
// one per lane.  The cell's ceil(P / 64) 64-pixel chunks are split evenly
// over its spl slices (spl is chosen on the host so that no slice has more
// than WG pixels), and every wave keeps an 8x8 block.
//
// Candidates are taken one at a time, the pixel's own cell first, then the
// four edge neighbours, then the corners; the winner is the smallest
// (D, slot) pair, which is the first strict minimum in ascending slot (hence
// ascending k) whatever the visiting order.  A lane skips a candidate whose
// lower bound fl(fl(lambda dcp) + fl(ds spw)) cannot beat the current best
// pair: with lambda in [0, 1], gamma >= 0 and every colour distance and w
// non-negative, A >= fl(lambda dcp) and B >= 1 in Eqs. (1)-(2), so
// D = fl(fl(A B) + fl(ds spw)) is at least that bound (FP32 rounding is
// monotone) and the skipped D could not have been chosen.  The labels are
// those of evaluating every candidate; a wave skips the walk when all of its
// lanes do (a NaN bound never skips).
// For candidate j the workgroup first writes, for every texel q of the
// rectangle spanned by the item's pixels and j's endpoint (every path to j
// lies inside it), the pair (d_c(q, j), w_q) into an LDS table; lanes then
// walk their paths over the table, two adds per sample.  Two tables
// alternate, so one barrier per candidate separates writing a table from
// reading it and reading it from overwriting it.  A candidate whose
// rectangle exceeds the budget (cap entries) walks its paths from global
// memory, computing d_c per sample.  All of these give the same FP32 values
// in the same order as the plain definition.
template <int WG, bool ACCUM, bool VOTED>
__device__ __forceinline__ void process_cell(const Img& im, int cell, int slice,
                                             const float4* __restrict__ packed,
                                             const float* __restrict__ centres,
                                             const int* __restrict__ endpoints,
                                             int* __restrict__ labels,
                                             long long* __restrict__ acc, float lambda, int cap,
                                             float2* lds, CellShared& sh) {
    const int tid = threadIdx.x;
    const int W = im.W, H = im.H, nx = im.nx, ny = im.ny;
    const int ci = cell / nx, cj = cell - ci * nx;
    const int x0 = cell_lo(cj, W, nx), x1 = cell_lo(cj + 1, W, nx);
    const int y0 = cell_lo(ci, H, ny), y1 = cell_lo(ci + 1, H, ny);
    const float4* __restrict__ img = packed + im.pix;
    const int cw = x1 - x0, ch = y1 - y0;
    const int P = cw * ch;
    const int spl = im.spl;
    const int chunks = (P + 63) >> 6;
    const int t0 = 64 * (int)((long long)chunks * slice / spl);
    const int t1 = min(P, 64 * (int)((long long)chunks * (slice + 1) / spl));
    // columns of the item's pixels: the 8-column strips its range touches
    int ix0 = x0, ix1 = x1;
    if (spl > 1 && t1 > t0) {
        ix0 = x0 + 8 * strip_of(t0, cw, ch);
        ix1 = min(x1, x0 + 8 * strip_of(t1 - 1, cw, ch) + 8);
    }

    if (tid < 9) {
        Cand c;
        const int ii = ci + tid / 3 - 1, jj = cj + tid % 3 - 1;
        c.tw = 0;
        c.tx0 = c.ty0 = c.th = 0;
        c.rpp = 0;
        c.mag = 0u;
        if (ii >= 0 && ii < ny && jj >= 0 && jj < nx) {
            const int k = ii * nx + jj;
            const float* ck = centres + 5LL * (im.sp + k);
            c.k = k;
            c.l = ck[0]; c.a = ck[1]; c.b = ck[2]; c.x = ck[3]; c.y = ck[4];
            // endpoints outside the image are clamped into it
            c.cx = min(max(endpoints[2LL * (im.sp + k)], 0), W - 1);
            c.cy = min(max(endpoints[2LL * (im.sp + k) + 1], 0), H - 1);
            const float4 fc = img[(long long)c.cy * W + c.cx];
            c.dcc = colour_dist(fc, c.l, c.a, c.b);
            c.wc = fc.w;
            const int ax0 = min(ix0, c.cx), ax1 = max(ix1, c.cx + 1);
            const int ay0 = min(y0, c.cy), ay1 = max(y1, c.cy + 1);
            // row pitch = 8 (mod 16) entries: the 8 rows of a wave's 8x8
            // block then start on 4 different quarters of the LDS banks
            const int pitch = (ax1 - ax0) + ((24 - (ax1 - ax0) % 16) % 16);
            if ((long long)pitch * (ay1 - ay0) <= cap) {
                c.tx0 = ax0; c.ty0 = ay0; c.tw = pitch; c.th = ay1 - ay0;
                c.rpp = WG / pitch;
                c.mag = (0x1000000u + (unsigned)pitch - 1u) / (unsigned)pitch;
            }
        } else {
            c.k = -1;
            c.l = c.a = c.b = c.x = c.y = 0.0f;
            c.cx = c.cy = 0;
            c.dcc = c.wc = 0.0f;
        }
        sh.cand[tid] = c;
    }
    if (VOTED && tid < 36) (&sh.box[0][0])[tid] = (tid & 2) ? INT_MIN : INT_MAX;
    if (ACCUM) {
        for (int t = tid; t < 54 * kBinCopies; t += WG) (&sh.bins[0][0])[t] = 0ULL;
    }
    __syncthreads();

    const float oml = 1.0f - lambda;
    const float gamma = im.gamma, spw = im.spw;
    const bool mine = tid < t1 - t0;               // this lane's pixel exists
    int x = 0, y = 0;
    if (mine) {
        cell_pixel(t0 + tid, cw, ch, x, y);
        x += x0;
        y += y0;
    }
    float best = INFINITY;
    int bestj = -1;
    int buf = 0;
    // the pixel's own texel, for the lower bounds
    const float4 fown = mine ? img[(long long)y * W + x] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    constexpr unsigned long long kOrder = 0x862075314ULL;   // slots 4, 1, 3, 5, 7, 0, 2, 6, 8
    if constexpr (VOTED) {
    // Voted tables: before each candidate's table is filled, the waves with
    // a lane that walks it report the box of their pixels; the table covers
    // that box and the endpoint, in one buffer of twice the entries (the
    // vote's barrier already orders the previous candidate's walks before
    // the fill), and is not filled at all when no lane walks.  Two barriers
    // per candidate instead of one, in return for smaller fills and more
    // tables within the budget (cells much larger than the workgroup).
    const int wx0 = wave_min_i32(mine ? x : INT_MAX), wy0 = wave_min_i32(mine ? y : INT_MAX);
    const int wx1 = wave_max_i32(mine ? x : INT_MIN), wy1 = wave_max_i32(mine ? y : INT_MIN);
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
        const int j = (int)((kOrder >> (4 * t)) & 15ULL);
        const int k = sh.cand[j].k;
        if (k < 0) continue;                       // uniform
        const float l = sh.cand[j].l, a = sh.cand[j].a, b = sh.cand[j].b;
        const int cx = sh.cand[j].cx, cy = sh.cand[j].cy;
        const float ccx = sh.cand[j].x, ccy = sh.cand[j].y;
        const float ex = (float)x - ccx;
        const float ey = (float)y - ccy;
        const float ds = ex * ex + ey * ey;
        const float lb = lambda * colour_dist(fown, l, a, b) + ds * spw;   // <= D
        const bool walks = mine && !(im.prune && (lb > best || (lb == best && j > bestj)));
        if (__ballot(walks) != 0ULL && (tid & 63) == 0) {
            atomicMin(&sh.box[j][0], wx0);
            atomicMin(&sh.box[j][1], wy0);
            atomicMax(&sh.box[j][2], wx1);
            atomicMax(&sh.box[j][3], wy1);
        }
        __syncthreads();   // the box is complete, and every wave is done with the table
        const int bx0 = __builtin_amdgcn_readfirstlane(sh.box[j][0]);
        const int bx1 = __builtin_amdgcn_readfirstlane(sh.box[j][2]);
        if (bx0 > bx1) continue;                   // uniform: no lane of the item walks j
        const int by0 = __builtin_amdgcn_readfirstlane(sh.box[j][1]);
        const int by1 = __builtin_amdgcn_readfirstlane(sh.box[j][3]);
        const int tx0 = min(bx0, cx), tx1 = max(bx1, cx) + 1;
        const int ty0 = min(by0, cy), ty1 = max(by1, cy) + 1;
        const int tw = (tx1 - tx0) + ((24 - (tx1 - tx0) % 16) % 16);
        const bool staged = (long long)tw * (ty1 - ty0) <= 2LL * cap;   // uniform
        if (staged) {
            if (tw <= WG)                          // uniform
                fill_table_cols<WG>(lds, img, W, tx0, ty0, tw, ty1 - ty0, WG / tw,
                                    (0x1000000u + (unsigned)tw - 1u) / (unsigned)tw, l, a, b);
            else
                fill_table<WG>(lds, img, W, tx0, ty0, tw, tw * (ty1 - ty0), l, a, b);
            __syncthreads();
        }
        if (walks) {
            const float dcc = sh.cand[j].dcc, wc = sh.cand[j].wc;
            const int dx = cx - x, dy = cy - y;
            const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
            const int n = adx > ady ? adx : ady;
            const double inv = path_recip(n);
            float dcp, sc, sw;
            if (staged) {
                const int lidx = (y - ty0) * tw + (x - tx0);
                const float2 e0 = lds[lidx];
                dcp = e0.x;
                sc = dcp;                          // sample i = 0 is p itself
                sw = e0.y;
                walk_table(lds, lidx, tw, dx, dy, sc, sw);
            } else {
                const int p = y * W + x;
                const float4 fp = img[p];
                dcp = colour_dist(fp, l, a, b);
                sc = dcp;
                sw = fp.w;
                walk_path(img, p, 1, W, dx, dy, l, a, b, sc, sw);
            }
            if (n > 0) {                           // sample i = n is the endpoint
                sc = sc + dcc;
                sw = sw + wc;
            }
            float qc, qw;                          // sc / |P|, sw / |P|
            div_path_len(sc, sw, n, inv, qc, qw);
            const float A = lambda * dcp + oml * qc;             // Eq. (1)
            const float B = 1.0f + gamma * qw;                   // Eq. (2)
            const float D = A * B + ds * spw;                    // Eq. (3)
            if (D < best || (D == best && j < bestj)) {
                best = D;
                bestj = j;
            }
        }
    }
    } else {
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
        const int j = (int)((kOrder >> (4 * t)) & 15ULL);
        const int k = sh.cand[j].k;
        if (k < 0) continue;                       // uniform
        const float l = sh.cand[j].l, a = sh.cand[j].a, b = sh.cand[j].b;
        const int cx = sh.cand[j].cx, cy = sh.cand[j].cy;
        const int tw = sh.cand[j].tw, tx0 = sh.cand[j].tx0, ty0 = sh.cand[j].ty0;
        float2* tab = lds + (buf ? cap : 0);
        if (tw > 0) {                              // uniform
            const int rpp = sh.cand[j].rpp;
            if (rpp > 0)                           // uniform
                fill_table_cols<WG>(tab, img, W, tx0, ty0, tw, sh.cand[j].th, rpp,
                                    sh.cand[j].mag, l, a, b);
            else
                fill_table<WG>(tab, img, W, tx0, ty0, tw, tw * sh.cand[j].th, l, a, b);
            __syncthreads();
            buf ^= 1;
        }
        const float ccx = sh.cand[j].x, ccy = sh.cand[j].y;
        const float dcc = sh.cand[j].dcc, wc = sh.cand[j].wc;
        const float ex = (float)x - ccx;
        const float ey = (float)y - ccy;
        const float ds = ex * ex + ey * ey;
        const float lb = lambda * colour_dist(fown, l, a, b) + ds * spw;   // <= D
        if (mine && !(im.prune && (lb > best || (lb == best && j > bestj)))) {
            const int dx = cx - x, dy = cy - y;
            const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
            const int n = adx > ady ? adx : ady;
            const double inv = path_recip(n);
            float dcp, sc, sw;
            if (tw > 0) {
                const int lidx = (y - ty0) * tw + (x - tx0);
                const float2 e0 = tab[lidx];
                dcp = e0.x;
                sc = dcp;                          // sample i = 0 is p itself
                sw = e0.y;
                walk_table(tab, lidx, tw, dx, dy, sc, sw);
            } else {
                const int p = y * W + x;
                const float4 fp = img[p];
                dcp = colour_dist(fp, l, a, b);
                sc = dcp;
                sw = fp.w;
                walk_path(img, p, 1, W, dx, dy, l, a, b, sc, sw);
            }
            if (n > 0) {                           // sample i = n is the endpoint
                sc = sc + dcc;
                sw = sw + wc;
            }
            float qc, qw;                          // sc / |P|, sw / |P|
            div_path_len(sc, sw, n, inv, qc, qw);
            const float A = lambda * dcp + oml * qc;             // Eq. (1)
            const float B = 1.0f + gamma * qw;                   // Eq. (2)
            const float D = A * B + ds * spw;                    // Eq. (3)
            if (D < best || (D == best && j < bestj)) {
                best = D;
                bestj = j;
            }
        }
    }
    }

    if (mine) {
        const int p = y * W + x;
        const int bj = bestj < 0 ? 4 : bestj;   // bestj < 0 only with non-finite input
        labels[im.pix + p] = sh.cand[bj].k;
        if (ACCUM) {
            const float4 fp = img[p];
            const int cp = (tid ^ (tid >> 3)) & (kBinCopies - 1);
            unsigned long long(*bin)[kBinCopies] = sh.bins + 6 * bj;
            atomicAdd(&bin[0][cp], 1ULL);
            atomicAdd(&bin[1][cp], (unsigned long long)x);
            atomicAdd(&bin[2][cp], (unsigned long long)y);
            atomicAdd(&bin[3][cp], (unsigned long long)to_fixed(fp.x));
            atomicAdd(&bin[4][cp], (unsigned long long)to_fixed(fp.y));
            atomicAdd(&bin[5][cp], (unsigned long long)to_fixed(fp.z));
        }
    }
    if (ACCUM) {
        __syncthreads();
        if (tid < 54) {
            const int j = tid / 6;
            const int k = sh.cand[j].k;
            unsigned long long n = 0, v = 0;
            for (int c = 0; c < kBinCopies; ++c) {
                n += sh.bins[6 * j][c];
                v += sh.bins[tid][c];
            }
            if (k >= 0 && n != 0ULL)
                atomicAdd((unsigned long long*)(acc + kAccStride * (long long)(im.sp + k) +
                                                (tid - 6 * j)),
                          v);
        }
    }
    __syncthreads();   // shared state is reused by the next cell of a persistent workgroup
}

template <int WG, bool ACCUM, bool VOTED>
__global__ __launch_bounds__(WG) void k_assign(Img im, const float4* __restrict__ packed,
                                               const float* __restrict__ centres,
                                               const int* __restrict__ endpoints,
                                               int* __restrict__ labels,
                                               long long* __restrict__ acc, int* ctrl,
                                               float lambda, int cap) {
    extern __shared__ float2 tab_dyn[];
    __shared__ CellShared sh;
    if (ACCUM && blockIdx.x == 0 && threadIdx.x == 0) ctrl[kCtrlProjCount] = 0;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int pos = item / im.spl;
    process_cell<WG, ACCUM, VOTED>(im, cell_in_strips(pos, im.nx, im.ny, im.strips),
                                   item - pos * im.spl, packed, centres, endpoints, labels, acc,
                                   lambda, cap, tab_dyn, sh);
}

// At most 64 VGPRs (8 waves per SIMD): two 1024-thread workgroups per CU.
template <int WG, bool VOTED>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8)))
void k_assign_persistent(const Img* __restrict__ imgs,
                                                          const int* __restrict__ item_start,
                                                          int n_img, int total,
                                                          const float4* __restrict__ packed,
                                                          const float* __restrict__ centres,
                                                          const int* __restrict__ endpoints,
                                                          int* __restrict__ labels,
                                                          long long* __restrict__ acc, int* ctrl,
                                                          float lambda, int cap) {
    extern __shared__ float2 tab_dyn[];
    __shared__ CellShared sh;
    __shared__ int item;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[kCtrlProjCount] = 0;
    // XCD x (workgroup b runs on XCD b mod 8) has its own run of items and
    // queue head: the x-th eighth of every image's items, in the cell order
    // of cell_in_strips, so its cells form a block and share its L2, and
    // every XCD starts on every image (images of few, large cells walk long
    // paths).  run x = item_start + (n_img + 1) (1 + x) holds where each
    // image's share starts in the run.  A workgroup takes the items of its
    // XCD's run, then those left in the other runs, in turn.
    for (int q = 0; q < 8;) {
        const int x = (int)((blockIdx.x + q) & 7u);
        const int* __restrict__ run = item_start + (n_img + 1) * (1 + x);
        if (threadIdx.x == 0) item = atomicAdd(&ctrl[kCtrlQueue + 32 * x], 1);
        __syncthreads();
        const int h = __builtin_amdgcn_readfirstlane(item);   // uniform: kept in SGPRs
        __syncthreads();
        if (h >= run[n_img]) {
            ++q;
            continue;
        }
        const int i = find_image(run, n_img, h);
        const Img im = imgs[i];
        const int ni = item_start[i + 1] - item_start[i];
        const int local = (int)((long long)ni * x >> 3) + (h - run[i]);
        const int pos = local / im.spl;
        process_cell<WG, true, VOTED>(im, cell_in_strips(pos, im.nx, im.ny, im.strips),
                                      local - pos * im.spl, packed, centres, endpoints, labels,
                                      acc, lambda, cap, tab_dyn, sh);
    }
}

// ---------------------------------------------------------------- window form

// Window candidate rule of Algorithm 1: a pixel's candidates are the
// clusters whose window (half-width R around the rounded barycenter)
// contains it, and it takes the smallest D of Eq. (3), the smallest k among
// equal distances.  One workgroup per cluster k scans k's window, computes D
// for every pixel of it along the path to k's endpoint, and offers (D, k) to
// the pixel with a 64-bit atomic minimum of (FP32 bits of D, k): D >= 0, so
// the minimum is the smallest D and, among equal D, the smallest k.
template <int WG>
__global__ __launch_bounds__(WG) void k_assign_window(Img im, const float4* __restrict__ packed,
                                                      const float* __restrict__ centres,
                                                      const int* __restrict__ endpoints,
                                                      unsigned long long* __restrict__ keys,
                                                      int R, float lambda, int cap) {
    extern __shared__ float2 win_tab[];
    const int tid = threadIdx.x;
    const int k = xcd_remap(blockIdx.x, gridDim.x);
    const int W = im.W, H = im.H;
    const float4* __restrict__ img = packed + im.pix;
    const float* ck = centres + 5LL * (im.sp + k);
    const float l = ck[0], a = ck[1], b = ck[2], xk = ck[3], yk = ck[4];
    const int wx = round_coord(xk, W - 1), wy = round_coord(yk, H - 1);
    const int cx = min(max(endpoints[2LL * (im.sp + k)], 0), W - 1);
    const int cy = min(max(endpoints[2LL * (im.sp + k) + 1], 0), H - 1);
    const int x0 = max(wx - R, 0), x1 = min(wx + R, W - 1) + 1;
    const int y0 = max(wy - R, 0), y1 = min(wy + R, H - 1) + 1;
    // the paths of the window end at (cx, cy): over bbox(window, endpoint)
    // the table holds (d_c(q, k), w_q), two 8-byte entries per 16-byte unit
    const int rx0 = min(x0, cx), rx1 = max(x1, cx + 1);
    const int ry0 = min(y0, cy), ry1 = max(y1, cy + 1);
    const bool staged = (long long)(rx1 - rx0) * (ry1 - ry0) <= 2LL * cap;
    const int rw = rx1 - rx0;
    if (staged) {
        if (rw <= WG)                                // uniform
            fill_table_cols<WG>(win_tab, img, W, rx0, ry0, rw, ry1 - ry0, WG / rw,
                                (0x1000000u + (unsigned)rw - 1u) / (unsigned)rw, l, a, b);
        else
            fill_table<WG>(win_tab, img, W, rx0, ry0, rw, rw * (ry1 - ry0), l, a, b);
    }
    __syncthreads();
    const float4 fc = img[(long long)cy * W + cx];
    const float dcc = colour_dist(fc, l, a, b), wc = fc.w;
    const int cw = x1 - x0, ch = y1 - y0, P = cw * ch;
    const int lane = tid & 63, wave = tid >> 6;
    const float oml = 1.0f - lambda;
    for (int chunk = wave; chunk * 64 < P; chunk += WG / 64) {
        const int t = chunk * 64 + lane;
        if (t >= P) continue;
        int x, y;
        cell_pixel(t, cw, ch, x, y);
        x += x0;
        y += y0;
        const int p = y * W + x;
        const float4 fp = img[p];
        const int dx = cx - x, dy = cy - y;
        const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
        const int n = adx > ady ? adx : ady;
        const double inv = path_recip(n);
        const float dcp = colour_dist(fp, l, a, b);
        float sc = dcp, sw = fp.w;
        if (staged)
            walk_table(win_tab, (y - ry0) * rw + (x - rx0), rw, dx, dy, sc, sw);
        else
            walk_path(img, p, 1, W, dx, dy, l, a, b, sc, sw);
        if (n > 0) {
            sc = sc + dcc;
            sw = sw + wc;
        }
        float qc, qw;
        div_path_len(sc, sw, n, inv, qc, qw);
        const float A = lambda * dcp + oml * qc;
        const float B = 1.0f + im.gamma * qw;
        const float ex = (float)x - xk, ey = (float)y - yk;
        const float D = A * B + (ex * ex + ey * ey) * im.spw;
        const unsigned long long key = ((unsigned long long)__float_as_uint(D) << 32) | (unsigned)k;
        // keys only ever decrease: a stored key at or below this one (even
        // read stale) means the atomic would change nothing
        unsigned long long* kp = &keys[im.pix + p];
        if (key < *reinterpret_cast<volatile unsigned long long*>(kp)) atomicMin(kp, key);
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, long long n, unsigned long long v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Labels from the window minima; pixels no window covered keep their label.
__global__ void k_window_labels(const unsigned long long* __restrict__ keys, int* __restrict__ labels,
                                long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const unsigned long long key = keys[i];
        if (key != ~0ULL) labels[i] = (int)(unsigned)(key & 0xffffffffULL);
    }
}

// ---------------------------------------------------------------- prepare

__global__ void k_prepare(long long n, const float* __restrict__ lab,
                          const float* __restrict__ contour, float sigma,
                          float4* __restrict__ packed) {
    const double s2 = (double)sigma * (double)sigma;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double c = (double)contour[i];
        const float w = (float)(1.0 - exp(-(c * c) / s2));
        packed[i] = make_float4(lab[3 * i], lab[3 * i + 1], lab[3 * i + 2], w);
    }
}

__global__ void k_clear(long long* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------- init

template <int WG>
__device__ __forceinline__ void init_cell(const Img& im, int cell, const float4* __restrict__ packed,
                                          int* __restrict__ labels, long long* __restrict__ acc) {
    __shared__ long long red[6][WG];
    const int tid = threadIdx.x;
    const int ci = cell / im.nx, cj = cell - ci * im.nx;
    const int x0 = cell_lo(cj, im.W, im.nx), x1 = cell_lo(cj + 1, im.W, im.nx);
    const int y0 = cell_lo(ci, im.H, im.ny), y1 = cell_lo(ci + 1, im.H, im.ny);
    const int cw = x1 - x0, P = cw * (y1 - y0);
    long long s[6] = {0, 0, 0, 0, 0, 0};
    for (int t = tid; t < P; t += WG) {
        const int r = t / cw;
        const int x = x0 + (t - r * cw), y = y0 + r;
        const long long p = (long long)y * im.W + x;
        const float4 f = packed[im.pix + p];
        labels[im.pix + p] = cell;
        s[0] += 1; s[1] += x; s[2] += y;
        s[3] += to_fixed(f.x); s[4] += to_fixed(f.y); s[5] += to_fixed(f.z);
    }
    for (int v = 0; v < 6; ++v) red[v][tid] = s[v];
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int v = 0; v < 6; ++v) red[v][tid] += red[v][tid + h];
        __syncthreads();
    }
    if (tid < 6) acc[kAccStride * (long long)(im.sp + cell) + tid] = red[tid][0];
    __syncthreads();
}

template <int WG>
__global__ __launch_bounds__(WG) void k_init_cells(Img im, const float4* __restrict__ packed,
                                                   int* __restrict__ labels,
                                                   long long* __restrict__ acc) {
    init_cell<WG>(im, blockIdx.x, packed, labels, acc);
}

template <int WG>
__global__ __launch_bounds__(WG) void k_init_cells_batched(const Img* __restrict__ imgs,
                                                           const int* __restrict__ cell_start,
                                                           int n_img, const float4* packed,
                                                           int* labels, long long* acc) {
    const int i = find_image(cell_start, n_img, blockIdx.x);
    init_cell<WG>(imgs[i], blockIdx.x - cell_start[i], packed, labels, acc);
}

// ---------------------------------------------------------------- update from labels

// Colour source of the update: the caller's lab array, or the packed texels.
struct LabSource {
    const float* lab;
    const float4* packed;
    __device__ __forceinline__ float3 operator()(long long p) const {
        if (packed) {
            const float4 f = packed[p];
            return make_float3(f.x, f.y, f.z);
        }
        return make_float3(lab[3 * p], lab[3 * p + 1], lab[3 * p + 2]);
    }
};

// Integer sums of the update for labels that need not be grid neighbours
// (window form, caller-supplied labels).  One workgroup per grid cell
// accumulates into a small LDS table keyed by label (open addressing, key
// claimed with a compare-and-swap); a label that finds no free slot goes
// straight to the global sums.  The sums are integers, so the result does
// not depend on the order of the atomics.
constexpr int kAccSlots = 32;

// wkeys (window form, else null): the pass's window minima; a pixel whose
// key is set takes its label from it (the others keep theirs), and every key
// is reset to the all-ones "no window" value for the next pass; the pass
// also empties the projection queue that the finalize step after it fills
// (ctrl, as the fused grid-form pass does).
template <int WG>
__global__ __launch_bounds__(WG) void k_accumulate(Img im, LabSource src,
                                                   int* __restrict__ labels,
                                                   unsigned long long* __restrict__ wkeys,
                                                   int* __restrict__ ctrl,
                                                   long long* __restrict__ acc) {
    __shared__ int keys[kAccSlots];
    // [slot * 6 + sum][copy]: the lanes of a wave mostly carry one label, so
    // each adds to copy (t ^ t >> 3) mod kBinCopies (see CellShared)
    __shared__ unsigned long long bins[kAccSlots * 6][kBinCopies];
    const int tid = threadIdx.x;
    const int cell = blockIdx.x;
    if (ctrl && cell == 0 && tid == 0) ctrl[kCtrlProjCount] = 0;
    const int ci = cell / im.nx, cj = cell - ci * im.nx;
    const int x0 = cell_lo(cj, im.W, im.nx), x1 = cell_lo(cj + 1, im.W, im.nx);
    const int y0 = cell_lo(ci, im.H, im.ny), y1 = cell_lo(ci + 1, im.H, im.ny);
    const int K = im.nx * im.ny;
    for (int t = tid; t < kAccSlots * 6 * kBinCopies; t += WG) (&bins[0][0])[t] = 0ULL;
    for (int t = tid; t < kAccSlots; t += WG) keys[t] = -1;
    const int cp = (tid ^ (tid >> 3)) & (kBinCopies - 1);
    __syncthreads();
    const int cw = x1 - x0, P = cw * (y1 - y0);
    for (int t = tid; t < P; t += WG) {
        const int r = t / cw;
        const int x = x0 + (t - r * cw), y = y0 + r;
        const long long p = (long long)y * im.W + x;
        int k;
        if (wkeys) {
            const unsigned long long key = wkeys[p];
            if (key != ~0ULL) {
                k = (int)(unsigned)(key & 0xffffffffULL);
                labels[p] = k;
            } else {
                k = labels[p];
            }
            wkeys[p] = ~0ULL;
        } else {
            k = labels[p];
        }
        if (k < 0 || k >= K) continue;
        const float3 f = src(p);
        const unsigned long long v[6] = {1ULL, (unsigned long long)x, (unsigned long long)y,
                                         (unsigned long long)to_fixed(f.x),
                                         (unsigned long long)to_fixed(f.y),
                                         (unsigned long long)to_fixed(f.z)};
        int slot = -1;
        for (int probe = 0, h = k & (kAccSlots - 1); probe < kAccSlots;
             ++probe, h = (h + 1) & (kAccSlots - 1)) {
            const int cur = keys[h];
            if (cur == k) { slot = h; break; }
            if (cur == -1) {
                const int old = atomicCAS(&keys[h], -1, k);
                if (old == -1 || old == k) { slot = h; break; }
            }
        }
        if (slot >= 0) {
            for (int q = 0; q < 6; ++q) atomicAdd(&bins[slot * 6 + q][cp], v[q]);
        } else {
            for (int q = 0; q < 6; ++q)
                atomicAdd((unsigned long long*)(acc + kAccStride * (long long)(im.sp + k) + q), v[q]);
        }
    }
    __syncthreads();
    for (int t = tid; t < kAccSlots * 6; t += WG) {
        const int slot = t / 6, q = t - 6 * (t / 6);
        const int k = keys[slot];
        unsigned long long n = 0, v = 0;
        for (int c = 0; c < kBinCopies; ++c) {
            n += bins[slot * 6][c];
            v += bins[t][c];
        }
        if (k >= 0 && n != 0ULL)
            atomicAdd((unsigned long long*)(acc + kAccStride * (long long)(im.sp + k) + q), v);
    }
}

// ---------------------------------------------------------------- finalize

// Superpixel k's centre, barycenter and count from its sums (which it
// clears); the endpoint is the rounded barycenter when that pixel is one of
// k's own or projection is off.  Returns true when the projection has to
// move the endpoint instead (then xk, yk, cnt are what it needs).
__device__ __forceinline__ bool finalize_core(const Img& im, int k, float* __restrict__ centres,
                                              int* __restrict__ endpoints,
                                              int* __restrict__ counts,
                                              long long* __restrict__ acc,
                                              const int* __restrict__ labels, bool project,
                                              float& xk, float& yk, int& cnt_out) {
    long long* a = acc + kAccStride * (long long)(im.sp + k);
    const long long cnt = a[0];
    bool move = false;
    if (cnt > 0) {
        const double n = (double)cnt;
        float* c = centres + 5LL * (im.sp + k);
        c[0] = (float)(((double)a[3] / n) * kFixInv);
        c[1] = (float)(((double)a[4] / n) * kFixInv);
        c[2] = (float)(((double)a[5] / n) * kFixInv);
        xk = (float)((double)a[1] / n);
        yk = (float)((double)a[2] / n);
        c[3] = xk;
        c[4] = yk;
        const int ex = round_coord(xk, im.W - 1), ey = round_coord(yk, im.H - 1);
        if (!project || labels[im.pix + (long long)ey * im.W + ex] == k) {
            endpoints[2LL * (im.sp + k)] = ex;
            endpoints[2LL * (im.sp + k) + 1] = ey;
        } else {
            move = true;
        }
    }
    counts[im.sp + k] = (int)cnt;
    cnt_out = (int)cnt;
    for (int v = 0; v < 6; ++v) a[v] = 0;
    return move;
}

__device__ __forceinline__ void finalize_one(const Img& im, int k, float* __restrict__ centres,
                                             int* __restrict__ endpoints,
                                             int* __restrict__ counts,
                                             long long* __restrict__ acc,
                                             const int* __restrict__ labels, int* ctrl,
                                             int* plist, bool project) {
    float xk, yk;
    int cnt;
    if (finalize_core(im, k, centres, endpoints, counts, acc, labels, project, xk, yk, cnt)) {
        const int slot = atomicAdd(&ctrl[kCtrlProjCount], 1);
        plist[slot] = im.sp + k;
    }
}

__global__ void k_finalize(Img im, float* centres, int* endpoints, int* counts, long long* acc,
                           const int* labels, int* ctrl, int* plist, int project) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < im.nx * im.ny)
        finalize_one(im, k, centres, endpoints, counts, acc, labels, ctrl, plist, project != 0);
}

__global__ void k_finalize_batched(const Img* __restrict__ imgs, const int* __restrict__ sp_start,
                                   int n_img, int total, float* centres, int* endpoints,
                                   int* counts, long long* acc, const int* labels, int* ctrl,
                                   int* plist, int project) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < 8) ctrl[kCtrlQueue + 32 * g] = 0;   // the next persistent assignment starts afresh
    if (g >= total) return;
    const int i = find_image(sp_start, n_img, g);
    const Img im = imgs[i];
    finalize_one(im, g - im.sp, centres, endpoints, counts, acc, labels, ctrl, plist,
                 project != 0);
}

// ---------------------------------------------------------------- projection

// Minimum key and member count over the workgroup: shuffles within each
// wave, then one LDS slot per wave (two barriers in all).
template <int WG>
__device__ __forceinline__ void block_min_sum(unsigned long long& key, int& cnt) {
    __shared__ unsigned long long rk[WG / 64];
    __shared__ int rc[WG / 64];
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long k2 = __shfl_xor(key, o, 64);
        key = k2 < key ? k2 : key;
        cnt += __shfl_xor(cnt, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        rk[threadIdx.x >> 6] = key;
        rc[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    key = rk[0];
    cnt = rc[0];
    for (int q = 1; q < WG / 64; ++q) {
        key = rk[q] < key ? rk[q] : key;
        cnt += rc[q];
    }
    __syncthreads();   // the slots are reused by the next reduction
}

// Squared FP32 distance to (xk, yk) in the high word, raster index in the
// low word: the minimum key is the nearest pixel, ties to the lowest index.
__device__ __forceinline__ unsigned long long proj_key(int x, int y, int W, float xk, float yk) {
    const float dx = (float)x - xk;
    const float dy = (float)y - yk;
    const float d = dx * dx + dy * dy;
    return ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)(y * W + x);
}

// Nearest member of cluster k (key of proj_key) and the number of members
// inside [X0, X1) x [Y0, Y1), reduced over the workgroup; four independent
// label loads in flight per thread per round.
template <int WG>
__device__ void scan_region(const int* __restrict__ lb, int W, int k, int X0, int X1, int Y0,
                            int Y1, float xk, float yk, unsigned long long& best, int& found) {
    const int tid = threadIdx.x;
    const int bw = X1 - X0, area = bw * (Y1 - Y0);
    best = ~0ULL;
    found = 0;
    // element e = r * bw + c; lanes step by WG elements = (dr rows, dc
    // columns), eight loads in flight per trip (the minimum over packed keys
    // does not depend on the order)
    constexpr int kU = 8;
    const int dr = WG / bw, dc = WG - dr * bw;
    int r = tid / bw, c = tid - r * bw;
    for (int e0 = tid; e0 < area; e0 += kU * WG) {
        int lbl[kU], xs[kU], ys[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            xs[u] = X0 + c;
            ys[u] = Y0 + r;
            lbl[u] = e0 + u * WG < area ? lb[(long long)ys[u] * W + xs[u]] : -1;
            c += dc;
            const bool wrap = c >= bw;
            c -= wrap ? bw : 0;
            r += dr + (wrap ? 1 : 0);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (lbl[u] == k) {
                ++found;
                const unsigned long long key = proj_key(xs[u], ys[u], W, xk, yk);
                best = key < best ? key : best;
            }
        }
    }
    block_min_sum<WG>(best, found);
}

// Eq. (4) for one queued cluster: the argmin over all its members, found by
// scanning regions of growing size until every member (counts) was seen:
// the 3x3 cell block around its grid cell (where the grid form's labels
// lie), then the square of half-width 2R + 2 around its rounded barycenter
// (the window form: members lie within R of the previous barycenter, which
// lies within R of the new one), then the whole image (any labels).
template <int WG>
__device__ void project_at(const Img& im, int k, float xk, float yk, int count,
                           const int* __restrict__ labels, int* __restrict__ endpoints) {
    const int W = im.W, H = im.H;
    const int* lb = labels + im.pix;
    const int ci = k / im.nx, cj = k - ci * im.nx;
    unsigned long long best;
    int found;
    scan_region<WG>(lb, W, k, cell_lo(max(cj - 1, 0), W, im.nx), cell_lo(min(cj + 2, im.nx), W, im.nx),
                    cell_lo(max(ci - 1, 0), H, im.ny), cell_lo(min(ci + 2, im.ny), H, im.ny), xk, yk,
                    best, found);
    if (found < count) {                           // uniform: reduced over the workgroup
        const int h = 2 * im.rad + 2;
        const int cx = round_coord(xk, W - 1), cy = round_coord(yk, H - 1);
        scan_region<WG>(lb, W, k, max(cx - h, 0), min(cx + h + 1, W), max(cy - h, 0),
                        min(cy + h + 1, H), xk, yk, best, found);
        if (found < count) scan_region<WG>(lb, W, k, 0, W, 0, H, xk, yk, best, found);
    }
    if (threadIdx.x == 0 && best != ~0ULL) {
        const unsigned idx = (unsigned)(best & 0xffffffffULL);
        endpoints[2LL * (im.sp + k)] = (int)(idx % (unsigned)W);
        endpoints[2LL * (im.sp + k) + 1] = (int)(idx / (unsigned)W);
    }
}

template <int WG>
__device__ void project_one(const Img& im, int k, const float* __restrict__ centres,
                            const int* __restrict__ counts, const int* __restrict__ labels,
                            int* __restrict__ endpoints) {
    project_at<WG>(im, k, centres[5LL * (im.sp + k) + 3], centres[5LL * (im.sp + k) + 4],
                   counts[im.sp + k], labels, endpoints);
}

// Finalize and projection in one pass, a workgroup per superpixel: thread 0
// takes the superpixel's sums, and when its rounded barycenter is not one of
// its pixels the workgroup moves the endpoint to the nearest member at once
// (no queue, no second launch; projecting k reads only k's own centre and
// count and the labels).
template <int WG>
__global__ __launch_bounds__(WG) void k_finalize_project(Img im, float* centres, int* endpoints,
                                                         int* counts, long long* acc,
                                                         const int* labels) {
    __shared__ float sx, sy;
    __shared__ int scnt, smove;
    const int k = blockIdx.x;
    if (threadIdx.x == 0) {
        float xk = 0.0f, yk = 0.0f;
        int cnt = 0;
        smove = finalize_core(im, k, centres, endpoints, counts, acc, labels, true, xk, yk, cnt)
                    ? 1 : 0;
        sx = xk;
        sy = yk;
        scnt = cnt;
    }
    __syncthreads();
    if (smove) project_at<WG>(im, k, sx, sy, scnt, labels, endpoints);   // uniform
}

// The same over a ragged batch, a workgroup per superpixel of the batch;
// like k_finalize_batched it resets the persistent assignment's queue heads.
template <int WG>
__global__ __launch_bounds__(WG) void k_finalize_project_batched(const Img* __restrict__ imgs,
                                                                 const int* __restrict__ sp_start,
                                                                 int n_img, float* centres,
                                                                 int* endpoints, int* counts,
                                                                 long long* acc, const int* labels,
                                                                 int* ctrl) {
    __shared__ float sx, sy;
    __shared__ int scnt, smove, simg;
    const int g = blockIdx.x;
    // the next persistent assignment starts afresh (block 0 clears all 8
    // heads: a batch may have fewer than 8 superpixels)
    if (g == 0 && threadIdx.x < 8) ctrl[kCtrlQueue + 32 * threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        const int i = find_image(sp_start, n_img, g);
        float xk = 0.0f, yk = 0.0f;
        int cnt = 0;
        smove = finalize_core(imgs[i], g - imgs[i].sp, centres, endpoints, counts, acc, labels,
                              true, xk, yk, cnt) ? 1 : 0;
        sx = xk;
        sy = yk;
        scnt = cnt;
        simg = i;
    }
    __syncthreads();
    if (smove) {                                   // uniform
        const Img im = imgs[simg];
        project_at<WG>(im, g - im.sp, sx, sy, scnt, labels, endpoints);
    }
}

template <int WG>
__global__ __launch_bounds__(WG) void k_project(Img im, const float* centres, const int* counts,
                                                const int* labels, int* endpoints,
                                                const int* ctrl, const int* plist) {
    const int n = ctrl[kCtrlProjCount];
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        project_one<WG>(im, plist[i] - im.sp, centres, counts, labels, endpoints);
}

// Small host tables (image descriptors) reach the device as kernel
// arguments, so no host buffer has to outlive the call and the copy can be
// captured into a graph.
struct ByteChunk {
    unsigned nbytes;
    unsigned char data[3072];
};

__global__ void k_write_bytes(unsigned char* __restrict__ dst, ByteChunk c) {
    for (unsigned i = threadIdx.x; i < c.nbytes; i += blockDim.x) dst[i] = c.data[i];
}

constexpr int kSmallWG = 256;
constexpr int kProjectWG = 1024;
constexpr int kProjectBlocks = 256;
// Workgroup of the finalize + projection pass: 256 lanes, or 1024 where a
// superpixel's 3x3 cell block holds more than kWideProjectPixels pixels (the
// coarse scales of the multi-scale batch: one projection then scans most of
// the image, and its workgroup alone bounds the pass).
constexpr int kFinProjectWG = 256;
constexpr int kWideProjectWG = 1024;
constexpr long long kWideProjectPixels = 32768;

size_t dyn_lds(const Tuning& t) { return (size_t)t.lds_pixels * sizeof(float4); }

template <typename K>
void allow_lds(K kernel, size_t bytes) {
    // Lift the dynamic-LDS limit to what the launch needs (gfx950: 160 KiB per CU).
    static_cast<void>(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)bytes));
    static_cast<void>(hipGetLastError());
}

}  // namespace

// 4800 x 16 B of tables (75 KiB) fit twice in 160 KiB: two 1024-thread
// workgroups per CU.
int default_lds_pixels() { return 4800; }

int launch_write_bytes(void* dst, const void* src, size_t n, hipStream_t s) {
    const unsigned char* in = static_cast<const unsigned char*>(src);
    unsigned char* out = static_cast<unsigned char*>(dst);
    for (size_t off = 0; off < n; off += sizeof(ByteChunk::data)) {
        ByteChunk c;
        c.nbytes = (unsigned)std::min(n - off, sizeof(c.data));
        std::copy(in + off, in + off + c.nbytes, c.data);
        hipLaunchKernelGGL(k_write_bytes, dim3(1), dim3(256), 0, s, out + off, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void lift_lds_limits() {
    const size_t cap = 160 * 1024 - sizeof(CellShared) - 64;
    allow_lds(k_assign_window<256>, cap);
    allow_lds(k_assign_window<512>, cap);
    allow_lds(k_assign_window<1024>, cap);
    allow_lds(k_assign<256, true, false>, cap);
    allow_lds(k_assign<256, false, false>, cap);
    allow_lds(k_assign<512, true, false>, cap);
    allow_lds(k_assign<512, false, false>, cap);
    allow_lds(k_assign<1024, true, false>, cap);
    allow_lds(k_assign<1024, false, false>, cap);
    allow_lds(k_assign<256, true, true>, cap);
    allow_lds(k_assign<256, false, true>, cap);
    allow_lds(k_assign<512, true, true>, cap);
    allow_lds(k_assign<512, false, true>, cap);
    allow_lds(k_assign<1024, true, true>, cap);
    allow_lds(k_assign<1024, false, true>, cap);
    allow_lds(k_assign_persistent<256, false>, cap);
    allow_lds(k_assign_persistent<512, false>, cap);
    allow_lds(k_assign_persistent<1024, false>, cap);
    allow_lds(k_assign_persistent<256, true>, cap);
    allow_lds(k_assign_persistent<512, true>, cap);
    allow_lds(k_assign_persistent<1024, true>, cap);
}

int launch_prepare(long long n, const float* lab, const float* contour, float sigma,
                   float4* packed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)blocks), dim3(256), 0, s, n, lab, contour, sigma,
                       packed);
    return hipGetLastError();
}

int launch_clear(long long* p, long long n_words, hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n_words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_clear, dim3((unsigned)blocks), dim3(256), 0, s, p, n_words);
    return hipGetLastError();
}

int launch_init_cells(const Img& im, const float4* packed, int* labels, long long* acc,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_init_cells<kSmallWG>, dim3(im.nx * im.ny), dim3(kSmallWG), 0, s, im,
                       packed, labels, acc);
    return hipGetLastError();
}

int launch_init_cells_batched(const Img* imgs, const int* cell_start, int n_img, int total_cells,
                              const float4* packed, int* labels, long long* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_init_cells_batched<kSmallWG>, dim3(total_cells), dim3(kSmallWG), 0, s,
                       imgs, cell_start, n_img, packed, labels, acc);
    return hipGetLastError();
}

template <int WG, bool ACCUM, bool VOTED>
static int launch_assign_t(const Img& im, const float4* packed, const float* centres,
                           const int* endpoints, int* labels, long long* acc, int* ctrl,
                           float lambda, const Tuning& t, hipStream_t s) {
    const size_t bytes = dyn_lds(t);
    hipLaunchKernelGGL((k_assign<WG, ACCUM, VOTED>), dim3(im.nx * im.ny * im.spl), dim3(WG), bytes,
                       s, im, packed, centres, endpoints, labels, acc, ctrl, lambda,
                       t.lds_pixels);
    return hipGetLastError();
}

template <int WG, bool VOTED>
static int launch_assign_wg(const Img& im, const float4* packed, const float* centres,
                            const int* endpoints, int* labels, long long* acc, int* ctrl,
                            float lambda, bool accumulate, const Tuning& t, hipStream_t s) {
    return accumulate ? launch_assign_t<WG, true, VOTED>(im, packed, centres, endpoints, labels,
                                                         acc, ctrl, lambda, t, s)
                      : launch_assign_t<WG, false, VOTED>(im, packed, centres, endpoints, labels,
                                                          acc, ctrl, lambda, t, s);
}

template <bool VOTED>
static int launch_assign_v(const Img& im, const float4* packed, const float* centres,
                           const int* endpoints, int* labels, long long* acc, int* ctrl,
                           float lambda, bool accumulate, const Tuning& t, hipStream_t s) {
    if (t.wg == 1024)
        return launch_assign_wg<1024, VOTED>(im, packed, centres, endpoints, labels, acc, ctrl,
                                             lambda, accumulate, t, s);
    if (t.wg == 512)
        return launch_assign_wg<512, VOTED>(im, packed, centres, endpoints, labels, acc, ctrl,
                                            lambda, accumulate, t, s);
    return launch_assign_wg<256, VOTED>(im, packed, centres, endpoints, labels, acc, ctrl, lambda,
                                        accumulate, t, s);
}

int launch_assign(const Img& im, const float4* packed, const float* centres,
                  const int* endpoints, int* labels, long long* acc, int* ctrl, float lambda,
                  bool accumulate, const Tuning& t, hipStream_t s) {
    return t.voted ? launch_assign_v<true>(im, packed, centres, endpoints, labels, acc, ctrl,
                                           lambda, accumulate, t, s)
                   : launch_assign_v<false>(im, packed, centres, endpoints, labels, acc, ctrl,
                                            lambda, accumulate, t, s);
}

template <int WG, bool VOTED>
static int launch_persistent_t(const Img* imgs, const int* item_start, int n_img, int total,
                               const float4* packed, const float* centres, const int* endpoints,
                               int* labels, long long* acc, int* ctrl, float lambda,
                               const Tuning& t, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_assign_persistent<WG, VOTED>), dim3(grid), dim3(WG), dyn_lds(t), s,
                       imgs, item_start, n_img, total, packed, centres, endpoints, labels, acc,
                       ctrl, lambda, t.lds_pixels);
    return hipGetLastError();
}

template <bool VOTED>
static int launch_persistent_v(const Img* imgs, const int* item_start, int n_img, int total,
                               const float4* packed, const float* centres, const int* endpoints,
                               int* labels, long long* acc, int* ctrl, float lambda,
                               const Tuning& t, int grid, hipStream_t s) {
    if (t.wg == 1024)
        return launch_persistent_t<1024, VOTED>(imgs, item_start, n_img, total, packed, centres,
                                                endpoints, labels, acc, ctrl, lambda, t, grid, s);
    if (t.wg == 512)
        return launch_persistent_t<512, VOTED>(imgs, item_start, n_img, total, packed, centres,
                                               endpoints, labels, acc, ctrl, lambda, t, grid, s);
    return launch_persistent_t<256, VOTED>(imgs, item_start, n_img, total, packed, centres,
                                           endpoints, labels, acc, ctrl, lambda, t, grid, s);
}

int launch_assign_persistent(const Img* imgs, const int* item_start, int n_img, int total_items,
                             const float4* packed, const float* centres, const int* endpoints,
                             int* labels, long long* acc, int* ctrl, float lambda,
                             const Tuning& t, int grid, hipStream_t s) {
    return t.voted ? launch_persistent_v<true>(imgs, item_start, n_img, total_items, packed,
                                               centres, endpoints, labels, acc, ctrl, lambda, t,
                                               grid, s)
                   : launch_persistent_v<false>(imgs, item_start, n_img, total_items, packed,
                                                centres, endpoints, labels, acc, ctrl, lambda, t,
                                                grid, s);
}

template <int WG, bool VOTED>
static int persistent_occupancy(int* per, size_t lds) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_assign_persistent<WG, VOTED>,
                                                             WG, lds);
}

int persistent_grid(const Tuning& t) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const size_t lds = dyn_lds(t);
    int e;
    if (t.wg == 1024)
        e = t.voted ? persistent_occupancy<1024, true>(&per, lds)
                    : persistent_occupancy<1024, false>(&per, lds);
    else if (t.wg == 512)
        e = t.voted ? persistent_occupancy<512, true>(&per, lds)
                    : persistent_occupancy<512, false>(&per, lds);
    else
        e = t.voted ? persistent_occupancy<256, true>(&per, lds)
                    : persistent_occupancy<256, false>(&per, lds);
    if (e != (int)hipSuccess || per < 1) per = 1;
    if (t.blocks_per_cu > 0 && t.blocks_per_cu < per) per = t.blocks_per_cu;
    return cus * per;
}

template <int WG>
static int launch_window_t(const Img& im, const float4* packed, const float* centres,
                           const int* endpoints, unsigned long long* keys, int R, float lambda,
                           const Tuning& t, hipStream_t s) {
    hipLaunchKernelGGL(k_assign_window<WG>, dim3(im.nx * im.ny), dim3(WG), dyn_lds(t), s, im,
                       packed, centres, endpoints, keys, R, lambda, t.lds_pixels);
    return hipGetLastError();
}

int launch_fill_keys(const Img& im, unsigned long long* keys, hipStream_t s) {
    const long long n = (long long)im.W * im.H;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, keys + im.pix, n, ~0ULL);
    return hipGetLastError();
}

int launch_assign_window(const Img& im, const float4* packed, const float* centres,
                         const int* endpoints, int* labels, unsigned long long* keys, int R,
                         float lambda, bool labels_out, const Tuning& t, hipStream_t s) {
    const long long n = (long long)im.W * im.H;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    if (labels_out) {
        const int e = launch_fill_keys(im, keys, s);
        if (e != hipSuccess) return e;
    }
    int r;
    if (t.wg == 1024) r = launch_window_t<1024>(im, packed, centres, endpoints, keys, R, lambda, t, s);
    else if (t.wg == 512) r = launch_window_t<512>(im, packed, centres, endpoints, keys, R, lambda, t, s);
    else r = launch_window_t<256>(im, packed, centres, endpoints, keys, R, lambda, t, s);
    if (r != hipSuccess || !labels_out) return r;
    hipLaunchKernelGGL(k_window_labels, dim3(blocks), dim3(256), 0, s, keys + im.pix,
                       labels + im.pix, n);
    return hipGetLastError();
}

int launch_accumulate(const Img& im, const float* lab, const int* labels, long long* acc,
                      hipStream_t s) {
    const LabSource src{lab, nullptr};
    hipLaunchKernelGGL(k_accumulate<kSmallWG>, dim3(im.nx * im.ny), dim3(kSmallWG), 0, s, im, src,
                       const_cast<int*>(labels), static_cast<unsigned long long*>(nullptr),
                       static_cast<int*>(nullptr), acc);
    return hipGetLastError();
}

int launch_accumulate_window(const Img& im, const float4* packed, int* labels,
                             unsigned long long* keys, int* ctrl, long long* acc, hipStream_t s) {
    const LabSource src{nullptr, packed};
    hipLaunchKernelGGL(k_accumulate<kSmallWG>, dim3(im.nx * im.ny), dim3(kSmallWG), 0, s, im, src,
                       labels, keys + im.pix, ctrl, acc);
    return hipGetLastError();
}

int launch_finalize(const Img& im, float* centres, int* endpoints, int* counts, long long* acc,
                    const int* labels, int* ctrl, int* plist, bool project, hipStream_t s) {
    const int K = im.nx * im.ny;
    hipLaunchKernelGGL(k_finalize, dim3((K + 255) / 256), dim3(256), 0, s, im, centres,
                       endpoints, counts, acc, labels, ctrl, plist, project ? 1 : 0);
    return hipGetLastError();
}

int launch_finalize_batched(const Img* imgs, const int* sp_start, int n_img, int total_sp,
                            float* centres, int* endpoints, int* counts, long long* acc,
                            const int* labels, int* ctrl, int* plist, bool project,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_batched, dim3((total_sp + 255) / 256), dim3(256), 0, s, imgs,
                       sp_start, n_img, total_sp, centres, endpoints, counts, acc, labels, ctrl,
                       plist, project ? 1 : 0);
    return hipGetLastError();
}

long long block_pixels(int W, int H, int nx, int ny) {
    return 9LL * ((W + nx - 1) / nx) * ((H + ny - 1) / ny);
}

int launch_finalize_project(const Img& im, float* centres, int* endpoints, int* counts,
                            long long* acc, const int* labels, hipStream_t s) {
    if (block_pixels(im.W, im.H, im.nx, im.ny) > kWideProjectPixels)
        hipLaunchKernelGGL(k_finalize_project<kWideProjectWG>, dim3(im.nx * im.ny),
                           dim3(kWideProjectWG), 0, s, im, centres, endpoints, counts, acc, labels);
    else
        hipLaunchKernelGGL(k_finalize_project<kFinProjectWG>, dim3(im.nx * im.ny),
                           dim3(kFinProjectWG), 0, s, im, centres, endpoints, counts, acc, labels);
    return hipGetLastError();
}

int launch_finalize_project_batched(const Img* imgs, const int* sp_start, int n_img,
                                    int total_sp, long long max_block_px, float* centres,
                                    int* endpoints, int* counts, long long* acc, const int* labels,
                                    int* ctrl, hipStream_t s) {
    if (max_block_px > kWideProjectPixels)
        hipLaunchKernelGGL(k_finalize_project_batched<kWideProjectWG>, dim3(total_sp),
                           dim3(kWideProjectWG), 0, s, imgs, sp_start, n_img, centres, endpoints,
                           counts, acc, labels, ctrl);
    else
        hipLaunchKernelGGL(k_finalize_project_batched<kFinProjectWG>, dim3(total_sp),
                           dim3(kFinProjectWG), 0, s, imgs, sp_start, n_img, centres, endpoints,
                           counts, acc, labels, ctrl);
    return hipGetLastError();
}

int launch_project(const Img& im, const float* centres, const int* counts, const int* labels,
                   int* endpoints, const int* ctrl, const int* plist, hipStream_t s) {
    hipLaunchKernelGGL(k_project<kProjectWG>, dim3(kProjectBlocks), dim3(kProjectWG), 0, s, im,
                       centres, counts, labels, endpoints, ctrl, plist);
    return hipGetLastError();
}

}  // namespace scalp
