// scalp_metrics.hip -- superpixel quality metrics of Sec. III-A.2 on the GPU:
// boundary recall (Eq. (5)), achievable segmentation accuracy (Eq. (6)),
// undersegmentation error (Eq. (7)) and compactness (Eq. (8)) of a label map
// against a ground-truth partition.
//
//   k_metric_pixels  one pass over the pixels in blocks of 256 columns by
//                    a few whole rows, each lane loading its pixel and four
//                    clamped neighbours of both maps (independent loads, no
//                    branches; the next row's loads issued before the
//                    current row is processed): the overlap table
//                    |S_k n G_i| and the perimeter of every superpixel in
//                    pixel edges (4-connectivity, image border included),
//                    gathered per distinct (k, i) pair among a wave's pixels
//                    into a hash table in LDS and added to global memory once
//                    per pair and block (device-scope atomics are the
//                    expensive part here); and two boundary bitmaps, one
//                    64-bit word per wave and row (bit b = pixel 64 w + b).
//   k_metric_recall  thread per bitmap word: boundary-recall counts
//                    (ground-truth boundary pixels, those with a superpixel
//                    boundary pixel at distance < epsilon, superpixel
//                    boundary pixels) from the superpixel bitmap dilated
//                    over the epsilon disc with word shifts; one partial sum
//                    per workgroup.
//   k_metric_rows    wave per superpixel: area, largest overlap, UE row sum
//                    (integers) and the CO term 4 pi A^2 / P^2 (FP64).
//   k_metric_final   one workgroup: fixed-order sums of the rows and of the
//                    recall partials, so the result does not depend on the
//                    order of the atomics.
#include <algorithm>

#include "scalp_internal.h"

namespace scalp {
namespace {

constexpr int kMetricWG = 256;

struct MetricGeom {
    int W, H, K, R;
    int Wq;         // bitmap words per row, ceil(W / 64)
    int rows;       // rows per k_metric_pixels block
    int nrb;        // k_metric_recall blocks (partial sums)
    int r;          // neighbourhood half-width for boundary recall
    float eps2;     // epsilon^2
};

// Pair table of one workgroup: open addressing over kPairSlots entries in
// LDS, key k * R + i (< 2^30, so kEmpty never collides with a key).
constexpr int kPairBits = 9, kPairSlots = 1 << kPairBits;
constexpr unsigned kEmpty = 0xffffffffu;

struct PairTable {
    unsigned key[kPairSlots], cnt[kPairSlots], edge[kPairSlots];
};

// For every distinct (k, i) among the wave's lanes with `ok`: popc(m) pixels
// and the lanes' edge counts into the workgroup's pair table (a wave covers
// 64 neighbouring pixels, which mostly share their superpixel and region).
// e0..e2 are the bit planes of the lanes' edge counts (0..4), so a group's
// edge sum is three masked popcounts.  A full table sends the pair straight
// to global memory.
__device__ __forceinline__ void wave_count(PairTable& pt, unsigned* __restrict__ table,
                                           unsigned* __restrict__ perim, int R, bool ok, int k,
                                           int i, unsigned long long e0, unsigned long long e1,
                                           unsigned long long e2) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(ok);
    while (pending != 0ULL) {                         // uniform over the wave
        const int leader = __ffsll((long long)pending) - 1;
        const int lk = __builtin_amdgcn_readlane(k, leader);
        const int li = __builtin_amdgcn_readlane(i, leader);
        const unsigned long long m = __ballot(ok && k == lk && i == li) & pending;
        if (lane == leader) {
            const unsigned n = (unsigned)__popcll(m);
            const unsigned edges = (unsigned)(__popcll(e0 & m) + 2 * __popcll(e1 & m) +
                                              4 * __popcll(e2 & m));
            const unsigned key = (unsigned)lk * (unsigned)R + (unsigned)li;
            unsigned h = (key * 2654435761u) >> (32 - kPairBits);
            bool done = false;
            for (int probe = 0; probe < kPairSlots && !done; ++probe) {
                const unsigned old = atomicCAS(&pt.key[h], kEmpty, key);
                if (old == kEmpty || old == key) {
                    atomicAdd(&pt.cnt[h], n);
                    if (edges) atomicAdd(&pt.edge[h], edges);
                    done = true;
                }
                h = (h + 1) & (kPairSlots - 1);
            }
            if (!done) {
                atomicAdd(&table[key], n);
                if (edges) atomicAdd(&perim[lk], edges);
            }
        }
        pending &= ~m;
    }
}

// A lane's pixel and its four clamped neighbours in both maps.
struct PixRow {
    int k, i, sl, sr, su, sd, gl, gr, gu, gd;
};

__device__ __forceinline__ PixRow load_row(const int* __restrict__ S, const int* __restrict__ G,
                                           const MetricGeom& g, int y, int xc, int xl, int xr) {
    const long long row = (long long)y * g.W;
    const long long up = (long long)max(y - 1, 0) * g.W;
    const long long dn = (long long)min(y + 1, g.H - 1) * g.W;
    PixRow p;
    p.k = S[row + xc];
    p.i = G[row + xc];
    p.sl = S[row + xl];
    p.sr = S[row + xr];
    p.su = S[up + xc];
    p.sd = S[dn + xc];
    p.gl = G[row + xl];
    p.gr = G[row + xr];
    p.gu = G[up + xc];
    p.gd = G[dn + xc];
    return p;
}

// Block (bx, by): columns [256 bx, 256 bx + 256) of rows [by * rows, ...).
// A pixel is a boundary pixel when a 4-neighbour inside the image has
// another label; the clamped neighbour of a border pixel is the pixel
// itself, which never differs.
__global__ __launch_bounds__(kMetricWG) void k_metric_pixels(MetricGeom g, const int* __restrict__ S,
                                                             const int* __restrict__ G,
                                                             unsigned* __restrict__ table,
                                                             unsigned* __restrict__ perim,
                                                             unsigned long long* __restrict__ smap,
                                                             unsigned long long* __restrict__ gmap) {
    __shared__ PairTable pt;
    for (int t = threadIdx.x; t < kPairSlots; t += kMetricWG) {
        pt.key[t] = kEmpty;
        pt.cnt[t] = 0u;
        pt.edge[t] = 0u;
    }
    __syncthreads();
    const int x = blockIdx.x * kMetricWG + threadIdx.x;
    const int word = (blockIdx.x * kMetricWG + (threadIdx.x & ~63)) >> 6;
    const bool store = word < g.Wq && (threadIdx.x & 63) == 0;
    const bool in = x < g.W;
    const int xc = min(x, g.W - 1), xl = max(xc - 1, 0), xr = min(xc + 1, g.W - 1);
    const int y0 = blockIdx.y * g.rows, y1 = min(y0 + g.rows, g.H);
    PixRow cur = load_row(S, G, g, y0, xc, xl, xr);
    for (int y = y0; y < y1; ++y) {                   // uniform
        PixRow nxt = cur;
        if (y + 1 < y1) nxt = load_row(S, G, g, y + 1, xc, xl, xr);
        const int k = cur.k, i = cur.i;
        const bool dl = cur.sl != k, dr = cur.sr != k, du = cur.su != k, dd = cur.sd != k;
        const bool sb = in && (dl || dr || du || dd);
        const bool gb = in && (cur.gl != i || cur.gr != i || cur.gu != i || cur.gd != i);
        const unsigned long long sm = __ballot(sb), gm = __ballot(gb);
        if (store) {
            smap[(long long)y * g.Wq + word] = sm;
            gmap[(long long)y * g.Wq + word] = gm;
        }
        const bool ok = in && k >= 0 && k < g.K && i >= 0 && i < g.R;
        const unsigned e = (unsigned)(dl || x == 0) + (unsigned)(dr || x + 1 >= g.W) +
                           (unsigned)(du || y == 0) + (unsigned)(dd || y + 1 >= g.H);
        const unsigned long long e0 = __ballot(ok && (e & 1u)), e1 = __ballot(ok && (e & 2u)),
                                 e2 = __ballot(ok && (e & 4u));
        wave_count(pt, table, perim, g.R, ok, k, i, e0, e1, e2);
        cur = nxt;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kPairSlots; t += kMetricWG) {
        const unsigned key = pt.key[t];
        if (key == kEmpty) continue;
        atomicAdd(&table[key], pt.cnt[t]);
        if (pt.edge[t]) atomicAdd(&perim[key / (unsigned)g.R], pt.edge[t]);
    }
}

// 192-bit window {lo, mid, hi} (lo holds the lowest pixel indices), dilated by
// [-a, a] along the row: intervals grow by {-s, 0, s} steps with s <= 2m + 1,
// so the union stays gap-free; for a <= 63 every shifted-in bit of mid comes
// from inside the window.
__device__ __forceinline__ unsigned long long dilate_mid(unsigned long long lo,
                                                         unsigned long long mid,
                                                         unsigned long long hi, int a) {
    int m = 0;
    while (m < a) {
        const int s = min(2 * m + 1, a - m), t = 64 - s;
        const unsigned long long l2 = lo | (lo << s) | (lo >> s) | (mid << t);
        const unsigned long long m2 = mid | (mid << s) | (lo >> t) | (mid >> s) | (hi << t);
        const unsigned long long h2 = hi | (hi << s) | (mid >> t) | (hi >> s);
        lo = l2;
        mid = m2;
        hi = h2;
        m += s;
    }
    return mid;
}

// Thread per bitmap word (row y, word w): a ground-truth boundary pixel is
// recalled when a superpixel boundary pixel lies at (dx, dy) with
// dx^2 + dy^2 < epsilon^2 (Eq. (5)); out-of-image pixels are zero bits.
// The disc rows are taken three at a time, their words loaded before any is
// dilated.  part[3 b + {0, 1, 2}] = this block's ground-truth boundary
// pixels, recalled ones, superpixel boundary pixels.
__global__ __launch_bounds__(kMetricWG) void k_metric_recall(MetricGeom g,
                                                             const unsigned long long* __restrict__ smap,
                                                             const unsigned long long* __restrict__ gmap,
                                                             unsigned long long* __restrict__ part) {
    __shared__ unsigned long long red[kMetricWG / 64][3];
    const long long words = (long long)g.H * g.Wq;
    unsigned long long gb = 0, hit = 0, sb = 0;
    for (long long t = blockIdx.x * (long long)kMetricWG + threadIdx.x; t < words;
         t += (long long)gridDim.x * kMetricWG) {
        const int y = (int)(t / g.Wq), w = (int)(t - (long long)y * g.Wq);
        const unsigned long long gw = gmap[t];
        sb += (unsigned long long)__popcll(smap[t]);
        if (gw == 0ULL) continue;
        gb += (unsigned long long)__popcll(gw);
        unsigned long long d = 0;
        for (int dy0 = -g.r; dy0 <= g.r && (gw & ~d) != 0ULL; dy0 += 3) {
            unsigned long long lo[3], mid[3], hi[3];
            int a[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int dy = dy0 + j, yy = y + dy;
                a[j] = -1;                            // largest |dx| inside the disc
                if (dy <= g.r && yy >= 0 && yy < g.H)
                    while (a[j] < g.r && (float)((a[j] + 1) * (a[j] + 1) + dy * dy) < g.eps2) ++a[j];
                lo[j] = mid[j] = hi[j] = 0ULL;
                if (a[j] >= 0) {
                    const unsigned long long* rw = smap + (long long)yy * g.Wq;
                    mid[j] = rw[w];
                    if (w > 0) lo[j] = rw[w - 1];
                    if (w + 1 < g.Wq) hi[j] = rw[w + 1];
                }
            }
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (a[j] >= 0) d |= dilate_mid(lo[j], mid[j], hi[j], a[j]);
        }
        hit += (unsigned long long)__popcll(gw & d);
    }
    for (int o = 32; o > 0; o >>= 1) {
        gb += __shfl_xor(gb, o, 64);
        hit += __shfl_xor(hit, o, 64);
        sb += __shfl_xor(sb, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = gb;
        red[wv][1] = hit;
        red[wv][2] = sb;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int q = 0; q < kMetricWG / 64; ++q) v += red[q][threadIdx.x];
        part[3LL * blockIdx.x + threadIdx.x] = v;
    }
}

// Per superpixel (one wave each, lanes striding over the regions): area,
// largest overlap (ASA), sum over meeting regions of |S_k| - |S_k n G_i|
// (UE), and the CO term.  Integer sums and maxima: exact in any order.
__global__ __launch_bounds__(256) void k_metric_rows(MetricGeom g,
                                                     const unsigned* __restrict__ table,
                                                     const unsigned* __restrict__ perim,
                                                     unsigned long long* __restrict__ row_max,
                                                     unsigned long long* __restrict__ row_ue,
                                                     double* __restrict__ row_co) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (k >= g.K) return;                             // uniform over the wave
    const unsigned* t = table + (long long)k * g.R;
    unsigned long long area = 0, meet = 0;
    unsigned mx = 0;
    for (int i = lane; i < g.R; i += 64) {
        const unsigned c = t[i];
        area += c;
        mx = c > mx ? c : mx;
        meet += c ? 1ULL : 0ULL;
    }
    for (int o = 32; o > 0; o >>= 1) {
        area += __shfl_xor(area, o, 64);
        meet += __shfl_xor(meet, o, 64);
        const unsigned m2 = __shfl_xor(mx, o, 64);
        mx = m2 > mx ? m2 : mx;
    }
    if (lane == 0) {
        row_max[k] = mx;
        row_ue[k] = meet * area - area;   // sum over meeting i of (area - c_i)
        const double P = (double)perim[k];
        row_co[k] = area ? 4.0 * 3.14159265358979323846 * (double)area * (double)area / (P * P)
                         : 0.0;
    }
}

__global__ __launch_bounds__(1024) void k_metric_final(MetricGeom g,
                                                       const unsigned long long* __restrict__ row_max,
                                                       const unsigned long long* __restrict__ row_ue,
                                                       const double* __restrict__ row_co,
                                                       const unsigned long long* __restrict__ part,
                                                       double* __restrict__ out) {
    __shared__ unsigned long long rm[1024], ru[1024], rg[1024], rh[1024], rs[1024];
    __shared__ double rc[1024];
    const int tid = threadIdx.x;
    unsigned long long m = 0, u = 0, gb = 0, hit = 0, sb = 0;
    double c = 0.0;
    for (int k = tid; k < g.K; k += 1024) {
        m += row_max[k];
        u += row_ue[k];
        c += row_co[k];
    }
    for (int b = tid; b < g.nrb; b += 1024) {
        gb += part[3LL * b];
        hit += part[3LL * b + 1];
        sb += part[3LL * b + 2];
    }
    rm[tid] = m;
    ru[tid] = u;
    rc[tid] = c;
    rg[tid] = gb;
    rh[tid] = hit;
    rs[tid] = sb;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (tid < h) {
            rm[tid] += rm[tid + h];
            ru[tid] += ru[tid + h];
            rc[tid] += rc[tid + h];
            rg[tid] += rg[tid + h];
            rh[tid] += rh[tid + h];
            rs[tid] += rs[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double N = (double)g.W * (double)g.H;
        out[0] = rg[0] ? (double)rh[0] / (double)rg[0] : 1.0;      // BR
        out[1] = (double)rm[0] / N;                                 // ASA
        out[2] = (double)ru[0] / N;                                 // UE
        out[3] = rc[0] / N;                                         // CO
        out[4] = (double)rg[0];                                     // |B(G)|
        out[5] = (double)rs[0];                                     // |B(S)|
    }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

constexpr int kRecallBlocks = 2048;   // most k_metric_recall blocks (partial sums)

size_t metrics_workspace_bytes(int W, int H, int K, int R) {
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t table = (size_t)K * (size_t)R * 4, perim = (size_t)K * 4;
    const size_t rows = (size_t)K * 8 * 3, part = (size_t)kRecallBlocks * 3 * 8;
    const size_t map = (size_t)H * (size_t)((W + 63) / 64) * 8;
    return up(table) + up(perim) + up(rows) + up(part) + 2 * up(map);
}

int launch_metrics(int W, int H, const int* S, int K, const int* G, int R, float eps, double* out,
                   void* ws, hipStream_t st) {
    MetricGeom g;
    g.W = W; g.H = H; g.K = K; g.R = R;
    g.Wq = (W + 63) / 64;
    g.r = (int)ceilf(eps) - 1;
    g.eps2 = eps * eps;
    // k_metric_pixels: about 1024 blocks of 256 columns by up to 16 rows (more
    // rows per block gather more pixels per pair in LDS before the atomics)
    const int bx = (W + kMetricWG - 1) / kMetricWG;
    g.rows = (int)std::max<long long>(
        std::min<long long>((long long)H * bx / 1024, 16),
        std::max<long long>(1, ((long long)H + 65534) / 65535));
    const int by = (H + g.rows - 1) / g.rows;
    const long long map = (long long)H * g.Wq;
    g.nrb = (int)std::min<long long>((map + kMetricWG - 1) / kMetricWG, kRecallBlocks);
    char* b = static_cast<char*>(ws);
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    unsigned* table = reinterpret_cast<unsigned*>(b);
    size_t off = up((size_t)K * R * 4);
    unsigned* perim = reinterpret_cast<unsigned*>(b + off);
    off += up((size_t)K * 4);
    unsigned long long* row_max = reinterpret_cast<unsigned long long*>(b + off);
    unsigned long long* row_ue = row_max + K;
    double* row_co = reinterpret_cast<double*>(row_ue + K);
    off += up((size_t)K * 8 * 3);
    unsigned long long* part = reinterpret_cast<unsigned long long*>(b + off);
    off += up((size_t)kRecallBlocks * 3 * 8);
    unsigned long long* smap = reinterpret_cast<unsigned long long*>(b + off);
    unsigned long long* gmap = smap + up((size_t)map * 8) / 8;
    // table and perim (contiguous up to row_max) start at zero; every bitmap
    // word and every partial sum is written before it is read
    const long long zero_words = (long long)(reinterpret_cast<char*>(row_max) - b) / 4;
    const unsigned zb = (unsigned)std::min<long long>((zero_words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u32, dim3(zb), dim3(256), 0, st, table, zero_words);
    hipLaunchKernelGGL(k_metric_pixels, dim3((unsigned)bx, (unsigned)by), dim3(kMetricWG), 0, st,
                       g, S, G, table, perim, smap, gmap);
    hipLaunchKernelGGL(k_metric_recall, dim3((unsigned)g.nrb), dim3(kMetricWG), 0, st, g, smap,
                       gmap, part);
    hipLaunchKernelGGL(k_metric_rows, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, st, g, table,
                       perim, row_max, row_ue, row_co);
    hipLaunchKernelGGL(k_metric_final, dim3(1), dim3(1024), 0, st, g, row_max, row_ue, row_co, part,
                       out);
    return hipGetLastError();
}

}  // namespace scalp
