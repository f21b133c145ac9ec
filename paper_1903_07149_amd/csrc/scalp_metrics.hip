// scalp_metrics.hip -- superpixel quality metrics of Sec. III-A.2 on the GPU:
// boundary recall (Eq. (5)), achievable segmentation accuracy (Eq. (6)),
// undersegmentation error (Eq. (7)) and compactness (Eq. (8)) of a label map
// against a ground-truth partition.
//
//   k_metric_pixels  one pass over the pixels, each lane loading its pixel
//                    and four clamped neighbours of both maps (independent
//                    loads, no branches): the overlap table |S_k n G_i| and
//                    the perimeter of every superpixel in pixel edges
//                    (4-connectivity, image border included), one 32-bit
//                    atomic each per distinct (k, i) pair among a wave's
//                    pixels; and two boundary bitmaps, one 64-bit word per
//                    wave and row (bit b = pixel 64 w + b of the row).
//   k_metric_recall  thread per bitmap word: boundary-recall counts
//                    (ground-truth boundary pixels, those with a superpixel
//                    boundary pixel at distance < epsilon, superpixel
//                    boundary pixels) from the superpixel bitmap dilated
//                    over the epsilon disc with word shifts.
//   k_metric_rows    wave per superpixel: area, largest overlap, UE row sum
//                    (integers) and the CO term 4 pi A^2 / P^2 (FP64).
//   k_metric_final   one workgroup: fixed-order sums, so the result does not
//                    depend on the order of the atomics.
#include <algorithm>

#include "scalp_internal.h"

namespace scalp {
namespace {

constexpr int kMetricWG = 256;

struct MetricGeom {
    int W, H, K, R;
    int Wq;         // bitmap words per row, ceil(W / 64)
    int r;          // neighbourhood half-width for boundary recall
    float eps2;     // epsilon^2
};

// Adds popc(m) to table[k * R + i] and the lanes' edge counts to perim[k]
// for every distinct (k, i) among the wave's lanes with `ok`: a wave covers
// 64 neighbouring pixels, which mostly share their superpixel and region, and
// atomics on one word serialise.  e0..e2 are the bit planes of the lanes'
// edge counts (0..4), so a group's edge sum is three masked popcounts.
__device__ __forceinline__ void wave_count(unsigned* __restrict__ table,
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
        const unsigned edges = (unsigned)(__popcll(e0 & m) + 2 * __popcll(e1 & m) +
                                          4 * __popcll(e2 & m));
        if (lane == leader) {
            atomicAdd(&table[(long long)lk * R + li], (unsigned)__popcll(m));
            if (edges) atomicAdd(&perim[lk], edges);
        }
        pending &= ~m;
    }
}

// Blocks of kMetricWG threads over row segments: x from the block column,
// rows strided by the grid's height.  A pixel is a boundary pixel when a
// 4-neighbour inside the image has another label; the clamped neighbour of a
// border pixel is the pixel itself, which never differs.
__global__ __launch_bounds__(kMetricWG) void k_metric_pixels(MetricGeom g, const int* __restrict__ S,
                                                             const int* __restrict__ G,
                                                             unsigned* __restrict__ table,
                                                             unsigned* __restrict__ perim,
                                                             unsigned long long* __restrict__ smap,
                                                             unsigned long long* __restrict__ gmap) {
    const int x = blockIdx.x * kMetricWG + threadIdx.x;
    const int word = (blockIdx.x * kMetricWG + (threadIdx.x & ~63)) >> 6;
    const bool store = word < g.Wq && (threadIdx.x & 63) == 0;
    const bool in = x < g.W;
    const int xc = min(x, g.W - 1), xl = max(xc - 1, 0), xr = min(xc + 1, g.W - 1);
    for (int y = blockIdx.y; y < g.H; y += gridDim.y) {  // uniform
        const long long row = (long long)y * g.W;
        const long long up = (long long)max(y - 1, 0) * g.W;
        const long long dn = (long long)min(y + 1, g.H - 1) * g.W;
        const int k = S[row + xc], i = G[row + xc];
        const int sl = S[row + xl], sr = S[row + xr], su = S[up + xc], sd = S[dn + xc];
        const int gl = G[row + xl], gr = G[row + xr], gu = G[up + xc], gd = G[dn + xc];
        const bool dl = sl != k, dr = sr != k, du = su != k, dd = sd != k;
        const bool sb = in && (dl || dr || du || dd);
        const bool gb = in && (gl != i || gr != i || gu != i || gd != i);
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
        wave_count(table, perim, g.R, ok, k, i, e0, e1, e2);
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
__global__ __launch_bounds__(kMetricWG) void k_metric_recall(MetricGeom g,
                                                             const unsigned long long* __restrict__ smap,
                                                             const unsigned long long* __restrict__ gmap,
                                                             unsigned long long* __restrict__ cnt) {
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
        for (int dy = -g.r; dy <= g.r && (gw & ~d) != 0ULL; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= g.H) continue;
            int a = -1;                               // largest |dx| inside the disc
            while (a < g.r && (float)((a + 1) * (a + 1) + dy * dy) < g.eps2) ++a;
            if (a < 0) continue;
            const unsigned long long* rw = smap + (long long)yy * g.Wq;
            const unsigned long long lo = w > 0 ? rw[w - 1] : 0ULL;
            const unsigned long long hi = w + 1 < g.Wq ? rw[w + 1] : 0ULL;
            d |= dilate_mid(lo, rw[w], hi, a);
        }
        hit += (unsigned long long)__popcll(gw & d);
    }
    for (int o = 32; o > 0; o >>= 1) {
        gb += __shfl_xor(gb, o, 64);
        hit += __shfl_xor(hit, o, 64);
        sb += __shfl_xor(sb, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&cnt[0], gb);
        atomicAdd(&cnt[1], hit);
        atomicAdd(&cnt[2], sb);
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
                                                       const unsigned long long* __restrict__ cnt,
                                                       double* __restrict__ out) {
    __shared__ unsigned long long rm[1024], ru[1024];
    __shared__ double rc[1024];
    const int tid = threadIdx.x;
    unsigned long long m = 0, u = 0;
    double c = 0.0;
    for (int k = tid; k < g.K; k += 1024) {
        m += row_max[k];
        u += row_ue[k];
        c += row_co[k];
    }
    rm[tid] = m;
    ru[tid] = u;
    rc[tid] = c;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (tid < h) {
            rm[tid] += rm[tid + h];
            ru[tid] += ru[tid + h];
            rc[tid] += rc[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double N = (double)g.W * (double)g.H;
        out[0] = cnt[0] ? (double)cnt[1] / (double)cnt[0] : 1.0;   // BR
        out[1] = (double)rm[0] / N;                                 // ASA
        out[2] = (double)ru[0] / N;                                 // UE
        out[3] = rc[0] / N;                                         // CO
        out[4] = (double)cnt[0];                                    // |B(G)|
        out[5] = (double)cnt[2];                                    // |B(S)|
    }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

size_t metrics_workspace_bytes(int W, int H, int K, int R) {
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t table = (size_t)K * (size_t)R * 4, perim = (size_t)K * 4;
    const size_t rows = (size_t)K * 8 * 3, cnt = 64;
    const size_t map = (size_t)H * (size_t)((W + 63) / 64) * 8;
    return up(table) + up(perim) + up(rows) + up(cnt) + 2 * up(map);
}

int launch_metrics(int W, int H, const int* S, int K, const int* G, int R, float eps, double* out,
                   void* ws, hipStream_t st) {
    MetricGeom g;
    g.W = W; g.H = H; g.K = K; g.R = R;
    g.Wq = (W + 63) / 64;
    g.r = (int)ceilf(eps) - 1;
    g.eps2 = eps * eps;
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
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(b + off);
    off += up(64);
    const size_t map = (size_t)H * g.Wq;
    unsigned long long* smap = reinterpret_cast<unsigned long long*>(b + off);
    unsigned long long* gmap = smap + up(map * 8) / 8;
    // table, perim (contiguous up to row_max) and the counters start at zero;
    // every bitmap word is written by k_metric_pixels
    const long long zero_words = (long long)(reinterpret_cast<char*>(row_max) - b) / 4;
    const unsigned zb = (unsigned)std::min<long long>((zero_words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u32, dim3(zb), dim3(256), 0, st, table, zero_words);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(cnt), 16);
    // about 2048 blocks: whole rows, the row stride set by the grid height
    const int bx = (W + kMetricWG - 1) / kMetricWG;
    const int by = std::max(1, std::min(H, std::max(1, 2048 / bx)));
    hipLaunchKernelGGL(k_metric_pixels, dim3((unsigned)bx, (unsigned)std::min(by, 65535)),
                       dim3(kMetricWG), 0, st, g, S, G, table, perim, smap, gmap);
    const long long rb = std::min<long long>(((long long)map + kMetricWG - 1) / kMetricWG, 2048);
    hipLaunchKernelGGL(k_metric_recall, dim3((unsigned)rb), dim3(kMetricWG), 0, st, g, smap, gmap,
                       cnt);
    hipLaunchKernelGGL(k_metric_rows, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, st, g, table,
                       perim, row_max, row_ue, row_co);
    hipLaunchKernelGGL(k_metric_final, dim3(1), dim3(1024), 0, st, g, row_max, row_ue, row_co, cnt,
                       out);
    return hipGetLastError();
}

}  // namespace scalp
