// scalp_metrics.hip -- superpixel quality metrics of Sec. III-A.2 on the GPU:
// boundary recall (Eq. (5)), achievable segmentation accuracy (Eq. (6)),
// undersegmentation error (Eq. (7)) and compactness (Eq. (8)) of a label map
// against a ground-truth partition.
//
//   k_metric_pixels  one pass over the pixels: the overlap table
//                    |S_k n G_i| (32-bit atomics, one per distinct pair
//                    among a wave's pixels), the perimeter of every
//                    superpixel in pixel edges (4-connectivity, image border
//                    included), and the boundary-recall counts (ground-truth
//                    boundary pixels, and those with a superpixel boundary
//                    pixel at distance < epsilon), reduced per workgroup.
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
    int r;          // neighbourhood half-width for boundary recall
    float eps2;     // epsilon^2
};

__device__ __forceinline__ int label_at(const int* L, int W, int H, int x, int y) {
    return L[(long long)y * W + x];
}

// p is a boundary pixel of L: a 4-neighbour inside the image differs.
__device__ __forceinline__ bool is_boundary(const int* L, int W, int H, int x, int y) {
    const int v = label_at(L, W, H, x, y);
    return (x + 1 < W && label_at(L, W, H, x + 1, y) != v) ||
           (x > 0 && label_at(L, W, H, x - 1, y) != v) ||
           (y + 1 < H && label_at(L, W, H, x, y + 1) != v) ||
           (y > 0 && label_at(L, W, H, x, y - 1) != v);
}

// Adds 1 to table[k * R + i] for every lane of the wave with `ok`, one
// atomic per distinct (k, i) among the lanes: a wave covers 64 neighbouring
// pixels, which mostly share their superpixel and region, and atomics on one
// word serialise.
__device__ __forceinline__ void wave_count(unsigned* __restrict__ table, int R, bool ok, int k,
                                           int i) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(ok);
    while (pending != 0ULL) {                         // uniform over the wave
        const int leader = __ffsll((long long)pending) - 1;
        const int lk = __builtin_amdgcn_readlane(k, leader);
        const int li = __builtin_amdgcn_readlane(i, leader);
        const unsigned long long m = __ballot(ok && k == lk && i == li) & pending;
        if (lane == leader) atomicAdd(&table[(long long)lk * R + li], (unsigned)__popcll(m));
        pending &= ~m;
    }
}

// Blocks of kMetricWG threads over row segments: x from the block column,
// rows strided by the grid's height.
__global__ __launch_bounds__(kMetricWG) void k_metric_pixels(MetricGeom g, const int* __restrict__ S,
                                                             const int* __restrict__ G,
                                                             unsigned* __restrict__ table,
                                                             unsigned* __restrict__ perim,
                                                             unsigned long long* __restrict__ cnt) {
    __shared__ unsigned long long red[3][kMetricWG];
    unsigned long long gb = 0, hit = 0, sb = 0;
    const int x = blockIdx.x * kMetricWG + threadIdx.x;
    for (int y = blockIdx.y; y < g.H; y += gridDim.y) {  // uniform
        const bool in = x < g.W;
        const long long p = (long long)y * g.W + x;
        const int k = in ? S[p] : -1, i = in ? G[p] : -1;
        const bool ok = k >= 0 && k < g.K && i >= 0 && i < g.R;
        wave_count(table, g.R, ok, k, i);
        if (!in) continue;
        if (ok) {
            unsigned e = 0;
            e += (x + 1 >= g.W || S[p + 1] != k) ? 1u : 0u;
            e += (x == 0 || S[p - 1] != k) ? 1u : 0u;
            e += (y + 1 >= g.H || S[p + g.W] != k) ? 1u : 0u;
            e += (y == 0 || S[p - g.W] != k) ? 1u : 0u;
            if (e) atomicAdd(&perim[k], e);
        }
        if (is_boundary(S, g.W, g.H, x, y)) ++sb;
        if (is_boundary(G, g.W, g.H, x, y)) {
            ++gb;
            bool found = false;
            for (int dy = -g.r; dy <= g.r && !found; ++dy)
                for (int dx = -g.r; dx <= g.r && !found; ++dx) {
                    if ((float)(dx * dx + dy * dy) >= g.eps2) continue;
                    const int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= g.W || qy < 0 || qy >= g.H) continue;
                    found = is_boundary(S, g.W, g.H, qx, qy);
                }
            hit += found ? 1ULL : 0ULL;
        }
    }
    const int tid = threadIdx.x;
    red[0][tid] = gb;
    red[1][tid] = hit;
    red[2][tid] = sb;
    __syncthreads();
    for (int h = kMetricWG / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int v = 0; v < 3; ++v) red[v][tid] += red[v][tid + h];
        __syncthreads();
    }
    if (tid < 3) atomicAdd(&cnt[tid], red[tid][0]);
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

size_t metrics_workspace_bytes(long long N, int K, int R) {
    const size_t table = (size_t)K * (size_t)R * 4, perim = (size_t)K * 4;
    const size_t rows = (size_t)K * 8 * 3, cnt = 64;
    (void)N;
    return ((table + 255) / 256 + (perim + 255) / 256 + (rows + 255) / 256 + 1) * 256 + cnt;
}

int launch_metrics(int W, int H, const int* S, int K, const int* G, int R, float eps, double* out,
                   void* ws, hipStream_t st) {
    MetricGeom g;
    g.W = W; g.H = H; g.K = K; g.R = R;
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
    // table, perim (contiguous up to row_max) and the counters start at zero
    const long long zero_words = (long long)(reinterpret_cast<char*>(row_max) - b) / 4;
    const unsigned zb = (unsigned)std::min<long long>((zero_words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u32, dim3(zb), dim3(256), 0, st, table, zero_words);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(cnt), 16);
    // about 2048 blocks: whole rows, the row stride set by the grid height
    const int bx = (W + kMetricWG - 1) / kMetricWG;
    const int by = std::max(1, std::min(H, std::max(1, 2048 / bx)));
    hipLaunchKernelGGL(k_metric_pixels, dim3((unsigned)bx, (unsigned)std::min(by, 65535)),
                       dim3(kMetricWG), 0, st, g, S, G, table, perim, cnt);
    hipLaunchKernelGGL(k_metric_rows, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, st, g, table,
                       perim, row_max, row_ue, row_co);
    hipLaunchKernelGGL(k_metric_final, dim3(1), dim3(1024), 0, st, g, row_max, row_ue, row_co, cnt,
                       out);
    return hipGetLastError();
}

}  // namespace scalp
