// scalp_maps.hip -- per-pixel maps around the clustering path.
//
//   k_boundary_frequency  fraction of a stack of label maps in which a pixel
//                         is a superpixel boundary pixel (a 4-neighbour inside
//                         the image carries another label): the multi-scale
//                         boundary map whose thresholds give the
//                         precision-recall curves of Sec. III-A.2.
//   k_gradient_*          a soft contour prior computed on the device: the
//                         central-difference gradient magnitude of the Lab
//                         image (replicated borders), divided by its maximum,
//                         in FP64 and rounded once to FP32.  The paper feeds
//                         the contour map C of Sec. II-D from an external
//                         detector (Sec. II-E); this is a detector-free
//                         stand-in that needs no trained model.
//   k_prepare_gradient    the same prior fused into the packing of
//                         (l, a, b, w): C never reaches memory.
#include <algorithm>

#include "scalp_internal.h"

namespace scalp {
namespace {

// All map kernels run 256-thread blocks over row segments: x from the block
// column, rows strided by the grid's height (no per-pixel division).
#define FOR_PIXELS(W, H)                                                     \
    const int x = blockIdx.x * 256 + threadIdx.x;                            \
    for (int y = blockIdx.y; y < (H); y += gridDim.y)                        \
        if (x < (W))

__global__ __launch_bounds__(256) void k_boundary_frequency(int W, int H, int n,
                                                            const int* __restrict__ labels,
                                                            float* __restrict__ out) {
    const long long N = (long long)W * H;
    FOR_PIXELS(W, H) {
        const long long p = (long long)y * W + x;
        int c = 0;
        for (int s = 0; s < n; ++s) {
            const int* L = labels + N * s;
            const int v = L[p];
            c += ((x + 1 < W && L[p + 1] != v) || (x > 0 && L[p - 1] != v) ||
                  (y + 1 < H && L[p + W] != v) || (y > 0 && L[p - W] != v)) ? 1 : 0;
        }
        out[p] = (float)c / (float)n;
    }
}

// Squared gradient magnitude of pixel p in FP64 (central differences,
// replicated borders), channels summed in order.
__device__ __forceinline__ double grad_sq(const float* __restrict__ lab, int W, int H, int x, int y) {
    const int xl = x > 0 ? x - 1 : 0, xr = x + 1 < W ? x + 1 : W - 1;
    const int yu = y > 0 ? y - 1 : 0, yd = y + 1 < H ? y + 1 : H - 1;
    const long long r = 3LL * ((long long)y * W + xr), l = 3LL * ((long long)y * W + xl);
    const long long d = 3LL * ((long long)yd * W + x), u = 3LL * ((long long)yu * W + x);
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double gx = 0.5 * ((double)lab[r + c] - (double)lab[l + c]);
        const double gy = 0.5 * ((double)lab[d + c] - (double)lab[u + c]);
        s = s + (gx * gx + gy * gy);
    }
    return s;
}

__device__ __forceinline__ double grad_mag(const float* __restrict__ lab, int W, int H, int x, int y) {
    return sqrt(grad_sq(lab, W, H, x, y));
}

__global__ __launch_bounds__(256) void k_gradient_max(const float* __restrict__ lab, int W, int H,
                                                      unsigned long long* __restrict__ mx) {
    __shared__ unsigned long long red[256];
    unsigned long long m = 0;
    FOR_PIXELS(W, H) {
        // squared magnitudes are >= 0, so their FP64 bit patterns order like
        // the values; the correctly rounded square root is monotone, so the
        // root of the largest square is the largest magnitude
        const unsigned long long b = (unsigned long long)__double_as_longlong(grad_sq(lab, W, H, x, y));
        m = b > m ? b : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + h] ? red[threadIdx.x]
                                                                       : red[threadIdx.x + h];
        __syncthreads();
    }
    // one of kGradSlots words per block; only a value above what the slot
    // holds goes to the atomic (a stale read only costs an atomic that
    // changes nothing)
    unsigned long long* slot = mx + (blockIdx.y * gridDim.x + blockIdx.x) % kGradSlots * kGradStride;
    if (threadIdx.x == 0 && red[0] > *reinterpret_cast<volatile unsigned long long*>(slot))
        atomicMax(slot, red[0]);
}

// Largest of the kGradSlots partial maxima, reduced within each wave (every
// wave of the reader computes the same value).
__device__ __forceinline__ double grad_max_of(const unsigned long long* __restrict__ mx) {
    const int lane = threadIdx.x & 63;
    unsigned long long v = lane < kGradSlots ? mx[lane * kGradStride] : 0ULL;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return sqrt(__longlong_as_double((long long)v));
}

// Contour value of pixel p as the standalone map stores it (FP32).
__device__ __forceinline__ float contour_at(const float* __restrict__ lab, int W, int H, int x, int y,
                                           double m) {
    return m > 0.0 ? (float)(grad_mag(lab, W, H, x, y) / m) : 0.0f;
}

__global__ __launch_bounds__(256) void k_gradient_normalise(const float* __restrict__ lab, int W,
                                                            int H,
                                                            const unsigned long long* __restrict__ mx,
                                                            float* __restrict__ out) {
    const double m = grad_max_of(mx);
    FOR_PIXELS(W, H) out[(long long)y * W + x] = contour_at(lab, W, H, x, y, m);
}

__global__ __launch_bounds__(256) void k_prepare_gradient(const float* __restrict__ lab, int W,
                                                          int H, float sigma,
                                                          const unsigned long long* __restrict__ mx,
                                                          float4* __restrict__ packed) {
    const double m = grad_max_of(mx);
    const double s2 = (double)sigma * (double)sigma;
    FOR_PIXELS(W, H) {
        const long long p = (long long)y * W + x;
        const double c = (double)contour_at(lab, W, H, x, y, m);
        const float w = (float)(1.0 - exp(-(c * c) / s2));
        packed[p] = make_float4(lab[3 * p], lab[3 * p + 1], lab[3 * p + 2], w);
    }
}

__global__ void k_zero_slots(unsigned long long* p) {
    if (threadIdx.x < kGradSlots) p[threadIdx.x * kGradStride] = 0ULL;
}

// About 2048 blocks of 256 threads: whole rows, the row stride set by the grid height.
dim3 grid_for(int W, int H) {
    const int bx = (W + 255) / 256;
    const int by = std::max(1, std::min(H, std::max(1, 2048 / bx)));
    return dim3((unsigned)bx, (unsigned)std::min(by, 65535));
}

}  // namespace

int launch_boundary_frequency(int W, int H, int n, const int* labels, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_boundary_frequency, grid_for(W, H), dim3(256), 0, s, W, H, n, labels, out);
    return hipGetLastError();
}

int launch_contour_from_lab(int W, int H, const float* lab, float* out, void* ws, hipStream_t s) {
    unsigned long long* mx = static_cast<unsigned long long*>(ws);
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(64), 0, s, mx);
    const dim3 b = grid_for(W, H);
    hipLaunchKernelGGL(k_gradient_max, dim3(b), dim3(256), 0, s, lab, W, H, mx);
    hipLaunchKernelGGL(k_gradient_normalise, dim3(b), dim3(256), 0, s, lab, W, H, mx, out);
    return hipGetLastError();
}

int launch_prepare_gradient(int W, int H, const float* lab, float sigma, float4* packed,
                            unsigned long long* mx, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(64), 0, s, mx);
    const dim3 b = grid_for(W, H);
    hipLaunchKernelGGL(k_gradient_max, dim3(b), dim3(256), 0, s, lab, W, H, mx);
    hipLaunchKernelGGL(k_prepare_gradient, dim3(b), dim3(256), 0, s, lab, W, H, sigma, mx, packed);
    return hipGetLastError();
}

}  // namespace scalp
