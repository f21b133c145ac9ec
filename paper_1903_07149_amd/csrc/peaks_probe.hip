// peaks_probe.hip -- measures the issue and bandwidth ceilings that bound the
// SCALP path kernels on this GPU: FP32 add/mul issue rate (separate multiply
// and add, no FMA contraction, no packed FP32: the operation mix of the path
// distance), 32-bit integer add/xor issue rate, an even FP32/integer mix (the
// path walk's), and conflict-free ds_read_b128 LDS bandwidth.  Every kernel
// runs a fixed, bounded loop over registers or a 64 KiB LDS array.
#include <hip/hip_runtime.h>
#include <cstdio>
#define CHECK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__global__ __launch_bounds__(256) void k_valu(float* out, int iters, float x, float y) {
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < iters; ++i) {
        // 16 independent-ish ops per iteration: 8 mul + 8 add (no contraction)
        a0 = a0 * x; a1 = a1 * x; a2 = a2 * x; a3 = a3 * x; a4 = a4 * x; a5 = a5 * x; a6 = a6 * x; a7 = a7 * x;
        a0 = a0 + y; a1 = a1 + y; a2 = a2 + y; a3 = a3 + y; a4 = a4 + y; a5 = a5 + y; a6 = a6 + y; a7 = a7 + y;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

__global__ __launch_bounds__(256) void k_int(unsigned* out, int iters, unsigned x) {
    unsigned a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < iters; ++i) {
        a0 += x; a1 += a0; a2 += x; a3 += a2; a4 += x; a5 += a4; a6 += x; a7 += a6;
        a0 ^= a7; a1 += x; a2 ^= a1; a3 += x; a4 ^= a3; a5 += x; a6 ^= a5; a7 += x;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

__global__ __launch_bounds__(256) void k_mix(float* out, int iters, float x, float y, unsigned u) {
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3;
    unsigned b0 = threadIdx.x, b1 = b0 + 1, b2 = b0 + 2, b3 = b0 + 3;
    for (int i = 0; i < iters; ++i) {
        a0 = a0 * x; b0 += u; a1 = a1 * x; b1 ^= b0; a2 = a2 * x; b2 += u; a3 = a3 * x; b3 ^= b2;
        a0 = a0 + y; b0 ^= b3; a1 = a1 + y; b1 += u; a2 = a2 + y; b2 ^= b1; a3 = a3 + y; b3 += u;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + (float)(b0 + b1 + b2 + b3);
}

__global__ __launch_bounds__(256) void k_lds(float* out, int iters) {
    __shared__ float4 t[4096];          // 64 KiB
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) t[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    float4 acc = make_float4(0, 0, 0, 0);
    unsigned idx = threadIdx.x;          // consecutive lanes -> consecutive 16 B: conflict-free
    for (int i = 0; i < iters; ++i) {
        const float4 v0 = t[(idx) & 4095];
        const float4 v1 = t[(idx + 256) & 4095];
        const float4 v2 = t[(idx + 512) & 4095];
        const float4 v3 = t[(idx + 768) & 4095];
        acc.x += (v0.x + v1.x) + (v2.x + v3.x);
        acc.y += (v0.y + v1.y) + (v2.y + v3.y);
        acc.z += (v0.z + v1.z) + (v2.z + v3.z);
        acc.w += (v0.w + v1.w) + (v2.w + v3.w);
        idx += 1024;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

int main() {
    int dev = 0, cus = 0, clk = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, dev));
    printf("CUs %d, clock %d kHz\n", cus, clk);
    const int blocks = cus * 16, threads = 256;
    float* out;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a)); CHECK(hipEventCreate(&b));
    const int iters = 20000;
    for (int rep = 0; rep < 3; ++rep) {
        hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 0.001f);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(a));
        hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 0.001f);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms; CHECK(hipEventElapsedTime(&ms, a, b));
        double ops = (double)blocks * threads * iters * 16;
        printf("VALU fp32 add/mul: %.3f ms, %.2f T lane-ops/s\n", ms, ops / (ms * 1e-3) / 1e12);
    }
    for (int rep = 0; rep < 2; ++rep) {
        hipLaunchKernelGGL(k_int, dim3(blocks), dim3(threads), 0, 0, (unsigned*)out, iters, 7u);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(a));
        hipLaunchKernelGGL(k_int, dim3(blocks), dim3(threads), 0, 0, (unsigned*)out, iters, 7u);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms; CHECK(hipEventElapsedTime(&ms, a, b));
        double ops = (double)blocks * threads * iters * 16;
        printf("VALU int add/xor: %.3f ms, %.2f T lane-ops/s\n", ms, ops / (ms * 1e-3) / 1e12);
        hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 0.001f, 7u);
        CHECK(hipEventRecord(a));
        hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 0.001f, 7u);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        CHECK(hipEventElapsedTime(&ms, a, b));
        printf("VALU 8 fp32 + 8 int: %.3f ms, %.2f T lane-ops/s\n", ms, ops / (ms * 1e-3) / 1e12);
    }
    const int liters = 20000;
    for (int rep = 0; rep < 3; ++rep) {
        hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(threads), 0, 0, out, liters);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(a));
        hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(threads), 0, 0, out, liters);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms; CHECK(hipEventElapsedTime(&ms, a, b));
        double bytes = (double)blocks * threads * liters * 4 * 16;
        printf("LDS ds_read_b128: %.3f ms, %.2f TB/s (%.1f B/clk/CU at %d kHz)\n", ms, bytes / (ms * 1e-3) / 1e12,
               bytes / (ms * 1e-3) / cus / (clk * 1e3), clk);
    }
    CHECK(hipFree(out));
    return 0;
}
