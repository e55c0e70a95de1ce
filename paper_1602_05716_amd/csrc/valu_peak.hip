// valu_peak.hip -- measures the vector-ALU issue rates that bound the sweep
// kernel's pair-term loop on this device: v_rsq_f32 alone, v_fma_f32 alone,
// and the two interleaved in the pair term's proportion (2 rsq : 13 other
// ops), to see whether the transcendental unit overlaps with the FMA pipe.
//
// Every lane runs 8 independent dependency chains so that latency is hidden;
// 16 waves per CU.  Prints one JSON line with rates in lane-operations per
// clock per CU at the nominal 2.4 GHz and per second.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <string>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e = (x);                                                               \
        if (e != hipSuccess) {                                                            \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));                   \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

constexpr int kChains = 8;
constexpr int kIters = 512;

__global__ void __launch_bounds__(256) rsq_only(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.001f * (threadIdx.x + c);
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_rsqf(x[c]);
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) fma_only(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 0.001f * (threadIdx.x + c);
    const float a = 0.999f, b = 0.0001f;
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// per chain and iteration: 2 rsq and 13 fma (the pair term's mix)
__global__ void __launch_bounds__(256) mixed(float* out, float seed) {
    float x[kChains], y[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c] = seed + 0.001f * (threadIdx.x + c);
        y[c] = seed + 0.002f * (threadIdx.x + c);
    }
    const float a = 0.999f, b = 0.0001f;
    for (int it = 0; it < kIters / 8; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            x[c] = __builtin_amdgcn_rsqf(x[c]);
            y[c] = __builtin_amdgcn_rsqf(y[c]);
#pragma unroll
            for (int k = 0; k < 13; ++k) x[c] = __builtin_fmaf(x[c], a, b);
        }
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c] + y[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// plain streaming copy, used to calibrate the HBM traffic counters
__global__ void __launch_bounds__(256) copy_f4(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename K>
double time_ms(K kernel, int blocks, float* out) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, 0, out, 1.5f);
    CHECK(hipDeviceSynchronize());
    double best = 1e30;
    for (int r = 0; r < 5; ++r) {
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, 0, out, 1.5f);
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
    }
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return best;
}

int main(int argc, char** argv) {
    if (argc > 1 && std::string(argv[1]) == "--copy") {
        // 256 MiB read + 256 MiB written, one launch
        const size_t n = (size_t)256 << 20 >> 4;
        float4 *a = nullptr, *b = nullptr;
        CHECK(hipMalloc(&a, n * sizeof(float4)));
        CHECK(hipMalloc(&b, n * sizeof(float4)));
        CHECK(hipMemset(a, 1, n * sizeof(float4)));
        hipLaunchKernelGGL(copy_f4, dim3(8192), dim3(256), 0, 0, a, b, n);
        CHECK(hipDeviceSynchronize());
        std::printf("{\"copy_bytes_read\": %zu, \"copy_bytes_written\": %zu}\n", n * sizeof(float4), n * sizeof(float4));
        CHECK(hipFree(a));
        CHECK(hipFree(b));
        return 0;
    }
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int cus = p.multiProcessorCount;
    const int blocks = cus * 4 * 16;  // 16 waves per CU, 16 rounds
    float* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * (size_t)blocks * 256));
    const double lanes = (double)blocks * 256;
    const double clk = 2.4e9;
    const double t_rsq = time_ms(rsq_only, blocks, out) * 1e-3;
    const double t_fma = time_ms(fma_only, blocks, out) * 1e-3;
    const double t_mix = time_ms(mixed, blocks, out) * 1e-3;
    const double n_rsq = lanes * kChains * kIters;
    const double n_fma = lanes * kChains * kIters;
    const double n_mix_rsq = lanes * kChains * (kIters / 8) * 2;
    const double n_mix_fma = lanes * kChains * (kIters / 8) * 13;
    const double r_rsq = n_rsq / t_rsq, r_fma = n_fma / t_fma;
    // if the two pipes overlapped, the mixed time would be max(), else the sum
    const double t_sum = n_mix_rsq / r_rsq + n_mix_fma / r_fma;
    const double t_max = n_mix_rsq / r_rsq > n_mix_fma / r_fma ? n_mix_rsq / r_rsq : n_mix_fma / r_fma;
    std::printf("{\"cus\": %d, \"rsq_per_s\": %.4e, \"fma_per_s\": %.4e, "
                "\"rsq_lanes_per_clk_cu\": %.2f, \"fma_lanes_per_clk_cu\": %.2f, "
                "\"mixed_s\": %.4e, \"mixed_if_serial_s\": %.4e, \"mixed_if_overlapped_s\": %.4e}\n",
                cus, r_rsq, r_fma, r_rsq / clk / cus, r_fma / clk / cus, t_mix, t_sum, t_max);
    CHECK(hipFree(out));
    return 0;
}
