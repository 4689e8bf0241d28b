// Vector-ALU issue-rate calibration: sixteen independent chains of one 32-bit
// VALU instruction per lane, at full occupancy, timed with HIP events.  Gives
// the achievable wave-instructions per second for the bitwise and shift forms
// the bit-sliced Life kernels issue (two-operand VOP2 and three-operand VOP3
// encodings) and for binary32 fused multiply-adds (the operation of the
// datasheet's vector FP32 rate), the ceiling against which the kernels'
// counter-measured issue rate is read, and the shader clock during such a
// loop.  Prints one JSON line per instruction and grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "HIP error %s (%s:%d)\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

constexpr int kChains = 16;

template <int OP>
__global__ void __launch_bounds__(256) k_valu(uint32_t *out, int iters, uint32_t seed)
{
    uint32_t a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = seed * (threadIdx.x + 1) + i * 0x9E3779B9u + blockIdx.x;
    const uint32_t m = seed ^ threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            const uint32_t b = a[(i + 3) & (kChains - 1)];
            if constexpr (OP == 0) asm volatile("v_and_b32 %0, %0, %1" : "+v"(a[i]) : "v"(m));
            if constexpr (OP == 1) asm volatile("v_lshrrev_b32 %0, 3, %0" : "+v"(a[i]));
            if constexpr (OP == 2) asm volatile("v_or3_b32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(m), "v"(b));
            if constexpr (OP == 3) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[i]) : "v"(m), "v"(b));
            if constexpr (OP == 4) asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(m), "v"(b));
            if constexpr (OP == 5) asm volatile("v_bfe_u32 %0, %0, 5, 1" : "+v"(a[i]));
            if constexpr (OP == 6) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a[i]) : "v"(m), "v"(b));
            if constexpr (OP == 7) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(m), "v"(b));
            if constexpr (OP == 8) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(m));
            if constexpr (OP == 9) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(m));
            if constexpr (OP == 10) asm volatile("v_lshl_or_b32 %0, %0, 3, %1" : "+v"(a[i]) : "v"(b));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
}

// Shader clock during a VALU-bound loop: the first lane of every wave reads the
// shader-clock counter (s_memtime) and the constant-rate real-time counter
// (s_memrealtime) before and after 4096 iterations of the v_and_b32 chains.
__global__ void __launch_bounds__(256) k_clock(unsigned long long *ticks, uint32_t *out, int iters, uint32_t seed)
{
    uint32_t a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = seed * (threadIdx.x + 1) + i * 0x9E3779B9u + blockIdx.x;
    const uint32_t m = seed ^ threadIdx.x;
    const unsigned long long c0 = clock64(), w0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) asm volatile("v_and_b32 %0, %0, %1" : "+v"(a[i]) : "v"(m));
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    const unsigned long long c1 = clock64(), w1 = wall_clock64();
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
    if ((threadIdx.x & 63) == 0) {
        const size_t w = (size_t)blockIdx.x * 4 + threadIdx.x / 64;
        ticks[2 * w] = c1 - c0;
        ticks[2 * w + 1] = w1 - w0;
    }
}

template <int OP>
int run(const char *name, uint32_t *d, int grid, int iters, int cus)
{
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_valu<OP>, dim3(grid), dim3(256), 0, 0, d, iters, 7u);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    const int reps = 5;
    CHECK(hipEventRecord(e0, 0));
    for (int rep = 0; rep < reps; ++rep) hipLaunchKernelGGL(k_valu<OP>, dim3(grid), dim3(256), 0, 0, d, iters, 7u);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    const double insts = (double)grid * 4 * iters * kChains;  // wave-instructions (4 waves per workgroup)
    printf("{\"inst\": \"%s\", \"workgroups\": %d, \"ms\": %.4f, \"G_wave_insts_per_s\": %.1f, "
           "\"per_cu_per_clock_at_2.4GHz\": %.3f}\n",
           name, grid, ms, insts / ms / 1e6, insts / (ms * 1e-3) / cus / 2.4e9);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    // 4, 6 and 8 (the maximum) waves per SIMD, the last in two rounds
    const int grids[3] = {cus * 4, cus * 6, cus * 16};
    uint32_t *d = nullptr;
    CHECK(hipMalloc(&d, (size_t)grids[2] * 256 * sizeof(uint32_t)));
    printf("{\"device\": \"%s\", \"compute_units\": %d}\n", prop.name, cus);
    for (int grid : grids) {
        const int iters = 4096;
        if (run<0>("v_and_b32 (VOP2)", d, grid, iters, cus) || run<1>("v_lshrrev_b32 (VOP2)", d, grid, iters, cus) ||
            run<2>("v_or3_b32 (VOP3)", d, grid, iters, cus) || run<3>("v_bitop3_b32 (VOP3)", d, grid, iters, cus) ||
            run<4>("v_and_or_b32 (VOP3)", d, grid, iters, cus) || run<5>("v_bfe_u32 (VOP3)", d, grid, iters, cus) ||
            run<6>("v_fmac_f32 (VOP2)", d, grid, iters, cus) || run<7>("v_fma_f32 (VOP3)", d, grid, iters, cus) ||
            run<8>("v_add_u32 (VOP2)", d, grid, iters, cus) || run<9>("v_xor_b32 (VOP2)", d, grid, iters, cus) ||
            run<10>("v_lshl_or_b32 (VOP3)", d, grid, iters, cus))
            return 1;
    }
    // shader clock under load: per-wave shader-clock ticks over real-time ticks
    int wall_khz = 0;
    CHECK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0));
    const int grid = grids[2];
    unsigned long long *dt = nullptr;
    CHECK(hipMalloc(&dt, (size_t)grid * 4 * 2 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_clock, dim3(grid), dim3(256), 0, 0, dt, d, 4096, 7u);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    std::vector<unsigned long long> h((size_t)grid * 4 * 2);
    CHECK(hipMemcpy(h.data(), dt, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    std::vector<double> mhz;
    for (size_t w = 0; w < h.size() / 2; ++w)
        if (h[2 * w + 1]) mhz.push_back((double)h[2 * w] / (double)h[2 * w + 1] * wall_khz / 1e3);
    std::sort(mhz.begin(), mhz.end());
    if (!mhz.empty())
        printf("{\"shader_clock_mhz\": {\"median\": %.1f, \"min\": %.1f, \"max\": %.1f, \"waves\": %zu}, "
               "\"wall_clock_khz\": %d}\n",
               mhz[mhz.size() / 2], mhz.front(), mhz.back(), mhz.size(), wall_khz);
    CHECK(hipFree(dt));
    CHECK(hipFree(d));
    return 0;
}
