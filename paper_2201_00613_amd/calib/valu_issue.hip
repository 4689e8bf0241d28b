// Vector-ALU issue-rate calibration: sixteen independent chains of one 32-bit
// VALU instruction per lane, at full occupancy, timed with HIP events.  Gives
// the achievable wave-instructions per second for the bitwise and shift forms
// the bit-sliced Life kernels issue (two-operand VOP2 and three-operand VOP3
// encodings), the ceiling against which their counter-measured issue rate is
// read.  Prints one JSON line per instruction and grid.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

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
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
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
    const int grids[2] = {cus * 4, cus * 16};  // 4 and 8 (the maximum) waves per SIMD, the latter in two rounds
    uint32_t *d = nullptr;
    CHECK(hipMalloc(&d, (size_t)grids[1] * 256 * sizeof(uint32_t)));
    printf("{\"device\": \"%s\", \"compute_units\": %d}\n", prop.name, cus);
    for (int grid : grids) {
        const int iters = 4096;
        if (run<0>("v_and_b32 (VOP2)", d, grid, iters, cus) || run<1>("v_lshrrev_b32 (VOP2)", d, grid, iters, cus) ||
            run<2>("v_or3_b32 (VOP3)", d, grid, iters, cus) || run<3>("v_bitop3_b32 (VOP3)", d, grid, iters, cus) ||
            run<4>("v_and_or_b32 (VOP3)", d, grid, iters, cus) || run<5>("v_bfe_u32 (VOP3)", d, grid, iters, cus))
            return 1;
    }
    CHECK(hipFree(d));
    return 0;
}
