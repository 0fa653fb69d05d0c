// Issue-rate microbenchmark for non-packed binary32 vector ALU instructions on
// gfx950: every thread runs 8 independent dependency chains of one operation
// (fused multiply-add, multiply or add) for `iters` iterations, so the SIMDs
// always have independent instructions to issue.  Built with packed-fp32
// instructions disabled, like the library; the host times the kernel with HIP
// events and reports wave-instructions and lane-operations per second.
// Measurement infrastructure (no part of the library).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

template <int OP>
__global__ __launch_bounds__(256) void chains(float* out, float a, float b, int iters)
{
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (OP == 0) x[c] = fmaf(x[c], a, b);
            else if constexpr (OP == 1) x[c] = x[c] * a;
            else x[c] = x[c] + b;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    if (s == 1234.5f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;   // keeps the chains live
}

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));         \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

template <int OP>
static double run(float* out, int blocks, int iters, int reps)
{
    hipEvent_t s, e;
    CHECK(hipEventCreate(&s));
    CHECK(hipEventCreate(&e));
    hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, nullptr, out, 0.999f, 1e-4f, iters);   // warm-up
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(s, nullptr));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, nullptr, out, 0.999f, 1e-4f, iters);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e, nullptr));
    CHECK(hipEventSynchronize(e));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, s, e));
    CHECK(hipEventDestroy(s));
    CHECK(hipEventDestroy(e));
    return ms / 1e3 / reps;
}

int main()
{
    int cus = 0, clock_khz = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    CHECK(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, 0));
    const int blocks = cus * 64, iters = 2048, reps = 5;
    float* out = nullptr;
    CHECK(hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)));
    const char* names[3] = {"fma", "mul", "add"};
    double sec[3] = {run<0>(out, blocks, iters, reps), run<1>(out, blocks, iters, reps),
                     run<2>(out, blocks, iters, reps)};
    const double lane_ops = (double)blocks * 256.0 * iters * 8.0;
    std::printf("{\"compute_units\": %d, \"clock_mhz\": %.0f, \"blocks\": %d, \"threads_per_block\": 256, "
                "\"iters\": %d, \"chains\": 8", cus, clock_khz / 1e3, blocks, iters);
    for (int i = 0; i < 3; ++i)
        std::printf(", \"%s\": {\"seconds\": %.6g, \"lane_ops_per_s\": %.6g, \"wave_insts_per_cu_clock\": %.4f}",
                    names[i], sec[i], lane_ops / sec[i], lane_ops / 64.0 / sec[i] / cus / (clock_khz * 1e3));
    std::printf("}\n");
    CHECK(hipFree(out));
    return 0;
}
