// The kernels' binary32 math functions evaluated on the GPU over every input of
// a range and compared with a reference (the oracle's function, passed in by
// the test) on host threads.  The cube root's device code starts from the
// device's own logarithm and exponential instructions, so only a device run
// checks it.  Test infrastructure: built by build() into
// tests/pins/libdevmath_gpu.so and loaded by tests/test_gpu_devmath.py.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "../../paper_2510_03964_amd/csrc/fwrs_device.hpp"

namespace {

constexpr uint64_t kChunk = uint64_t(1) << 25;   // inputs per device pass (128 MiB of results)

__global__ void cube_root_kernel(uint32_t lo, uint32_t stride, uint64_t n, float* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fwrs::cube_root(__builtin_bit_cast(float, (uint32_t)(lo + i * stride)));
}

__global__ void log2_unit_kernel(uint32_t m0, uint64_t n, float* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fwrs::log2_unit((uint32_t)(m0 + i - 1u) << 8);
}

// Counts the inputs (bit patterns in[i]) whose device result differs from ref.
template <typename In, typename Ref>
void compare(const std::vector<float>& got, uint64_t n, In in, Ref ref, int threads, int64_t& bad, uint32_t& first)
{
    std::vector<int64_t> count(threads, 0);
    std::vector<uint32_t> low(threads, 0xFFFFFFFFu);
    std::vector<std::thread> pool;
    for (int w = 0; w < threads; ++w)
        pool.emplace_back([&, w] {
            for (uint64_t i = (uint64_t)w; i < n; i += (uint64_t)threads) {
                const uint32_t x = in(i);
                const float b = ref(x);
                uint32_t ua, ub;
                std::memcpy(&ua, &got[i], 4);
                std::memcpy(&ub, &b, 4);
                if (ua != ub) {
                    ++count[w];
                    if (x < low[w]) low[w] = x;
                }
            }
        });
    for (auto& t : pool) t.join();
    for (int w = 0; w < threads; ++w) {
        bad += count[w];
        if (low[w] < first) first = low[w];
    }
}

}  // namespace

extern "C" {

// fwrs::cube_root on the GPU for every binary32 whose bit pattern is in [lo, hi)
// with the given stride, against reference(t) on the host.  Returns the number
// of differing inputs (-1 on a HIP error); *first = the smallest such bit
// pattern (0xFFFFFFFF if none).
int64_t gpu_cube_root_mismatches(uint32_t lo, uint32_t hi, uint32_t stride, float (*reference)(float), int threads,
                                 uint32_t* first)
{
    if (threads < 1) threads = 1;
    if (stride < 1) stride = 1;
    const uint64_t total = hi > lo ? ((uint64_t)hi - lo + stride - 1) / stride : 0;
    float* d = nullptr;
    if (hipMalloc(&d, kChunk * 4) != hipSuccess) return -1;
    std::vector<float> got(kChunk);
    int64_t bad = 0;
    uint32_t low = 0xFFFFFFFFu;
    for (uint64_t at = 0; at < total; at += kChunk) {
        const uint64_t n = total - at < kChunk ? total - at : kChunk;
        const uint32_t base = (uint32_t)(lo + at * stride);
        hipLaunchKernelGGL(cube_root_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, 0, base, stride, n, d);
        if (hipMemcpy(got.data(), d, n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipFree(d);
            return -1;
        }
        compare(got, n, [&](uint64_t i) { return (uint32_t)(base + i * stride); },
                [&](uint32_t x) { float t; std::memcpy(&t, &x, 4); return reference(t); }, threads, bad, low);
    }
    (void)hipFree(d);
    if (first) *first = low;
    return bad;
}

// fwrs::log2_unit on the GPU for every variate (m = 1 .. 2^24, bits = (m - 1) << 8)
// against reference(bits) on the host; as above.
int64_t gpu_log2_unit_mismatches(float (*reference)(uint32_t), int threads, uint32_t* first)
{
    if (threads < 1) threads = 1;
    const uint64_t total = uint64_t(1) << 24;
    float* d = nullptr;
    if (hipMalloc(&d, kChunk * 4) != hipSuccess) return -1;
    std::vector<float> got(kChunk);
    int64_t bad = 0;
    uint32_t low = 0xFFFFFFFFu;
    for (uint64_t at = 0; at < total; at += kChunk) {
        const uint64_t n = total - at < kChunk ? total - at : kChunk;
        const uint32_t m0 = (uint32_t)(1 + at);
        hipLaunchKernelGGL(log2_unit_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, 0, m0, n, d);
        if (hipMemcpy(got.data(), d, n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipFree(d);
            return -1;
        }
        compare(got, n, [&](uint64_t i) { return (uint32_t)(m0 + i - 1u) << 8; },
                [&](uint32_t x) { return reference(x); }, threads, bad, low);
    }
    (void)hipFree(d);
    if (first) *first = low;
    return bad;
}

}  // extern "C"
