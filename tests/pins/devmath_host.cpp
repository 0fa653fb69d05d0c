// The kernel's binary32 math functions (cube root, log2 of a variate, CIE Lab,
// CIE94), compiled for the host from the same header the gfx950 library is
// built from, so that CPU tests can compare them with the oracle over every
// input of a range.  Test infrastructure, built for the host only
// (hipcc --cuda-host-only).
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "../../paper_2510_03964_amd/csrc/fwrs_device.hpp"

extern "C" {

float dev_cube_root(float t) { return fwrs::cube_root(t); }

float dev_log2_unit(uint32_t bits) { return fwrs::log2_unit(bits); }

void dev_lab(float r, float g, float b, float* lab)
{
    const float3 v = fwrs::rgb_to_lab(r, g, b);
    lab[0] = v.x;
    lab[1] = v.y;
    lab[2] = v.z;
}

float dev_de94(const float* ref, const float* x)
{
    return fwrs::cie94(make_float3(ref[0], ref[1], ref[2]), make_float3(x[0], x[1], x[2]));
}

int dev_lab_bounded(float r, float g, float b)
{
    return fwrs::lab_bounded(r, g, b) ? 1 : 0;
}

// Compares fwrs::cube_root with `reference` on every binary32 whose bit pattern
// is in [lo, hi) with the given stride, on `threads` threads.  Returns the
// number of inputs whose results differ bit for bit; *first is the bit pattern
// of the smallest such input (0xFFFFFFFF if none).
int64_t cube_root_mismatches(uint32_t lo, uint32_t hi, uint32_t stride, float (*reference)(float), int threads,
                             uint32_t* first)
{
    if (threads < 1) threads = 1;
    std::vector<int64_t> count(threads, 0);
    std::vector<uint32_t> bad(threads, 0xFFFFFFFFu);
    const uint64_t n = (hi > lo) ? ((uint64_t)hi - lo + stride - 1) / stride : 0;
    std::vector<std::thread> pool;
    for (int w = 0; w < threads; ++w) {
        pool.emplace_back([&, w] {
            for (uint64_t i = (uint64_t)w; i < n; i += (uint64_t)threads) {
                const uint32_t bits = lo + (uint32_t)(i * stride);
                float t;
                std::memcpy(&t, &bits, 4);
                const float a = fwrs::cube_root(t), b = reference(t);
                uint32_t ua, ub;
                std::memcpy(&ua, &a, 4);
                std::memcpy(&ub, &b, 4);
                if (ua != ub) {
                    ++count[w];
                    if (bits < bad[w]) bad[w] = bits;
                }
            }
        });
    }
    for (auto& th : pool) th.join();
    int64_t total = 0;
    uint32_t f = 0xFFFFFFFFu;
    for (int w = 0; w < threads; ++w) {
        total += count[w];
        if (bad[w] < f) f = bad[w];
    }
    if (first) *first = f;
    return total;
}

// The same for fwrs::log2_unit over every variate: m = (bits >> 8) + 1 for
// m = 1 .. 2^24 (bits = (m - 1) << 8).
int64_t log2_unit_mismatches(float (*reference)(uint32_t), int threads, uint32_t* first)
{
    if (threads < 1) threads = 1;
    std::vector<int64_t> count(threads, 0);
    std::vector<uint32_t> bad(threads, 0xFFFFFFFFu);
    std::vector<std::thread> pool;
    for (int w = 0; w < threads; ++w) {
        pool.emplace_back([&, w] {
            for (uint32_t m = 1u + (uint32_t)w; m <= (1u << 24); m += (uint32_t)threads) {
                const uint32_t bits = (m - 1u) << 8;
                const float a = fwrs::log2_unit(bits), b = reference(bits);
                uint32_t ua, ub;
                std::memcpy(&ua, &a, 4);
                std::memcpy(&ub, &b, 4);
                if (ua != ub) {
                    ++count[w];
                    if (bits < bad[w]) bad[w] = bits;
                }
            }
        });
    }
    for (auto& th : pool) th.join();
    int64_t total = 0;
    uint32_t f = 0xFFFFFFFFu;
    for (int w = 0; w < threads; ++w) {
        total += count[w];
        if (bad[w] < f) f = bad[w];
    }
    if (first) *first = f;
    return total;
}

}  // extern "C"
