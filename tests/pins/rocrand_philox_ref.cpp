// Independent reference for the oracle's Philox4x32-10: rocRAND's host-callable
// Philox4x32-10 engine.  A derived class reaches the engine's own ten-round
// block function so that an arbitrary (key, counter) pair can be evaluated
// without the engine's offset bookkeeping (whose 64-bit offset cannot express
// every 128-bit counter).  Test infrastructure, built for the host only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstddef>
#include <cstdint>

namespace {
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};
}  // namespace

extern "C" void ref_philox_many(const uint32_t* keys, const uint32_t* ctrs, uint32_t* out, size_t n)
{
    Probe probe;
    for (size_t i = 0; i < n; ++i) {
        const uint32_t* k = keys + 2 * i;
        const uint32_t* c = ctrs + 4 * i;
        uint4 r = probe.block(uint4{c[0], c[1], c[2], c[3]}, uint2{k[0], k[1]});
        out[4 * i + 0] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}

// The engine's public interface as a cross-check of the mapping above, valid
// while ctr1 < 2^30: seed = key1:key0, subsequence = ctr3:ctr2,
// offset = 4 * (ctr1:ctr0); four next() calls return the block's words.
extern "C" void ref_philox_engine_many(const uint32_t* keys, const uint32_t* ctrs, uint32_t* out, size_t n)
{
    for (size_t i = 0; i < n; ++i) {
        const uint32_t* k = keys + 2 * i;
        const uint32_t* c = ctrs + 4 * i;
        unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
        unsigned long long offset = 4ull * (((unsigned long long)c[1] << 32) | c[0]);
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        for (int w = 0; w < 4; ++w) out[4 * i + w] = eng.next();
    }
}
