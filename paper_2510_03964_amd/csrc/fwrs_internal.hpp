// Internal interface between the C ABI (fwrs_api.hip) and the kernels
// (fwrs_kernels.hip).  Not installed; callers use include/fwrs.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwrs_device.hpp"

namespace fwrs {

constexpr int kMaxK = 16;
constexpr int kMaxBlurRadius = 32;
constexpr int kGaussR1 = 3;             // ceil(3 sigma) of the Gaussian levels, sigma = 1 and 2
constexpr int kGaussR2 = 6;
constexpr int kGaussCols = 64;          // columns (threads) per block of the Gaussian level kernel

// The kernels' ops (the launchers take them as int).
constexpr int kOpPush = 1;          // update only
constexpr int kOpResolve = 2;       // resolve only
constexpr int kOpFused = 3;         // update + resolve of every pixel from its slots
constexpr int kOpIncremental = 5;   // update + resolve of the changed pixels only
constexpr int kOpCached = 7;        // update + resolve, unchanged pixels from the resolve plane
constexpr int kOpFill = 9;          // kOpFused that also writes the resolve plane
constexpr int kOpGroup = 11;        // batched ticks: a group's frames with the pixel state held in registers
hipError_t launch_frame(const FrameDesc& d, int op, hipStream_t stream);

// A batched tick's table in device memory: this head, then (at kTickDescOffset)
// the n group leaders' descriptors in the order their work items are numbered
// (descs[f].first increasing, descs[f].items > 0), then the groups' later
// frames (descs[leader.more .. leader.more + leader.nf - 2] for each leader);
// `total` = the tick's work items.
struct alignas(16) TickHead {
    uint32_t n, total, pad0, pad1;
};
constexpr size_t kTickDescOffset = 16;
static_assert(sizeof(TickHead) == kTickDescOffset, "descriptors follow the head");
inline size_t tick_table_bytes(size_t frames) { return kTickDescOffset + frames * sizeof(FrameDesc); }

// The batched kernel on `grid` blocks, one per work item of the table's tick
// (grid = head.total; blocks past the last item do nothing), in the
// instantiation for the kind of tick the table holds: no groups (no leader
// with nf > 1), groups, or groups among which one with op kOpGroup and k = 8.
constexpr int kTickAlone = 0;
constexpr int kTickGroups = 1;
constexpr int kTickGroups8 = 2;
constexpr int kTickKinds = 3;
hipError_t launch_tick(const void* table, uint32_t grid, int kind, hipStream_t stream);
// Its entry points, for HIP graph kernel nodes: arguments (const TickHead*, const FrameDesc*).
void* tick_kernel_entry(int kind);

// A tick of at most kArgFrames frames carries its whole table in the kernel's
// arguments: one launch, no copy.
constexpr int kArgFrames = 21;
struct TickArgs {
    TickHead head;
    FrameDesc descs[kArgFrames];
};
static_assert(sizeof(TickArgs) <= 4096, "kernel arguments are limited to 4 KiB");
hipError_t launch_tick_args(const TickArgs& a, int kind, hipStream_t stream);

// One launch of the table-fill kernel: writes `count` descriptors (kernel
// arguments) to table slots at .. at + count - 1, and the head if write_head.
constexpr int kFillFrames = 20;
struct TickFill {
    TickHead head;
    uint32_t at, count, write_head, pad;
    FrameDesc descs[kFillFrames];
};
static_assert(sizeof(TickFill) <= 4096, "kernel arguments are limited to 4 KiB");
hipError_t launch_tick_fill(void* table, const TickFill& f, hipStream_t stream);

// Reprojected frame: gather from the previous bank, dense write to this one.
hipError_t launch_reproject(const ReprojDesc& r, hipStream_t stream);

// Foveation generator: mip 1 and 2 of a frame; the Gaussian plane of a frame
// for a gaze (each pixel blurred at its own level's radius; weights
// g1[2 kGaussR1 + 1], g2[2 kGaussR2 + 1]); the degraded frame + level map; the
// reservoir pass fed by the generator (no intermediate frame).
hipError_t launch_mips(const float* full, float* m1, float* m2, uint32_t w, uint32_t h, hipStream_t stream);
hipError_t launch_gauss_levels(const float* full, float* dst, uint32_t w, uint32_t h, float gx, float gy, float r0sq,
                               float r1sq, const float* g1, const float* g2, hipStream_t stream);
hipError_t launch_foveate(const FovSrc& s, float* color, uint8_t* level, uint32_t w, uint32_t h, float gx, float gy,
                          hipStream_t stream);
hipError_t launch_foveated(const FovDesc& fd, int op, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream);


}  // namespace fwrs
