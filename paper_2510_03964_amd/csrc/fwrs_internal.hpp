// Internal interface between the C ABI (fwrs_api.hip) and the kernels
// (fwrs_kernels.hip).  Not installed; callers use include/fwrs.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwrs_device.hpp"

namespace fwrs {

constexpr int kMaxK = 16;

// op: 1 = update only, 2 = resolve only, 3 = update + resolve,
// 5 = update + resolve of the changed pixels only.
hipError_t launch_frame(const FrameDesc& d, int op, hipStream_t stream);

// Arguments of one batched launch: n frames, `total` work items, frame f owns
// items [begins[f], begins[f + 1]).  Passed by value (< 4 KiB).
struct TickArgs {
    uint32_t n, total;
    uint32_t begins[kTickFrames];
    FrameDesc descs[kTickFrames];
};
static_assert(sizeof(TickArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// Batched kernel, one block per work item of the launch's frames.
hipError_t launch_tick(const TickArgs& a, hipStream_t stream);

// Reprojected frame: gather from the previous bank, dense write to this one.
hipError_t launch_reproject(const ReprojDesc& r, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream);

// Entry point of the batched kernel, for HIP graph kernel nodes.
void* tick_kernel_entry();

}  // namespace fwrs
