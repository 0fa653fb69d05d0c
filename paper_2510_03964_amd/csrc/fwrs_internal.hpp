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

// Persistent batched kernel over a device table of frame descriptors.
// hdr[0] = number of frames, hdr[1] = total work items.
hipError_t launch_tick(const FrameDesc* descs, const uint32_t* hdr, uint32_t grid, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream);

hipError_t tick_occupancy(int* blocks_per_cu);

// Entry point of the persistent batched kernel, for HIP graph kernel nodes.
void* tick_kernel_entry();

}  // namespace fwrs
