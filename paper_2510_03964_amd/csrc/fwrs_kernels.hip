// HIP kernels of the weighted-reservoir-sampling pass for gfx950.
//
// One thread owns a quad of 4 horizontally adjacent pixels, so that every
// structure-of-arrays plane is read and written with one 128-bit access per
// thread and the RGB (HWC) frame and output with three.  A block of 256
// threads covers one work item of 1024 pixels laid out as 1, 2 or 4 tiles of
// tile_x quads by tile_y rows (the tile shape changes the access pattern,
// never the results).  The pass is bound by HBM traffic, not arithmetic: there
// is no contraction anywhere, so no matrix cores.
//
// Per pixel and frame (Sec. 4.1-4.2 of the paper):
//   w    = Eq. 4 weight from the eccentricity to the gaze (level 0 -> 1)
//   W1'  = Eq. 6 biased w_sum (BERNOULLI) or w_sum (NONE)
//   slot j takes (colour, w, t) when u_j * (W1' + w) > W1'   (Alg. 2)
//   w_sum <- W1' + w;  m <- m + 1
//   out  = sum_j wt_j col_j / sum_j wt_j                      (resolve)
// The new colour is read only for quads in which some slot takes it, and a
// slot plane is written only where some pixel of the quad replaced that slot.
#include "fwrs_device.hpp"
#include "fwrs_internal.hpp"

namespace fwrs {

enum Op : int { kPush = 1, kResolve = 2, kFused = 3 };

// ---------------------------------------------------------------------------
// Decisions of one pixel: bit j set when slot j takes the new candidate.
// K > 0: compile-time slot count; K == 0: d.k at run time.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ uint32_t decide(const FrameDesc& d, uint32_t p, float W1b, float s)
{
    const int kk = K ? K : (int)d.k;
    uint32_t mask = 0u;
#pragma unroll
    for (int b = 0; b < (K ? (K + 3) / 4 : 4); ++b) {
        if (!K && 4 * b >= kk) break;
        const uint4 r = philox4x32_10(p, d.t, (uint32_t)b, 0u, d.seed, d.stream_id);
        const uint32_t words[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < kk) {
                const float u = unit_variate(words[q]);
                if (u * s > W1b) mask |= 1u << j;
            }
        }
    }
    return mask;
}

__device__ __forceinline__ float sel4(const float4& v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// ---------------------------------------------------------------------------
// A full quad with 16-byte aligned accesses: x0 % 4 == 0, x0 + 3 < width and
// width % 4 == 0, so p0 = y * width + x0 is a multiple of 4.
// ---------------------------------------------------------------------------
template <int K, int OP>
__device__ __forceinline__ uint32_t quad_vec(const FrameDesc& d, uint32_t x0, uint32_t y)
{
    const uint32_t p0 = y * d.width + x0;
    const size_t P = d.pitch;
    const int kk = K ? K : (int)d.k;
    uint32_t tk[4] = {0u, 0u, 0u, 0u};
    float w[4] = {0.f, 0.f, 0.f, 0.f};
    uint32_t ntakes = 0u;

    if (OP & kPush) {
        const uint32_t lv = *reinterpret_cast<const uint32_t*>(d.level + p0);
        const float4 W1 = *reinterpret_cast<const float4*>(d.wsum + p0);
        const uint4 m = *reinterpret_cast<const uint4*>(d.cnt + p0);
        const float dy = ((float)y + 0.5f) - d.gy;
        const float dy2 = dy * dy;
        const float W1v[4] = {W1.x, W1.y, W1.z, W1.w};
        float sv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float dx = ((float)(x0 + i) + 0.5f) - d.gx;
            w[i] = weight_eq4(d.c, dx * dx + dy2, (lv >> (8 * i)) & 0xFFu);
            const float W1b = bias_eq6(W1v[i], w[i], d.bias);
            sv[i] = W1b + w[i];
            tk[i] = decide<K>(d, p0 + i, W1b, sv[i]);
            ntakes += __popc(tk[i]);
        }
        *reinterpret_cast<float4*>(d.wsum + p0) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        *reinterpret_cast<uint4*>(d.cnt + p0) = make_uint4(m.x + 1u, m.y + 1u, m.z + 1u, m.w + 1u);
    }

    const uint32_t any = tk[0] | tk[1] | tk[2] | tk[3];
    float cin[12];
    if (any) {
        const float4* src = reinterpret_cast<const float4*>(d.color + 3 * (size_t)p0);
        const float4 a = src[0], b = src[1], c = src[2];
        cin[0] = a.x; cin[1] = a.y; cin[2] = a.z; cin[3] = a.w;
        cin[4] = b.x; cin[5] = b.y; cin[6] = b.z; cin[7] = b.w;
        cin[8] = c.x; cin[9] = c.y; cin[10] = c.z; cin[11] = c.w;
    }

    float4 S = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 acc[3] = {S, S, S};
#pragma unroll
    for (int j = 0; j < (K ? K : kMaxK); ++j) {
        if (!K && j >= kk) break;
        const uint32_t qm = ((tk[0] >> j) & 1u) | (((tk[1] >> j) & 1u) << 1) | (((tk[2] >> j) & 1u) << 2) |
                            (((tk[3] >> j) & 1u) << 3);
        float* wtp = d.wt + (size_t)j * P + p0;
        float* c0p = d.col + ((size_t)j * 3 + 0) * P + p0;
        float* c1p = d.col + ((size_t)j * 3 + 1) * P + p0;
        float* c2p = d.col + ((size_t)j * 3 + 2) * P + p0;
        float4 wj = make_float4(0.f, 0.f, 0.f, 0.f), cj0 = wj, cj1 = wj, cj2 = wj;
        const bool need_old = (OP & kResolve) || (qm != 0u && qm != 0xFu);
        if (need_old) {
            wj = *reinterpret_cast<const float4*>(wtp);
            cj0 = *reinterpret_cast<const float4*>(c0p);
            cj1 = *reinterpret_cast<const float4*>(c1p);
            cj2 = *reinterpret_cast<const float4*>(c2p);
        }
        if (qm) {
            float* wv = &wj.x;
            float* v0 = &cj0.x;
            float* v1 = &cj1.x;
            float* v2 = &cj2.x;
            uint32_t* ip = d.idx + (size_t)j * P + p0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (qm & (1u << i)) {
                    wv[i] = w[i];
                    v0[i] = cin[3 * i + 0];
                    v1[i] = cin[3 * i + 1];
                    v2[i] = cin[3 * i + 2];
                    ip[i] = d.t;
                }
            }
            *reinterpret_cast<float4*>(wtp) = wj;
            *reinterpret_cast<float4*>(c0p) = cj0;
            *reinterpret_cast<float4*>(c1p) = cj1;
            *reinterpret_cast<float4*>(c2p) = cj2;
        }
        if (OP & kResolve) {
            S.x = S.x + wj.x; S.y = S.y + wj.y; S.z = S.z + wj.z; S.w = S.w + wj.w;
            acc[0].x = acc[0].x + wj.x * cj0.x; acc[0].y = acc[0].y + wj.y * cj0.y;
            acc[0].z = acc[0].z + wj.z * cj0.z; acc[0].w = acc[0].w + wj.w * cj0.w;
            acc[1].x = acc[1].x + wj.x * cj1.x; acc[1].y = acc[1].y + wj.y * cj1.y;
            acc[1].z = acc[1].z + wj.z * cj1.z; acc[1].w = acc[1].w + wj.w * cj1.w;
            acc[2].x = acc[2].x + wj.x * cj2.x; acc[2].y = acc[2].y + wj.y * cj2.y;
            acc[2].z = acc[2].z + wj.z * cj2.z; acc[2].w = acc[2].w + wj.w * cj2.w;
        }
    }

    if (OP & kResolve) {
        float o[12];
        const float Sv[4] = {S.x, S.y, S.z, S.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // S == 0 only before the first frame (every kept weight is > 0): output 0.
            const float r = Sv[i] > 0.0f ? 1.0f / Sv[i] : 0.0f;
            o[3 * i + 0] = sel4(acc[0], i) * r;
            o[3 * i + 1] = sel4(acc[1], i) * r;
            o[3 * i + 2] = sel4(acc[2], i) * r;
        }
        float4* dst = reinterpret_cast<float4*>(d.out + 3 * (size_t)p0);
        dst[0] = make_float4(o[0], o[1], o[2], o[3]);
        dst[1] = make_float4(o[4], o[5], o[6], o[7]);
        dst[2] = make_float4(o[8], o[9], o[10], o[11]);
    }
    return ntakes;
}

// ---------------------------------------------------------------------------
// Any single pixel, scalar accesses (ragged widths, unaligned buffers, the
// right edge).  Same arithmetic as quad_vec.
// ---------------------------------------------------------------------------
template <int K, int OP>
__device__ __forceinline__ uint32_t pixel_scalar(const FrameDesc& d, uint32_t x, uint32_t y)
{
    const uint32_t p = y * d.width + x;
    const size_t P = d.pitch;
    const int kk = K ? K : (int)d.k;
    uint32_t tk = 0u;
    float w = 0.f;
    if (OP & kPush) {
        const uint32_t lv = d.level[p];
        const float W1 = d.wsum[p];
        const float dy = ((float)y + 0.5f) - d.gy;
        const float dx = ((float)x + 0.5f) - d.gx;
        w = weight_eq4(d.c, dx * dx + dy * dy, lv);
        const float W1b = bias_eq6(W1, w, d.bias);
        const float s = W1b + w;
        tk = decide<K>(d, p, W1b, s);
        d.wsum[p] = s;
        d.cnt[p] = d.cnt[p] + 1u;
    }
    float cin0 = 0.f, cin1 = 0.f, cin2 = 0.f;
    if (tk) {
        cin0 = d.color[3 * (size_t)p + 0];
        cin1 = d.color[3 * (size_t)p + 1];
        cin2 = d.color[3 * (size_t)p + 2];
    }
    float S = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int j = 0; j < (K ? K : kMaxK); ++j) {
        if (!K && j >= kk) break;
        const size_t o = (size_t)j * P + p;
        float wj, c0, c1, c2;
        if ((tk >> j) & 1u) {
            wj = w; c0 = cin0; c1 = cin1; c2 = cin2;
            d.wt[o] = wj;
            d.idx[o] = d.t;
            d.col[((size_t)j * 3 + 0) * P + p] = c0;
            d.col[((size_t)j * 3 + 1) * P + p] = c1;
            d.col[((size_t)j * 3 + 2) * P + p] = c2;
        } else if (OP & kResolve) {
            wj = d.wt[o];
            c0 = d.col[((size_t)j * 3 + 0) * P + p];
            c1 = d.col[((size_t)j * 3 + 1) * P + p];
            c2 = d.col[((size_t)j * 3 + 2) * P + p];
        } else {
            continue;
        }
        if (OP & kResolve) {
            S = S + wj;
            a0 = a0 + wj * c0;
            a1 = a1 + wj * c1;
            a2 = a2 + wj * c2;
        }
    }
    if (OP & kResolve) {
        const float r = S > 0.0f ? 1.0f / S : 0.0f;
        d.out[3 * (size_t)p + 0] = a0 * r;
        d.out[3 * (size_t)p + 1] = a1 * r;
        d.out[3 * (size_t)p + 2] = a2 * r;
    }
    return __popc(tk);
}

// ---------------------------------------------------------------------------
// One work item (1024 pixels) of a frame.  The wave index is made explicit
// as a uniform value so the tile arithmetic runs on the scalar unit.
// ---------------------------------------------------------------------------
template <int K, int OP>
__device__ __forceinline__ uint32_t process_item(const FrameDesc& d, uint32_t item)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t lane = tid & 63u;
    const uint32_t tlog = d.tile_x_log2 + d.tile_y_log2;            // log2(threads per tile): 6..8
    const uint32_t waves_per_tile_log2 = tlog - 6u;
    const uint32_t tiles_per_item_log2 = 8u - tlog;
    const uint32_t tile = (item << tiles_per_item_log2) + (wave >> waves_per_tile_log2);
    const uint32_t local = ((wave & ((1u << waves_per_tile_log2) - 1u)) << 6) | lane;
    const uint32_t ty = tile / d.tiles_x;
    const uint32_t tx = tile - ty * d.tiles_x;
    const uint32_t qx = local & ((1u << d.tile_x_log2) - 1u);
    const uint32_t ly = local >> d.tile_x_log2;
    const uint32_t x0 = ((tx << d.tile_x_log2) + qx) * kQuad;
    const uint32_t y = (ty << d.tile_y_log2) + ly;
    if (y >= d.height || x0 >= d.width) return 0u;
    if (d.vec_ok && x0 + 3u < d.width) return quad_vec<K, OP>(d, x0, y);
    uint32_t n = 0u;
    for (uint32_t x = x0; x < x0 + kQuad && x < d.width; ++x) n += pixel_scalar<K, OP>(d, x, y);
    return n;
}

__device__ __forceinline__ void add_stats(unsigned long long* stats, uint32_t v)
{
    // Wave sum, then one 64-bit atomic per wave on a counter chosen by the wave's id.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63u) == 0u && v) {
        const uint32_t slot = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) & (kStatSlots - 1);
        atomicAdd(stats + slot, (unsigned long long)v);
    }
}

template <int K, int OP>
__global__ __launch_bounds__(kBlock) void frame_kernel(FrameDesc d)
{
    const uint32_t n = process_item<K, OP>(d, blockIdx.x);
    if ((OP & kPush) && d.stats) add_stats(d.stats, n);
}

// ---------------------------------------------------------------------------
// Batched tick: a persistent grid walks the concatenated work items of all
// frames in the table (sorted by item_begin); each block keeps the index of
// the frame its current item belongs to, which only moves forward.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void tick_kernel(const FrameDesc* __restrict__ descs, const uint32_t* __restrict__ hdr)
{
    const uint32_t nframes = hdr[0];
    const uint32_t total = hdr[1];
    uint32_t f = 0u;
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        while (f + 1u < nframes && descs[f + 1u].item_begin <= item) ++f;
        const FrameDesc& d = descs[f];
        const uint32_t local = item - d.item_begin;
        uint32_t n;
        switch (d.k) {
            case 2: n = process_item<2, kFused>(d, local); break;
            case 4: n = process_item<4, kFused>(d, local); break;
            case 8: n = process_item<8, kFused>(d, local); break;
            default: n = process_item<0, kFused>(d, local); break;
        }
        if (d.stats) add_stats(d.stats, n);
    }
}

// ---------------------------------------------------------------------------
// Store initialisation: the empty reservoir.
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <int OP>
static hipError_t launch_frame_op(const FrameDesc& d, hipStream_t stream)
{
    const dim3 grid(d.items), block(kBlock);
    switch (d.k) {
        case 1: hipLaunchKernelGGL((frame_kernel<1, OP>), grid, block, 0, stream, d); break;
        case 2: hipLaunchKernelGGL((frame_kernel<2, OP>), grid, block, 0, stream, d); break;
        case 4: hipLaunchKernelGGL((frame_kernel<4, OP>), grid, block, 0, stream, d); break;
        case 8: hipLaunchKernelGGL((frame_kernel<8, OP>), grid, block, 0, stream, d); break;
        default: hipLaunchKernelGGL((frame_kernel<0, OP>), grid, block, 0, stream, d); break;
    }
    return hipGetLastError();
}

hipError_t launch_frame(const FrameDesc& d, int op, hipStream_t stream)
{
    if (d.items == 0u) return hipSuccess;
    switch (op) {
        case kPush: return launch_frame_op<kPush>(d, stream);
        case kResolve: return launch_frame_op<kResolve>(d, stream);
        default: return launch_frame_op<kFused>(d, stream);
    }
}

hipError_t launch_tick(const FrameDesc* descs, const uint32_t* hdr, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL(tick_kernel, dim3(grid), dim3(kBlock), 0, stream, descs, hdr);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, p, n, v);
    return hipGetLastError();
}

void* tick_kernel_entry() { return reinterpret_cast<void*>(&tick_kernel); }

hipError_t tick_occupancy(int* blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, tick_kernel, kBlock, 0);
}

}  // namespace fwrs
