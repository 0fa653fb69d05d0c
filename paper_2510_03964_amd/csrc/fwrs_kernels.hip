// HIP kernels of the weighted-reservoir-sampling pass for gfx950.
//
// Store layout (per context, N pixels, k slots): a w_sum plane w_sum[N],
// one record of k slots per pixel, rec[p * k + j] = {w, r, g, b} (16k bytes,
// so at k = 4 a pixel's record is exactly one 64-byte sector), the slots'
// frame indices idx[p * k + j], and the resolve plane res[N][3] (each pixel's
// resolve as of its last change).  A slot replacement therefore dirties only
// the sector of the pixel that replaced it, not one sector in each of k * 4
// planes; reads of whole records stay contiguous across a wave.  Alg. 2's
// candidate count m is the same for every pixel (each pixel receives exactly
// one candidate per frame), so it is the context's frame count, not a plane.
//
// One thread per pixel; a block of 256 threads covers one work item laid out
// as 1, 2 or 4 tiles of tile_x pixels by tile_y rows (the tile shape changes
// the access pattern, never the results).  A pixel's loads that do not depend
// on its decision (level, w_sum, the resolve plane or the record) are issued
// first and overlap the Philox rounds and the weight; the colour and, where
// needed, the record of a pixel that takes the candidate follow the decision.
// The pass is bound by HBM traffic; there is no contraction anywhere, so no
// matrix cores.
//
// Per pixel and frame (Sec. 4.1-4.2 of the paper):
//   w    = Eq. 4 weight from the eccentricity to the gaze (level 0 -> 1)
//   W1'  = Eq. 6 biased w_sum (BERNOULLI) or w_sum (NONE); under FULL every
//          slot has its own w_sum, biased by Eq. 7 against its own sample
//   slot j takes (colour, w, t) when u_j * (W1' + w) > W1'   (Alg. 2)
//   w_sum <- W1' + w
//   out  = sum_j wt_j col_j / sum_j wt_j                      (resolve)
// The new colour is read only by pixels in which some slot takes it; the
// output is written with non-temporal stores (it is not read again here).
#include "fwrs_device.hpp"
#include "fwrs_internal.hpp"

// Which streams use non-temporal loads / stores (bits, see kNt* below); a
// launch-shape tuning constant that never changes results.
#ifndef FWRS_NT_MASK
#define FWRS_NT_MASK 0x3C7u
#endif

namespace fwrs {

// kPush: update only; kResolve: resolve only; kFused: update + resolve of every
// pixel from its slots; kIncremental: update + resolve of the pixels whose record
// changed (the output already holds the previous frame's resolve everywhere
// else); kCached: update + resolve of every pixel, where a pixel without a
// replacement copies its resolve from the store's resolve plane (which holds it
// unchanged since the pixel last changed) and a changed pixel recomputes it and
// refreshes the plane; kFill: kFused that also writes every pixel's resolve into
// the plane, making it valid for the kCached frames that follow.
enum Op : int {
    kPush = kOpPush, kResolve = kOpResolve, kFused = kOpFused, kIncremental = kOpIncremental, kCached = kOpCached,
    kFill = kOpFill, kGroup = kOpGroup,
};

enum : uint32_t {
    kNtLevel = 1u, kNtWsumLd = 2u, kNtWsumSt = 4u, kNtRecLd = 8u, kNtRecSt = 16u, kNtIdxSt = 32u,
    kNtColor = 64u, kNtOut = 128u, kNtResLd = 256u, kNtResSt = 512u,
};
constexpr uint32_t kNt = FWRS_NT_MASK;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Every access of the pass goes through these helpers, which address global
// memory explicitly: a descriptor read from a table in device memory (the
// batched kernel) yields generic pointers, which would otherwise compile to
// flat instructions.
#define FWRS_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const FWRS_GLOBAL T* gbl(const T* p)
{
    return (const FWRS_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ FWRS_GLOBAL T* gbl(T* p)
{
    return (FWRS_GLOBAL T*)p;
}

template <uint32_t BIT, typename T>
__device__ __forceinline__ T ld(const T* p)
{
    if constexpr ((kNt & BIT) != 0u) return __builtin_nontemporal_load(gbl(p));
    return *gbl(p);
}

template <uint32_t BIT, typename T>
__device__ __forceinline__ void st(T* p, T v)
{
    if constexpr ((kNt & BIT) != 0u) __builtin_nontemporal_store(v, gbl(p));
    else *gbl(p) = v;
}

template <uint32_t BIT>
__device__ __forceinline__ float4 ld4(const float4* p)
{
    const v4f v = ld<BIT>(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

template <uint32_t BIT>
__device__ __forceinline__ float2 ld2(const float* p)
{
    const v2f v = ld<BIT>(reinterpret_cast<const v2f*>(p));
    return make_float2(v.x, v.y);
}

template <uint32_t BIT>
__device__ __forceinline__ void st4(float4* p, const float4& v)
{
    st<BIT>(reinterpret_cast<v4f*>(p), v4f{v.x, v.y, v.z, v.w});
}

// ---------------------------------------------------------------------------
// Variates and decisions of one pixel.  The Philox words depend only on the
// pixel index and the frame, so they are computed while the pixel's loads are
// in flight; the decision (bit j set when slot j takes the new candidate)
// needs the loaded w_sum.  K > 0: compile-time slot count; K == 0: d.k.
// ---------------------------------------------------------------------------
template <int K>
struct Words {
    uint32_t w[K ? 4 * ((K + 3) / 4) : 4];
};

template <int K>
__device__ __forceinline__ Words<K> philox_words(const FrameDesc& d, uint32_t p)
{
    static_assert(K > 0, "compile-time slot count");
    Words<K> out;
#pragma unroll
    for (int b = 0; b < (K + 3) / 4; ++b) {
        const uint4 r = philox4x32_10(p, d.t, (uint32_t)b, 0u, d.seed, d.stream_id);
        out.w[4 * b + 0] = r.x;
        out.w[4 * b + 1] = r.y;
        out.w[4 * b + 2] = r.z;
        out.w[4 * b + 3] = r.w;
    }
    return out;
}

template <int K>
__device__ __forceinline__ uint32_t decide_words(const Words<K>& words, float W1b, float s)
{
    uint32_t mask = 0u;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (unit_variate(words.w[j]) * s > W1b) mask |= 1u << j;
    return mask;
}

// Run-time slot count: blocks drawn as needed.
__device__ __forceinline__ uint32_t decide_any(const FrameDesc& d, uint32_t p, float W1b, float s)
{
    const int kk = (int)d.k;
    uint32_t mask = 0u;
    for (int b = 0; 4 * b < kk; ++b) {
        const uint4 r = philox4x32_10(p, d.t, (uint32_t)b, 0u, d.seed, d.stream_id);
        const uint32_t words[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < kk && unit_variate(words[q]) * s > W1b) mask |= 1u << j;
        }
    }
    return mask;
}

// Whether the resolve plane is read before the decision (with the pixel's other
// loads, so an unchanged pixel has it at hand) or only by unchanged pixels
// after it; a scheduling choice that never changes results.
#ifndef FWRS_RES_EARLY
#define FWRS_RES_EARLY 1
#endif

// The resolve of a record held in registers: sum_j w_j col_j / sum_j w_j, the
// sums taken in slot order; 0 for a record with no weight (only the empty
// reservoir: every kept weight is > 0).
template <int R>
__device__ __forceinline__ void resolve_slots(const float4 (&r)[R], float& q0, float& q1, float& q2)
{
    float S = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        S = S + r[j].x;
        a0 = a0 + r[j].x * r[j].y;
        a1 = a1 + r[j].x * r[j].z;
        a2 = a2 + r[j].x * r[j].w;
    }
    const float rs = S > 0.0f ? 1.0f / S : 0.0f;
    q0 = a0 * rs;
    q1 = a1 * rs;
    q2 = a2 * rs;
}

// ---------------------------------------------------------------------------
// One pixel.  K > 0 keeps the pixel's whole record in registers; K == 0
// (any slot count up to kMaxK) streams the record one slot at a time.
// Returns the number of slots replaced plus 2^16 if there was any.
// ---------------------------------------------------------------------------
template <int K, int OP, bool FOV = false>
__device__ __forceinline__ uint32_t pixel(const FrameDesc& d, uint32_t x, uint32_t y, const FovSrc* fs = nullptr)
{
    const uint32_t p = y * d.width + x;
    const int kk = K ? K : (int)d.k;
    constexpr int R = K ? K : 1;
    constexpr bool kUpdates = OP != kResolve;
    constexpr bool kResolves = OP != kPush;
    // every slot's record is read before the decision: the resolve needs them all
    constexpr bool kEager = OP == kFused || OP == kFill || OP == kResolve;
    // a recomputed resolve is also written to the resolve plane
    constexpr bool kKeepsRes = OP == kCached || OP == kFill;
    constexpr bool kResEarly = OP == kCached && FWRS_RES_EARLY;
    float4* rec = reinterpret_cast<float4*>(d.rec) + (size_t)p * (size_t)kk;
    uint32_t* idx = d.idx + (size_t)p * (size_t)kk;
    const float* color = d.color + 3 * (size_t)p;
    float* res = d.res + 3 * (size_t)p;
    // Frame 0 of a context meets the empty store (every slot zero): nothing to read.
    const bool empty = d.t == 0u;

    // 1. every load that does not depend on this frame's decisions (the compiler's
    //    own schedule interleaves them with step 2; forcing all of them ahead of
    //    the arithmetic measured slower)
    uint32_t lv = 0u;
    float W1 = 0.f;
    if (kUpdates) {
        if constexpr (FOV) lv = fov_level(*fs, d.gx, d.gy, x, y);
        else lv = ld<kNtLevel>(d.level + p);
        W1 = ld<kNtWsumLd>(d.wsum + p);
    }
    float4 r[R];
#pragma unroll
    for (int j = 0; j < R; ++j) r[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (K && kEager && !empty) {
#pragma unroll
        for (int j = 0; j < R; ++j) r[j] = ld4<kNtRecLd>(rec + j);
    }
    float q0 = 0.f, q1 = 0.f, q2 = 0.f;
    if (kResEarly) {
        q0 = ld<kNtResLd>(res + 0);
        q1 = ld<kNtResLd>(res + 1);
        q2 = ld<kNtResLd>(res + 2);
    }

    // 2. arithmetic that needs no loaded value: the Philox words and the weight's geometry
    Words<R> words;
    float outside = 0.f, e = 0.f;
    if (kUpdates) {
        if (K) words = philox_words<R>(d, p);
        const float dx = ((float)x + 0.5f) - d.gx;
        const float dy = ((float)y + 0.5f) - d.gy;
        outside = weight_outside(d.c, dx * dx + dy * dy, e);
    }

    // 3. weight (Eq. 4), bias (Eq. 6) and the Alg. 2 decision per slot
    uint32_t tk = 0u;
    float w = 0.f, s = 0.f;
    if (kUpdates) {
        w = select_eq4(d.c, outside, e, lv);
        const float W1b = bias_shared(W1, w, d.bias, d.c.decay);
        s = W1b + w;
        tk = K ? decide_words<R>(words, W1b, s) : decide_any(d, p, W1b, s);
    }

    // 4. the loads the decision calls for, all issued before any is waited for:
    //    the records of the slots that keep their sample (where only now needed)
    //    and the new colour, where some slot takes it; then the stores -- w_sum
    //    and the replaced slots -- which thus delay none of these loads
    if (K && (OP == kIncremental || OP == kCached) && tk && !empty) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (!((tk >> j) & 1u)) r[j] = ld4<kNtRecLd>(rec + j);
    }
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (tk) {
        if constexpr (FOV) {
            const float3 c = fov_colour(*fs, x, y, p, lv);
            c0 = c.x;
            c1 = c.y;
            c2 = c.z;
        } else {
            c0 = ld<kNtColor>(color + 0);
            c1 = ld<kNtColor>(color + 1);
            c2 = ld<kNtColor>(color + 2);
        }
    }
    if (kUpdates) st<kNtWsumSt>(d.wsum + p, s);
    const float4 fresh = make_float4(w, c0, c1, c2);
    if (K) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if ((tk >> j) & 1u) r[j] = fresh;
        if constexpr (K >= 8) {
            // Each lane's next replaced slot per store instruction: a wave issues
            // as many as its pixels' most replacements instead of one per slot,
            // nearly all lanes masked off (3% faster at k = 8, 6% slower at k = 4).
            for (uint32_t m = tk; m != 0u; m &= m - 1u) {
                const uint32_t j = (uint32_t)__builtin_ctz(m);
                st4<kNtRecSt>(rec + j, fresh);
                st<kNtIdxSt>(idx + j, d.t);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j)
                if ((tk >> j) & 1u) {
                    st4<kNtRecSt>(rec + j, fresh);
                    st<kNtIdxSt>(idx + j, d.t);
                }
        }
    }

    // 5. resolve: sum_j w_j col_j / sum_j w_j in slot order -- recomputed, or for a
    //    pixel without a replacement the unchanged value (kCached: from the
    //    resolve plane; kIncremental: the output already holds it)
    if (kResolves) {
        const bool recompute = (OP != kIncremental && OP != kCached) || tk != 0u;
        float* o = d.out + 3 * (size_t)p;
        if (recompute) {
            if (K) {
                resolve_slots<R>(r, q0, q1, q2);
            } else {
                float S = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
                for (int j = 0; j < kk; ++j) {
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    if ((tk >> j) & 1u) {
                        v = fresh;
                        st4<kNtRecSt>(rec + j, fresh);
                        st<kNtIdxSt>(idx + j, d.t);
                    } else if (!empty) {
                        v = ld4<kNtRecLd>(rec + j);
                    }
                    S = S + v.x;
                    a0 = a0 + v.x * v.y;
                    a1 = a1 + v.x * v.z;
                    a2 = a2 + v.x * v.w;
                }
                // S == 0 only before the first frame (every kept weight is > 0): output 0.
                const float rs = S > 0.0f ? 1.0f / S : 0.0f;
                q0 = a0 * rs;
                q1 = a1 * rs;
                q2 = a2 * rs;
            }
            if (kKeepsRes) {
                st<kNtResSt>(res + 0, q0);
                st<kNtResSt>(res + 1, q1);
                st<kNtResSt>(res + 2, q2);
            }
        } else if (OP == kCached && !kResEarly) {
            q0 = ld<kNtResLd>(res + 0);
            q1 = ld<kNtResLd>(res + 1);
            q2 = ld<kNtResLd>(res + 2);
        }
        if (recompute || OP == kCached) {
            st<kNtOut>(o + 0, q0);
            st<kNtOut>(o + 1, q1);
            st<kNtOut>(o + 2, q2);
        }
    } else if (!K) {
        for (int j = 0; j < kk; ++j)
            if ((tk >> j) & 1u) {
                st4<kNtRecSt>(rec + j, fresh);
                st<kNtIdxSt>(idx + j, d.t);
            }
    }
    return __popc(tk) + (tk ? 0x10000u : 0u);
}

// ---------------------------------------------------------------------------
// One pixel over a group of consecutive frames of one context (batched ticks;
// K > 0 slots, one w_sum per pixel): d0 is the group's first frame, later[f - 1]
// its frame f.  The pixel's state stays in registers from the group's first
// frame to its last -- w_sum, the pixel's resolve (read from the resolve plane
// where that holds it, else computed from the record, which is then read up
// front) and, from the first replacement on, the whole record -- so the store
// is read once and written once per group.  Each frame runs the single-frame
// arithmetic in the same order (the Philox words of its own frame index, the
// Eq. 4 weight at its own gaze, the bias, the Alg. 2 decision per slot, the
// resolve of a changed pixel in slot order) and writes its own output; at the
// end go w_sum, the replaced slots' records and frame indices, and the
// resolve plane (where the pixel changed, or everywhere if it did not hold the
// resolve), so the results are those of the frames run one by one, bit for bit.
//
// The frames are software-pipelined so that no frame waits for its own loads:
// a frame's level is read one frame ahead, and a frame is applied (slots
// replaced, resolve, output) one frame after its decision, once the next
// frame's loads are in flight.  The decision chain needs only w_sum and the
// level, so deciding frame f before applying frame f - 1 changes nothing.
// The colour load is issued by every pixel (those that take nothing read the
// frame's first texel, one line per wave), so no load sits in a branch and
// each wait covers exactly the loads it needs.
// Adds the replaced slots and the frames in which the pixel changed.
// ---------------------------------------------------------------------------
template <int K>
struct GroupPixel {
    float4 r[K];
    uint32_t tj[K];                             // the replaced slots' last frame index
    uint32_t dirty = 0u;                        // slots replaced in the group
    float q0 = 0.f, q1 = 0.f, q2 = 0.f;         // the resolve as of the last applied frame

    // Frame d's decision tk (weight w, colour c) becomes part of the record.
    __device__ __forceinline__ void apply(const FrameDesc& d, uint32_t p, uint32_t tk, float w, float c0, float c1,
                                          float c2, uint32_t& slots, uint32_t& changed)
    {
        if (tk) {
            const float4 fresh = make_float4(w, c0, c1, c2);
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((tk >> j) & 1u) {
                    r[j] = fresh;
                    tj[j] = d.t;
                }
            dirty |= tk;
            resolve_slots<K>(r, q0, q1, q2);
            slots += (uint32_t)__popc(tk);
            changed += 1u;
        }
        float* o = d.out + 3 * (size_t)p;
        st<kNtOut>(o + 0, q0);
        st<kNtOut>(o + 1, q1);
        st<kNtOut>(o + 2, q2);
    }
};

template <int K>
__device__ __forceinline__ void pixel_group(const FrameDesc& d0, const FrameDesc* __restrict__ later, uint32_t x,
                                            uint32_t y, uint32_t& slots, uint32_t& changed)
{
    const uint32_t p = y * d0.width + x;
    const uint32_t nf = d0.nf;
    float4* rec = reinterpret_cast<float4*>(d0.rec) + (size_t)p * K;
    uint32_t* idx = d0.idx + (size_t)p * K;
    float* res = d0.res + 3 * (size_t)p;
    const bool keep = d0.res != nullptr;
    const bool empty = d0.t == 0u;              // the empty store: every slot zero, nothing to read
    const bool from_plane = keep && d0.res_ok != 0u && !empty;

    GroupPixel<K> g;
    float W1 = ld<kNtWsumLd>(d0.wsum + p);
    uint32_t lv = ld<kNtLevel>(d0.level + p);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        g.r[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        g.tj[j] = 0u;
    }
    bool have = true;                           // the record is in registers (or on its way)
    if (from_plane) {
        g.q0 = ld<kNtResLd>(res + 0);
        g.q1 = ld<kNtResLd>(res + 1);
        g.q2 = ld<kNtResLd>(res + 2);
        have = false;
    } else if (!empty) {
#pragma unroll
        for (int j = 0; j < K; ++j) g.r[j] = ld4<kNtRecLd>(rec + j);
        resolve_slots<K>(g.r, g.q0, g.q1, g.q2);
    }

    // the decided frame still to apply
    uint32_t ptk = 0u;
    float pw = 0.f, pc0 = 0.f, pc1 = 0.f, pc2 = 0.f;
    for (uint32_t f = 0; f < nf; ++f) {
        const FrameDesc& d = f == 0u ? d0 : later[f - 1u];
        uint32_t lv_next = 0u;
        if (f + 1u < nf) lv_next = ld<kNtLevel>(later[f].level + p);
        // the decision: Eq. 4 weight, bias, Alg. 2 per slot
        const float dx = ((float)x + 0.5f) - d.gx;
        const float dy = ((float)y + 0.5f) - d.gy;
        float e = 0.f;
        const float outside = weight_outside(d.c, dx * dx + dy * dy, e);
        const float w = select_eq4(d.c, outside, e, lv);
        const float W1b = bias_shared(W1, w, d.bias, d.c.decay);
        const float s = W1b + w;
        const uint32_t tk = decide_words<K>(philox_words<K>(d, p), W1b, s);
        W1 = s;
        // its colour, and at the pixel's first replacement the slots it keeps
        const float* cp = d.color + (tk ? 3 * (size_t)p : 0);
        const float c0 = ld<kNtColor>(cp + 0), c1 = ld<kNtColor>(cp + 1), c2 = ld<kNtColor>(cp + 2);
        // the previous frame
        if (f) g.apply(f == 1u ? d0 : later[f - 2u], p, ptk, pw, pc0, pc1, pc2, slots, changed);
        if (tk && !have) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (!((tk >> j) & 1u)) g.r[j] = ld4<kNtRecLd>(rec + j);
            have = true;
        }
        ptk = tk;
        pw = w;
        pc0 = c0;
        pc1 = c1;
        pc2 = c2;
        lv = lv_next;
    }
    g.apply(nf == 1u ? d0 : later[nf - 2u], p, ptk, pw, pc0, pc1, pc2, slots, changed);

    st<kNtWsumSt>(d0.wsum + p, W1);
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((g.dirty >> j) & 1u) {
            st4<kNtRecSt>(rec + j, g.r[j]);
            st<kNtIdxSt>(idx + j, g.tj[j]);
        }
    if (keep && (g.dirty != 0u || !from_plane)) {
        st<kNtResSt>(res + 0, g.q0);
        st<kNtResSt>(res + 1, g.q1);
        st<kNtResSt>(res + 2, g.q2);
    }
}

// ---------------------------------------------------------------------------
// One pixel under a per-slot mode, one value per slot in wslot[p * k + j]:
//  - Eq. 7 (FULL): the slot's own w_sum, biased by the slot's colour
//    difference to the new pixel before its Alg. 2 decision;
//  - A-ES: the log2 key of the slot's sample; the candidate's key log2(u) / w
//    replaces it when larger (Sec. 3.1).
// Needs the new colour for every pixel and every slot's record, so the records
// are read by every op that updates.  Same store layout otherwise.
// ---------------------------------------------------------------------------
template <int K, int OP, bool FOV = false>
__device__ __forceinline__ uint32_t pixel_per_slot(const FrameDesc& d, uint32_t x, uint32_t y,
                                                   const FovSrc* fs = nullptr)
{
    const uint32_t p = y * d.width + x;
    const int kk = K ? K : (int)d.k;
    constexpr int R = K ? K : 1;
    constexpr bool kUpdates = OP == kPush || OP == kFused || OP == kIncremental;
    constexpr bool kResolves = OP == kFused || OP == kIncremental;
    float4* rec = reinterpret_cast<float4*>(d.rec) + (size_t)p * (size_t)kk;
    uint32_t* idx = d.idx + (size_t)p * (size_t)kk;
    float* wslot = d.wsum + (size_t)p * (size_t)kk;

    // every slot's record and sum up front (K > 0), then the pixel's own inputs
    float4 r[R];
    float W[R];
    if (K) {
#pragma unroll
        for (int j = 0; j < R; ++j) r[j] = ld4<kNtRecLd>(rec + j);
        if (K % 4 == 0) {
#pragma unroll
            for (int j = 0; j < R; j += 4) {
                const float4 v = ld4<kNtWsumLd>(reinterpret_cast<const float4*>(wslot + j));
                W[j] = v.x;
                W[(j + 1) % R] = v.y;
                W[(j + 2) % R] = v.z;
                W[(j + 3) % R] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) W[j] = ld<kNtWsumLd>(wslot + j);
        }
    }
    uint32_t lv;
    float c0, c1, c2;
    if constexpr (FOV) {
        lv = fov_level(*fs, d.gx, d.gy, x, y);
        const float3 c = fov_colour(*fs, x, y, p, lv);
        c0 = c.x;
        c1 = c.y;
        c2 = c.z;
    } else {
        lv = ld<kNtLevel>(d.level + p);
        const float* color = d.color + 3 * (size_t)p;
        c0 = ld<kNtColor>(color + 0);
        c1 = ld<kNtColor>(color + 1);
        c2 = ld<kNtColor>(color + 2);
    }
    const float dx = ((float)x + 0.5f) - d.gx;
    const float dy = ((float)y + 0.5f) - d.gy;
    const float w = weight_eq4(d.c, dx * dx + dy * dy, lv);
    const bool aes = d.bias == kAes;
    // Eq. 7: a slot whose sample has the new pixel's colour has |dL| = 0 exactly
    // (same_colour), so its Lab and CIE94 are not evaluated, nor the new
    // pixel's Lab when that holds for every slot.
    const bool bounded = lab_bounded(c0, c1, c2);
    uint32_t same = 0u;
    if (K && !aes) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (bounded && same_colour(r[j], c0, c1, c2)) same |= 1u << j;
    }
    float3 lab_new = make_float3(0.f, 0.f, 0.f);
    if (!aes && (!K || same != (1u << R) - 1u)) lab_new = rgb_to_lab(c0, c1, c2);
    const float4 fresh = make_float4(w, c0, c1, c2);

    float S = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
    uint32_t tk = 0u;
    uint4 words = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int j = 0; j < kk; ++j) {
        float4 v = K ? r[K ? j : 0] : ld4<kNtRecLd>(rec + j);
        const float W1 = K ? W[K ? j : 0] : ld<kNtWsumLd>(wslot + j);
        if ((j & 3) == 0) words = philox4x32_10(p, d.t, (uint32_t)(j >> 2), 0u, d.seed, d.stream_id);
        const uint32_t word = (j & 3) == 0 ? words.x : (j & 3) == 1 ? words.y : (j & 3) == 2 ? words.z : words.w;
        bool take;
        float s;
        if (aes) {
            // A-ES: the larger key log2(u) / w wins; the slot keeps its sample's key
            const float kn = log2_unit(word) / w;
            take = kn > W1;
            s = take ? kn : W1;
        } else {
            // Eq. 7 against this slot's sample, then the slot's Alg. 2 decision
            const bool same_j = K ? ((same >> j) & 1u) != 0u : bounded && same_colour(v, c0, c1, c2);
            float dl = 0.0f;
            if (!same_j) dl = delta_l(v.y, v.z, v.w, lab_new);
            const float W1b = bias_eq7(W1, w, dl);
            s = W1b + w;
            take = unit_variate(word) * s > W1b;
        }
        if (take) {
            tk |= 1u << j;
            v = fresh;
            st4<kNtRecSt>(rec + j, fresh);
            st<kNtIdxSt>(idx + j, d.t);
        }
        if (K) W[K ? j : 0] = s;
        else st<kNtWsumSt>(wslot + j, s);
        S = S + v.x;
        a0 = a0 + v.x * v.y;
        a1 = a1 + v.x * v.z;
        a2 = a2 + v.x * v.w;
    }
    if (K) {
        if (K % 4 == 0) {
#pragma unroll
            for (int j = 0; j < R; j += 4)
                st4<kNtWsumSt>(reinterpret_cast<float4*>(wslot + j),
                               make_float4(W[j], W[(j + 1) % R], W[(j + 2) % R], W[(j + 3) % R]));
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) st<kNtWsumSt>(wslot + j, W[j]);
        }
    }
    if (kResolves && (OP != kIncremental || tk)) {
        const float rs = S > 0.0f ? 1.0f / S : 0.0f;
        float* o = d.out + 3 * (size_t)p;
        st<kNtOut>(o + 0, a0 * rs);
        st<kNtOut>(o + 1, a1 * rs);
        st<kNtOut>(o + 2, a2 * rs);
    }
    static_assert(kUpdates, "the resolve-only pass is the same under every bias mode");
    return __popc(tk) + (tk ? 0x10000u : 0u);
}

// ---------------------------------------------------------------------------
// One work item (256 pixels).  The wave index is made explicit as a uniform
// value so the tile arithmetic runs on the scalar unit.
// ---------------------------------------------------------------------------
// Pixel of this thread in work item `item`; false outside the image (or past
// the frame's last item).  The wave index is made explicit as a uniform value
// so the tile arithmetic runs on the scalar unit.
__device__ __forceinline__ bool item_pixel_of(const FrameDesc& d, uint32_t item, uint32_t wave, uint32_t lane,
                                              uint32_t& x, uint32_t& y)
{
    const uint32_t tlog = d.tile_x_log2 + d.tile_y_log2;            // log2(threads per tile): 6..8
    const uint32_t waves_per_tile_log2 = tlog - 6u;
    const uint32_t tiles_per_item_log2 = 8u - tlog;
    const uint32_t tile = (item << tiles_per_item_log2) + (wave >> waves_per_tile_log2);
    const uint32_t local = ((wave & ((1u << waves_per_tile_log2) - 1u)) << 6) | lane;
    const uint32_t ty = tile / d.tiles_x;
    const uint32_t tx = tile - ty * d.tiles_x;
    x = (tx << d.tile_x_log2) + (local & ((1u << d.tile_x_log2) - 1u));
    y = (ty << d.tile_y_log2) + (local >> d.tile_x_log2);
    return item < d.items && y < d.height && x < d.width;
}

__device__ __forceinline__ bool item_pixel(const FrameDesc& d, uint32_t item, uint32_t& x, uint32_t& y)
{
    const uint32_t tid = threadIdx.x;
    return item_pixel_of(d, item, __builtin_amdgcn_readfirstlane(tid >> 6), tid & 63u, x, y);
}

// One work item (256 pixels, one per thread).
template <int K, int OP, bool PER_SLOT = false, bool FOV = false>
__device__ __forceinline__ uint32_t process_item(const FrameDesc& d, uint32_t item, const FovSrc* fs = nullptr)
{
    uint32_t x, y;
    if (!item_pixel(d, item, x, y)) return 0u;
    if constexpr (PER_SLOT) return pixel_per_slot<K, OP, FOV>(d, x, y, fs);
    return pixel<K, OP, FOV>(d, x, y, fs);
}

// add_stats for counts beyond its packed fields' range (a group of frames):
// replaced slots and changed pixel-frames as separate wave sums.
__device__ __forceinline__ void add_stats_wide(unsigned long long* stats, uint32_t slots, uint32_t changed)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        slots += __shfl_xor(slots, off);
        changed += __shfl_xor(changed, off);
    }
    if ((threadIdx.x & 63u) == 0u && changed) {
        const uint32_t slot = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) & (kStatSlots - 1);
        atomicAdd(stats + 3 * slot, (unsigned long long)slots);
        atomicAdd(stats + 3 * slot + 1, (unsigned long long)changed);
    }
}

__device__ __forceinline__ void add_stats(unsigned long long* stats, uint32_t v)
{
    // v = replaced slots + 2^16 * (pixel changed) + 2^24 * (pixel flushed).  Wave sum (at
    // most 1024 slots and 64 pixels per field), then one 64-bit atomic per non-zero counter
    // and wave on a triple chosen by the wave's id.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63u) == 0u && v) {
        const uint32_t slot = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) & (kStatSlots - 1);
        atomicAdd(stats + 3 * slot, (unsigned long long)(v & 0xFFFFu));
        atomicAdd(stats + 3 * slot + 1, (unsigned long long)((v >> 16) & 0xFFu));
        if (v >> 24) atomicAdd(stats + 3 * slot + 2, (unsigned long long)(v >> 24));
    }
}

// Work items are visited in reverse order on odd frames, so each frame starts
// where the previous one ended: the store it touched last is still in the
// 256 MB Infinity Cache (a third of a 4K, k = 4 store) when it is read again.
// The order never changes a result.
__device__ __forceinline__ uint32_t frame_item(uint32_t block, uint32_t items, uint32_t t)
{
    return (t & 1u) ? items - 1u - block : block;
}

template <int K, int OP, bool PER_SLOT = false>
__global__ __launch_bounds__(kBlock) void frame_kernel(FrameDesc d)
{
    const uint32_t n = process_item<K, OP, PER_SLOT>(d, frame_item(blockIdx.x, d.items, d.t));
    if (OP != kResolve && d.stats) add_stats(d.stats, n);
}

// ---------------------------------------------------------------------------
// Batched tick: one launch for all the frames of a tick, any number of them.
// The frames' descriptors are a table in device memory or in the kernel's
// arguments (uniform data, read with scalar loads).  The consecutive frames of
// one context in a tick form a group, whose first frame (the leader) stands for
// it among the table's leaders, in the order the tick visits them; the tick's
// 256-pixel work items are numbered leader after leader, and a leader whose
// `rev` is set visits its own items last first (the host reverses the group
// order and sets `rev` on every other tick, so such a tick runs entirely
// backwards).  The grid has one block per work item (blocks past the last item
// exit): this measured faster than a persistent grid of resident blocks looping
// over the items -- the hardware's block dispatch balances the uneven per-item
// cost of the pass better than a fixed stride -- and without a loop over items
// the kernel keeps fewer values live (one more wave per SIMD).  A block finds
// its item's leader by binary search over the leaders' first items.  An item of
// a lone frame runs the single-frame per-pixel code for the frame's slot count
// and op (kFused, kCached or kFill); an item of a group runs pixel_group (op
// kGroup), or else (run-time slot counts, per-slot modes) each of the group's
// frames in turn through the store, every pixel in the same thread, so each
// frame reads what the one before wrote.
// ---------------------------------------------------------------------------
template <int K, int OP, bool PER_SLOT = false>
__device__ __forceinline__ uint32_t process_wave(const FrameDesc& d, uint32_t item, uint32_t wave)
{
    uint32_t x, y;
    if (!item_pixel_of(d, item, wave, threadIdx.x & 63u, x, y)) return 0u;
    if constexpr (PER_SLOT) return pixel_per_slot<K, OP>(d, x, y);
    return pixel<K, OP>(d, x, y);
}

__device__ __forceinline__ uint32_t tick_item(const FrameDesc& d, uint32_t local, uint32_t wave)
{
    if (per_slot_mode(d.bias)) return process_wave<0, kFused, true>(d, local, wave);
#define FWRS_TICK_OPS(KK)                                                                  \
    return d.op == kCached ? process_wave<KK, kCached>(d, local, wave)                     \
         : d.op == kFill ? process_wave<KK, kFill>(d, local, wave) : process_wave<KK, kFused>(d, local, wave)
    switch (d.k) {
        case 1: FWRS_TICK_OPS(1);
        case 2: FWRS_TICK_OPS(2);
        case 4: FWRS_TICK_OPS(4);
        case 8: FWRS_TICK_OPS(8);
        default: FWRS_TICK_OPS(0);
    }
#undef FWRS_TICK_OPS
}

// One work item of a group of d.nf > 1 frames (d its leader); G as tick_kernel's.
template <int G>
__device__ __forceinline__ void tick_group_item(const FrameDesc& d, const FrameDesc* __restrict__ descs,
                                                uint32_t local, uint32_t wave)
{
    const FrameDesc* later = descs + d.more;
    if (d.op == kGroup) {
        uint32_t x, y, slots = 0u, changed = 0u;
        if (item_pixel_of(d, local, wave, threadIdx.x & 63u, x, y)) {
            switch (d.k) {
                case 1: pixel_group<1>(d, later, x, y, slots, changed); break;
                case 2: pixel_group<2>(d, later, x, y, slots, changed); break;
                case 4: pixel_group<4>(d, later, x, y, slots, changed); break;
                default:                                 // the host sets kGroup only for k in {1, 2, 4, 8}
                    if constexpr (G == kTickGroups8) pixel_group<8>(d, later, x, y, slots, changed);
                    break;
            }
        }
        if (d.stats) add_stats_wide(d.stats, slots, changed);
        return;
    }
    for (uint32_t f = 0; f < d.nf; ++f) {
        const FrameDesc& df = f == 0u ? d : later[f - 1u];
        const uint32_t v = tick_item(df, local, wave);
        if (df.stats) add_stats(df.stats, v);
    }
}

// The tick of table (head, descs), block by block; G: what the tick holds
// (kTickAlone: no groups; kTickGroups: groups, none run as kGroup with k = 8;
// kTickGroups8: some are).  A group holds its pixels' whole records across
// its frames, which takes more registers than the single-frame paths (at k = 8
// far more), so each kind of tick runs the instantiation with only the paths
// it needs, at the best occupancy they allow.
template <int G>
__device__ __forceinline__ void tick_blocks(const TickHead& head, const FrameDesc* __restrict__ descs)
{
    const uint32_t item = blockIdx.x;
    if (item >= head.total) return;
    uint32_t f = 0u, hi = head.n - 1u;               // last leader whose first item <= item
    while (f < hi) {
        const uint32_t mid = (f + hi + 1u) >> 1;
        if (descs[mid].first <= item) f = mid;
        else hi = mid - 1u;
    }
    const FrameDesc& d = descs[f];
    uint32_t local = item - d.first;
    if (d.rev) local = d.items - 1u - local;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (G != kTickAlone && d.nf > 1u) {
        tick_group_item<G>(d, descs, local, wave);
    } else {
        const uint32_t v = tick_item(d, local, wave);
        if (d.stats) add_stats(d.stats, v);
    }
}

// The table in device memory.
template <int G>
__global__ __launch_bounds__(kBlock) void tick_kernel(const TickHead* __restrict__ head,
                                                      const FrameDesc* __restrict__ descs)
{
    tick_blocks<G>(*head, descs);
}

// The table carried in the kernel's arguments (a tick of at most kArgFrames
// frames), read in place from the kernel-argument segment: indexing the
// by-value parameter itself would copy it to private memory first.
template <int G>
__global__ __launch_bounds__(kBlock) void tick_args_kernel(const TickArgs a)
{
    (void)a;
    const TickArgs* in = (const TickArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    tick_blocks<G>(in->head, in->descs);
}

// Writes descriptors carried as kernel arguments into a tick table.
__global__ __launch_bounds__(64) void tick_fill_kernel(uint32_t* __restrict__ table, const TickFill f)
{
    constexpr uint32_t kDescWords = sizeof(FrameDesc) / 4;
    static_assert(sizeof(FrameDesc) % 4 == 0, "descriptors are copied as words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(f.descs);
    uint32_t* dst = table + kTickDescOffset / 4 + (size_t)f.at * kDescWords;
    for (uint32_t i = threadIdx.x; i < f.count * kDescWords; i += blockDim.x) st<0u>(dst + i, src[i]);
    if (f.write_head && threadIdx.x < 4u) st<0u>(table + threadIdx.x, reinterpret_cast<const uint32_t*>(&f.head)[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Store initialisation: the empty reservoir.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Reprojected frame (Sec. 4.3).  Pixel p continues the reservoir of the pixel
// containing its centre moved back by its motion vector, if that point is in
// the image and its previous depth agrees with p's depth within the relative
// tolerance; otherwise p starts from the empty reservoir (flush).  Then the
// frame's update as in the other kernels (Eq. 4, the bias, Alg. 2 per slot),
// written densely to this frame's bank, and the resolve.  A gather from the
// previous bank, so the banks alternate; every slot is rewritten.
// ---------------------------------------------------------------------------
template <int K, bool PER_SLOT>
__device__ __forceinline__ uint32_t pixel_reproject(const ReprojDesc& r, uint32_t x, uint32_t y)
{
    const FrameDesc& d = r.f;
    const uint32_t p = y * d.width + x;
    const int kk = K ? K : (int)d.k;
    constexpr int R = K ? K : 1;

    // 1. the motion-compensated source and the depth test
    const float2 mv = ld2<kNtColor>(r.motion + 2 * (size_t)p);
    const float dc = ld<kNtColor>(r.depth + p);
    const float sx = ((float)x + 0.5f) - mv.x;
    const float sy = ((float)y + 0.5f) - mv.y;
    bool keep = false;
    uint32_t q = 0u;
    if (sx >= 0.0f && sx < (float)d.width && sy >= 0.0f && sy < (float)d.height) {
        const uint32_t qx = (uint32_t)floorf(sx);
        const uint32_t qy = (uint32_t)floorf(sy);
        q = qy * d.width + qx;
        const float dp = r.src_depth[q];
        keep = fabsf(dc - dp) <= r.tol * dc;      // NaN (no previous frame) compares false
    }

    // 2. the history: the source reservoir, or the empty one
    const float4* src = reinterpret_cast<const float4*>(r.src_rec) + (size_t)q * (size_t)kk;
    const uint32_t* sidx = r.src_idx + (size_t)q * (size_t)kk;
    float4 rv[R];
    uint32_t iv[R];
    float W[R];
    const float4 empty = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool aes = d.bias == kAes;
    const float empty_slot = aes ? -INFINITY : 0.f;      // A-ES key / Eq. 7 sum of an empty slot
    // loads are unconditional (q = 0 is a valid pixel when the history is dropped) and the
    // empty values are selected afterwards, so every load is a plain global load
    if (K) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float4 v = src[j];
            const uint32_t i = sidx[j];
            rv[j] = keep ? v : empty;
            iv[j] = keep ? i : 0xFFFFFFFFu;
            if (PER_SLOT) {
                const float ws = r.src_wsum[(size_t)q * (size_t)kk + j];
                W[j] = keep ? ws : empty_slot;
            }
        }
    }
    float W1 = 0.f;
    uint32_t m = 0u;
    {
        const float ws = PER_SLOT ? 0.f : r.src_wsum[q];
        const uint32_t mc = r.src_cnt[q];
        W1 = keep ? ws : 0.f;
        m = keep ? mc : 0u;
    }

    // 3. this frame's candidate
    const uint32_t lv = ld<kNtLevel>(d.level + p);
    const float* color = d.color + 3 * (size_t)p;
    const float c0 = ld<kNtColor>(color + 0);
    const float c1 = ld<kNtColor>(color + 1);
    const float c2 = ld<kNtColor>(color + 2);
    const float dx = ((float)x + 0.5f) - d.gx;
    const float dy = ((float)y + 0.5f) - d.gy;
    const float w = weight_eq4(d.c, dx * dx + dy * dy, lv);
    const float4 fresh = make_float4(w, c0, c1, c2);
    // Eq. 7: a slot whose sample has the new pixel's colour has |dL| = 0 exactly
    // (same_colour); neither Lab is evaluated for it
    const bool bounded = lab_bounded(c0, c1, c2);
    uint32_t same = 0u;
    if (K && PER_SLOT && !aes) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (bounded && same_colour(rv[j], c0, c1, c2)) same |= 1u << j;
    }
    float3 lab_new = make_float3(0.f, 0.f, 0.f);
    if (PER_SLOT && !aes && (!K || same != (1u << R) - 1u)) lab_new = rgb_to_lab(c0, c1, c2);
    const float W1b = PER_SLOT ? 0.f : bias_shared(W1, w, d.bias, d.c.decay);
    const float s = W1b + w;

    // 4. Alg. 2 per slot, dense stores to this frame's bank, resolve sums
    float4* rec = reinterpret_cast<float4*>(d.rec) + (size_t)p * (size_t)kk;
    uint32_t* idx = d.idx + (size_t)p * (size_t)kk;
    float S = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f;
    uint32_t tk = 0u;
    uint4 words = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int j = 0; j < kk; ++j) {
        float4 v;
        uint32_t vi;
        float Wj = 0.f;
        if (K) {
            v = rv[K ? j : 0];
            vi = iv[K ? j : 0];
            if (PER_SLOT) Wj = W[K ? j : 0];
        } else {
            const float4 sv = src[j];
            const uint32_t si = sidx[j];
            v = keep ? sv : empty;
            vi = keep ? si : 0xFFFFFFFFu;
            if (PER_SLOT) {
                const float ws = r.src_wsum[(size_t)q * (size_t)kk + j];
                Wj = keep ? ws : empty_slot;
            }
        }
        if ((j & 3) == 0) words = philox4x32_10(p, d.t, (uint32_t)(j >> 2), 0u, d.seed, d.stream_id);
        const uint32_t word = (j & 3) == 0 ? words.x : (j & 3) == 1 ? words.y : (j & 3) == 2 ? words.z : words.w;
        float W1j = W1b, sj = s;
        bool take;
        if (PER_SLOT && aes) {
            const float kn = log2_unit(word) / w;
            take = kn > Wj;
            st<kNtWsumSt>(d.wsum + (size_t)p * (size_t)kk + j, take ? kn : Wj);
        } else {
            if (PER_SLOT) {
                const bool same_j = K ? ((same >> j) & 1u) != 0u : bounded && same_colour(v, c0, c1, c2);
                float dl = 0.0f;
                if (!same_j) dl = delta_l(v.y, v.z, v.w, lab_new);
                W1j = bias_eq7(Wj, w, dl);
                sj = W1j + w;
                st<kNtWsumSt>(d.wsum + (size_t)p * (size_t)kk + j, sj);
            }
            take = unit_variate(word) * sj > W1j;
        }
        if (take) {
            tk |= 1u << j;
            v = fresh;
            vi = d.t;
        }
        st4<kNtRecSt>(rec + j, v);
        st<kNtIdxSt>(idx + j, vi);
        S = S + v.x;
        a0 = a0 + v.x * v.y;
        a1 = a1 + v.x * v.z;
        a2 = a2 + v.x * v.w;
    }
    if (!PER_SLOT) st<kNtWsumSt>(d.wsum + p, s);
    st<kNtWsumSt>(r.cnt + p, m + 1u);
    st<kNtWsumSt>(r.depth_out + p, dc);
    if (d.out) {
        const float rs = S > 0.0f ? 1.0f / S : 0.0f;
        float* o = d.out + 3 * (size_t)p;
        st<kNtOut>(o + 0, a0 * rs);
        st<kNtOut>(o + 1, a1 * rs);
        st<kNtOut>(o + 2, a2 * rs);
    }
    return __popc(tk) + (tk ? 0x10000u : 0u) + (keep ? 0u : 0x1000000u);
}

template <int K, bool PER_SLOT>
__global__ __launch_bounds__(kBlock) void reproject_kernel(ReprojDesc r)
{
    const FrameDesc& d = r.f;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t lane = tid & 63u;
    const uint32_t tlog = d.tile_x_log2 + d.tile_y_log2;
    const uint32_t waves_per_tile_log2 = tlog - 6u;
    const uint32_t tiles_per_item_log2 = 8u - tlog;
    // forward order every frame: this dense pass (221 B per pixel) gains nothing
    // from the Infinity Cache and streams slightly slower backwards
    const uint32_t tile = (blockIdx.x << tiles_per_item_log2) + (wave >> waves_per_tile_log2);
    const uint32_t local = ((wave & ((1u << waves_per_tile_log2) - 1u)) << 6) | lane;
    const uint32_t ty = tile / d.tiles_x;
    const uint32_t tx = tile - ty * d.tiles_x;
    const uint32_t x = (tx << d.tile_x_log2) + (local & ((1u << d.tile_x_log2) - 1u));
    const uint32_t y = (ty << d.tile_y_log2) + (local >> d.tile_x_log2);
    uint32_t n = 0u;
    if (y < d.height && x < d.width) n = pixel_reproject<K, PER_SLOT>(r, x, y);
    if (d.stats) add_stats(d.stats, n);
}

// ---------------------------------------------------------------------------
// Foveation generator (Sec. 4.3).  mip_kernel: one lane per mip-1 texel, the
// mip-2 texels from their mip-1 children by wave shuffles; each texel the mean
// of the children that exist, summed in row-major order.
// gauss_levels_kernel: the separable Gaussian levels, clamp to edge,
// accumulation in offset order.  foveate_kernel: the degraded frame and level map on their own;
// foveated_kernel: the same sampling fused into the reservoir pass.
// ---------------------------------------------------------------------------
struct MipArgs {
    const float* full;
    float* m1;
    float* m2;
    uint32_t w, h, w1, h1, w2, h2;
};

// 1 / n for the child counts a texel can have (1, 2 or 4): a power of two, so
// s * (1 / n) is exactly the correctly rounded s / n.
__device__ __forceinline__ float inv_count(uint32_t n)
{
    return n == 4u ? 0.25f : (n == 2u ? 0.5f : 1.0f);
}

// Mean of the children (2i + dx, 2j + dy) of a texel; every load is issued
// before the sums (children outside the source read the texel's first child
// and are not added).
__device__ __forceinline__ float3 texel_mean(const float* src, uint32_t sw, uint32_t sh, uint32_t i, uint32_t j)
{
    float3 v[4];
    bool in[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t x = 2 * i + (q & 1u), y = 2 * j + (q >> 1);
        in[q] = x < sw && y < sh;
        const float* c = src + ((size_t)(in[q] ? y : 2 * j) * sw + (in[q] ? x : 2 * i)) * 3;
        v[q] = make_float3(c[0], c[1], c[2]);
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    uint32_t n = 0u;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        if (in[q]) {
            s0 = s0 + v[q].x;
            s1 = s1 + v[q].y;
            s2 = s2 + v[q].z;
            n = n + 1u;
        }
    const float r = inv_count(n);
    return make_float3(s0 * r, s1 * r, s2 * r);
}

__global__ __launch_bounds__(kBlock) void mip_kernel(MipArgs a)
{
    // One lane per mip-1 texel: a wave covers 32 mip-1 columns of the two
    // mip-1 rows under one mip-2 row (lanes 0-31 the upper row, 32-63 the
    // lower); lane pairs (2m, 2m + 1) of each half are the children of one
    // mip-2 texel, gathered by wave shuffles in row-major order.
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6, lane = threadIdx.x & 63u;
    const uint32_t strips = (a.w1 + 31u) / 32u;
    if (wave >= strips * a.h2) return;                 // whole waves only
    const uint32_t i1 = (wave % strips) * 32u + (lane & 31u), j2 = wave / strips;
    const uint32_t j1 = 2u * j2 + (lane >> 5);
    const bool own = i1 < a.w1 && j1 < a.h1;
    const float3 m = texel_mean(a.full, a.w, a.h, own ? i1 : 0u, own ? j1 : 0u);
    if (own) {
        float* o = a.m1 + ((size_t)j1 * a.w1 + i1) * 3;
        o[0] = m.x;
        o[1] = m.y;
        o[2] = m.z;
    }
    // children of mip-2 texel (i1 / 2, j2) for the even lanes of the upper row
    const int src[3] = {(int)(lane ^ 1u), (int)(lane + 32u) & 63, (int)((lane ^ 1u) + 32u) & 63};
    float v[4][3] = {{m.x, m.y, m.z}};
    bool in[4] = {own};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        v[q + 1][0] = __shfl(m.x, src[q]);
        v[q + 1][1] = __shfl(m.y, src[q]);
        v[q + 1][2] = __shfl(m.z, src[q]);
        in[q + 1] = __shfl((int)own, src[q]) != 0;
    }
    if ((lane & 33u) == 0u && own) {                   // even lane of the upper row, texel exists
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
        uint32_t n = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (in[q]) {
                s0 = s0 + v[q][0];
                s1 = s1 + v[q][1];
                s2 = s2 + v[q][2];
                n = n + 1u;
            }
        const float r = inv_count(n);
        float* o = a.m2 + ((size_t)j2 * a.w2 + i1 / 2u) * 3;
        o[0] = s0 * r;
        o[1] = s1 * r;
        o[2] = s2 * r;
    }
}

// Gaussian levels from one read of the frame, into one plane: every pixel of
// level l >= 1 gets the frame blurred with sigma 2^(l-1) (radius kGaussR1 or
// kGaussR2) at that pixel; level-0 pixels are not written.  A block owns COLS
// columns (one per thread) and a strip of ROWS output rows.  It walks the
// strip's rows and a halo of kGaussR2 rows above and below (row indices clamped
// to the image): each row segment, columns x0 - kGaussR2 .. x0 + COLS - 1 +
// kGaussR2 (clamped), is staged in LDS as three channel planes; every thread
// takes the horizontal sums of the radii the block needs at its column and
// keeps the last rows' sums in registers; an output row's vertical sum is taken
// once its last tap row is in.  The loads of the next rows are in flight while
// the current row is summed.  Sums start at zero and add the taps in offset order,
// the order of two separate passes (horizontal, then vertical).  Which levels
// a block needs comes from its rectangle's distances to the gaze, widened by
// 2^-10 relative so that rounding can only make it need more.
struct GaussArgs {
    const float* src;
    float* dst;
    uint32_t w, h, cols;                               // cols: blocks per strip
    float gx, gy, r0sq, r1sq;
    float g1[2 * kGaussR1 + 1];
    float g2[2 * kGaussR2 + 1];
};

template <int ROWS, int COLS>
__global__ __launch_bounds__(COLS) void gauss_levels_kernel(GaussArgs a)
{
    constexpr int R1 = kGaussR1, R2 = kGaussR2;
    constexpr int PF = 2;                              // rows in flight
    constexpr int SEG = COLS + 2 * R2;                 // pixels of a staged row segment
    constexpr int NF = 3 * SEG;                        // floats of it
    constexpr int PER = (NF + COLS - 1) / COLS;        // floats staged per thread
    constexpr int NV = ROWS + 2 * R2;                  // rows walked (halo included)
    static_assert(R1 <= R2, "the sigma-1 taps are a subset of the sigma-2 taps");
    static_assert(NV % PF == 0 && PF % 2 == 0, "whole, even prefetch groups");
    __shared__ float seg[2][3 * SEG];

    const int tid = (int)threadIdx.x;
    const int W = (int)a.w, H = (int)a.h;
    const uint32_t bx = blockIdx.x % a.cols, by = blockIdx.x / a.cols;   // one-dimensional grid, row-major
    const int x0 = (int)bx * COLS, y0 = (int)by * ROWS;
    const int x = x0 + tid;

    // Levels present in the block's pixels (block-uniform, conservative).
    bool need1, need2;
    {
        const float xa = (float)x0 + 0.5f, xb = (float)min(x0 + COLS, W) - 0.5f;
        const float ya = (float)y0 + 0.5f, yb = (float)min(y0 + ROWS, H) - 0.5f;
        const float nx = fminf(fmaxf(a.gx, xa), xb) - a.gx, ny = fminf(fmaxf(a.gy, ya), yb) - a.gy;
        const float fx = fmaxf(fabsf(xa - a.gx), fabsf(xb - a.gx)), fy = fmaxf(fabsf(ya - a.gy), fabsf(yb - a.gy));
        const float dmin = nx * nx + ny * ny, dmax = fx * fx + fy * fy;
        need1 = dmin * (1.0f - 0x1p-10f) <= a.r1sq && dmax * (1.0f + 0x1p-10f) > a.r0sq;
        need2 = dmax * (1.0f + 0x1p-10f) > a.r1sq;
    }
    if (!need1 && !need2) return;                      // every pixel at level 0

    // This thread stages floats f = tid + q COLS of a segment: channel f % 3
    // of segment pixel f / 3 (image column x0 - R2 + f / 3, clamped).
    int goff[PER], loff[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int f = tid + q * COLS;
        const int e = f / 3, ch = f - 3 * e;
        const int xx = min(max(x0 - R2 + e, 0), W - 1);
        goff[q] = xx * 3 + ch;
        loff[q] = f < NF ? ch * SEG + e : -1;
    }
    // Walked row v is loaded into stage[v % PF] PF rows ahead: rows v + 1 ..
    // v + PF are in flight while row v is summed (the loop is unrolled by PF,
    // so every index is a constant and the ring stays in registers).
    float stage[PF][PER];
    auto fetch = [&](int v, float* dst) {
        const int yy = min(max(y0 - R2 + v, 0), H - 1);
        const float* row = a.src + (size_t)yy * (size_t)W * 3;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (loff[q] >= 0) dst[q] = row[goff[q]];
    };

    float3 h2[2 * R2 + 1];     // sigma-2 horizontal sums of walked rows v - 2 R2 .. v (oldest first)
    float3 h1[2 * R1 + 1];     // sigma-1 horizontal sums of walked rows v - 2 R1 .. v
#pragma unroll
    for (int u = 0; u < PF; ++u) fetch(u, stage[u]);
    for (int vb = 0; vb < NV; vb += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int v = vb + u;
        float* s = seg[u & 1];                         // PF is even: u & 1 == v & 1
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (loff[q] >= 0) s[loff[q]] = stage[u][q];
        __syncthreads();
        if (v + PF < NV) fetch(v + PF, stage[u]);

        const float* c = s + tid;                      // c[ch SEG + i]: channel ch, column x - R2 + i
        if (need2) {
#pragma unroll
            for (int i = 0; i < 2 * R2; ++i) h2[i] = h2[i + 1];
            float t[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i <= 2 * R2; ++i) acc = acc + a.g2[i] * c[ch * SEG + i];
                t[ch] = acc;
            }
            h2[2 * R2] = make_float3(t[0], t[1], t[2]);
        }
        if (need1) {
#pragma unroll
            for (int i = 0; i < 2 * R1; ++i) h1[i] = h1[i + 1];
            float t[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i <= 2 * R1; ++i) acc = acc + a.g1[i] * c[ch * SEG + R2 - R1 + i];
                t[ch] = acc;
            }
            h1[2 * R1] = make_float3(t[0], t[1], t[2]);
        }

        // Walked row j is image row y0 - R2 + j (clamped); its radius-r sums
        // are complete once walked row j + r is in, i.e. at v = j + r.
        const int y1 = y0 + v - R1 - R2;
        if (need1 && v >= R1 + R2 && v < R1 + R2 + ROWS && y1 < H && x < W &&
            ring_level(a.r0sq, a.r1sq, a.gx, a.gy, (uint32_t)x, (uint32_t)y1) == 1u) {
            float3 o = make_float3(0.f, 0.f, 0.f);
#pragma unroll
            for (int i = 0; i <= 2 * R1; ++i) {
                const float g = a.g1[i];
                o.x = o.x + g * h1[i].x;
                o.y = o.y + g * h1[i].y;
                o.z = o.z + g * h1[i].z;
            }
            float* d = a.dst + ((size_t)y1 * (size_t)W + (size_t)x) * 3;
            d[0] = o.x;
            d[1] = o.y;
            d[2] = o.z;
        }
        const int y2 = y0 + v - 2 * R2;
        if (need2 && v >= 2 * R2 && y2 < H && x < W &&
            ring_level(a.r0sq, a.r1sq, a.gx, a.gy, (uint32_t)x, (uint32_t)y2) == 2u) {
            float3 o = make_float3(0.f, 0.f, 0.f);
#pragma unroll
            for (int i = 0; i <= 2 * R2; ++i) {
                const float g = a.g2[i];
                o.x = o.x + g * h2[i].x;
                o.y = o.y + g * h2[i].y;
                o.z = o.z + g * h2[i].z;
            }
            float* d = a.dst + ((size_t)y2 * (size_t)W + (size_t)x) * 3;
            d[0] = o.x;
            d[1] = o.y;
            d[2] = o.z;
        }
      }
    }
}

struct FoveateArgs {
    FovSrc s;
    float* color;
    uint8_t* level;
    uint32_t w, h;
    float gx, gy;
};

__global__ __launch_bounds__(kBlock) void foveate_kernel(FoveateArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.w * a.h) return;
    const uint32_t x = p % a.w, y = p / a.w;
    const uint32_t lv = fov_level(a.s, a.gx, a.gy, x, y);
    const float3 c = fov_colour(a.s, x, y, p, lv);
    float* o = a.color + (size_t)p * 3;
    o[0] = c.x;
    o[1] = c.y;
    o[2] = c.z;
    a.level[p] = (uint8_t)lv;
}

template <int K, bool PER_SLOT, int OP>
__global__ __launch_bounds__(kBlock) void foveated_kernel(FovDesc fd)
{
    const uint32_t n = process_item<K, OP, PER_SLOT, true>(fd.f, frame_item(blockIdx.x, fd.f.items, fd.f.t), &fd.s);
    if (fd.f.stats) add_stats(fd.f.stats, n);
}

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
    // the per-slot modes keep no resolve plane: they run kPush, kFused or kIncremental
    if constexpr (OP == kPush || OP == kFused || OP == kIncremental) {
        if (per_slot_mode(d.bias)) {
            switch (d.k) {
                case 4: hipLaunchKernelGGL((frame_kernel<4, OP, true>), grid, block, 0, stream, d); break;
                case 8: hipLaunchKernelGGL((frame_kernel<8, OP, true>), grid, block, 0, stream, d); break;
                default: hipLaunchKernelGGL((frame_kernel<0, OP, true>), grid, block, 0, stream, d); break;
            }
            return hipGetLastError();
        }
    }
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
        case kIncremental: return launch_frame_op<kIncremental>(d, stream);
        case kCached: return launch_frame_op<kCached>(d, stream);
        case kFill: return launch_frame_op<kFill>(d, stream);
        default: return launch_frame_op<kFused>(d, stream);
    }
}

hipError_t launch_tick(const void* table, uint32_t grid, int kind, hipStream_t stream)
{
    if (grid == 0u) return hipSuccess;
    const TickHead* head = static_cast<const TickHead*>(table);
    const FrameDesc* descs = reinterpret_cast<const FrameDesc*>(static_cast<const char*>(table) + kTickDescOffset);
    if (kind == kTickGroups8)
        hipLaunchKernelGGL(tick_kernel<kTickGroups8>, dim3(grid), dim3(kBlock), 0, stream, head, descs);
    else if (kind == kTickGroups)
        hipLaunchKernelGGL(tick_kernel<kTickGroups>, dim3(grid), dim3(kBlock), 0, stream, head, descs);
    else
        hipLaunchKernelGGL(tick_kernel<kTickAlone>, dim3(grid), dim3(kBlock), 0, stream, head, descs);
    return hipGetLastError();
}

hipError_t launch_tick_fill(void* table, const TickFill& f, hipStream_t stream)
{
    hipLaunchKernelGGL(tick_fill_kernel, dim3(1), dim3(64), 0, stream, static_cast<uint32_t*>(table), f);
    return hipGetLastError();
}

hipError_t launch_reproject(const ReprojDesc& r, hipStream_t stream)
{
    const dim3 grid(r.f.items), block(kBlock);
    const bool eq7 = per_slot_mode(r.f.bias);
    switch (r.f.k) {
        case 4:
            if (eq7) hipLaunchKernelGGL((reproject_kernel<4, true>), grid, block, 0, stream, r);
            else hipLaunchKernelGGL((reproject_kernel<4, false>), grid, block, 0, stream, r);
            break;
        case 8:
            if (eq7) hipLaunchKernelGGL((reproject_kernel<8, true>), grid, block, 0, stream, r);
            else hipLaunchKernelGGL((reproject_kernel<8, false>), grid, block, 0, stream, r);
            break;
        default:
            if (eq7) hipLaunchKernelGGL((reproject_kernel<0, true>), grid, block, 0, stream, r);
            else hipLaunchKernelGGL((reproject_kernel<0, false>), grid, block, 0, stream, r);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_mips(const float* full, float* m1, float* m2, uint32_t w, uint32_t h, hipStream_t stream)
{
    MipArgs a{full, m1, m2, w, h, (w + 1) / 2, (h + 1) / 2, 0u, 0u};
    a.w2 = (a.w1 + 1) / 2;
    a.h2 = (a.h1 + 1) / 2;
    const uint64_t threads = (uint64_t)((a.w1 + 31u) / 32u) * a.h2 * 64u;   // whole waves
    hipLaunchKernelGGL(mip_kernel, dim3((uint32_t)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_gauss_levels(const float* full, float* dst, uint32_t w, uint32_t h, float gx, float gy, float r0sq,
                               float r1sq, const float* g1, const float* g2, hipStream_t stream)
{
    GaussArgs a{};
    a.src = full;
    a.dst = dst;
    a.w = w;
    a.h = h;
    a.gx = gx;
    a.gy = gy;
    a.r0sq = r0sq;
    a.r1sq = r1sq;
    for (int i = 0; i <= 2 * kGaussR1; ++i) a.g1[i] = g1[i];
    for (int i = 0; i <= 2 * kGaussR2; ++i) a.g2[i] = g2[i];
    // One-wave blocks; the tallest strip (32, 16, 8 or 4 rows; the halo costs
    // 12 walked rows per strip) whose grid still gives the compute units about
    // 16 waves each, else 4 rows: with fewer waves the per-row barrier and load
    // latency are not hidden.
    constexpr int C = kGaussCols;
    a.cols = (w + C - 1) / C;
    auto blocks = [&](uint32_t rows) { return (uint64_t)a.cols * ((h + rows - 1) / rows); };
    const dim3 block(C);
    if (blocks(32) >= 4000u)
        hipLaunchKernelGGL((gauss_levels_kernel<32, C>), dim3((uint32_t)blocks(32)), block, 0, stream, a);
    else if (blocks(16) >= 4000u)
        hipLaunchKernelGGL((gauss_levels_kernel<16, C>), dim3((uint32_t)blocks(16)), block, 0, stream, a);
    else if (blocks(8) >= 4000u)
        hipLaunchKernelGGL((gauss_levels_kernel<8, C>), dim3((uint32_t)blocks(8)), block, 0, stream, a);
    else
        hipLaunchKernelGGL((gauss_levels_kernel<4, C>), dim3((uint32_t)blocks(4)), block, 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_foveate(const FovSrc& s, float* color, uint8_t* level, uint32_t w, uint32_t h, float gx, float gy,
                          hipStream_t stream)
{
    FoveateArgs a{s, color, level, w, h, gx, gy};
    const uint32_t n = w * h;
    hipLaunchKernelGGL(foveate_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_foveated(const FovDesc& fd, int op, hipStream_t stream)
{
    if (fd.f.items == 0u) return hipSuccess;
    const dim3 grid(fd.f.items), block(kBlock);
    const bool ps = per_slot_mode(fd.f.bias);
#define FWRS_FOV_LAUNCH(KK, PS, OPV) hipLaunchKernelGGL((foveated_kernel<KK, PS, OPV>), grid, block, 0, stream, fd)
#define FWRS_FOV_OPS(KK)                                      \
    do {                                                      \
        if (op == kCached) FWRS_FOV_LAUNCH(KK, false, kCached);   \
        else if (op == kFill) FWRS_FOV_LAUNCH(KK, false, kFill);  \
        else if (op == kPush) FWRS_FOV_LAUNCH(KK, false, kPush);  \
        else FWRS_FOV_LAUNCH(KK, false, kFused);              \
    } while (0)
    if (ps) {
        const bool push = op == kPush;
        if (fd.f.k == 4) {
            if (push) FWRS_FOV_LAUNCH(4, true, kPush);
            else FWRS_FOV_LAUNCH(4, true, kFused);
        } else {
            if (push) FWRS_FOV_LAUNCH(0, true, kPush);
            else FWRS_FOV_LAUNCH(0, true, kFused);
        }
    } else {
        switch (fd.f.k) {
            case 4: FWRS_FOV_OPS(4); break;
            case 8: FWRS_FOV_OPS(8); break;
            default: FWRS_FOV_OPS(0); break;
        }
    }
#undef FWRS_FOV_OPS
#undef FWRS_FOV_LAUNCH
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

hipError_t launch_tick_args(const TickArgs& a, int kind, hipStream_t stream)
{
    const uint32_t grid = a.head.total;
    if (grid == 0u) return hipSuccess;
    if (kind == kTickGroups8)
        hipLaunchKernelGGL(tick_args_kernel<kTickGroups8>, dim3(grid), dim3(kBlock), 0, stream, a);
    else if (kind == kTickGroups)
        hipLaunchKernelGGL(tick_args_kernel<kTickGroups>, dim3(grid), dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL(tick_args_kernel<kTickAlone>, dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

void* tick_kernel_entry(int kind)
{
    if (kind == kTickGroups8) return reinterpret_cast<void*>(&tick_kernel<kTickGroups8>);
    if (kind == kTickGroups) return reinterpret_cast<void*>(&tick_kernel<kTickGroups>);
    return reinterpret_cast<void*>(&tick_kernel<kTickAlone>);
}


}  // namespace fwrs
