// C ABI of the weighted-reservoir-sampling library (include/fwrs.h):
// contexts with their reservoir store in HBM (per-pixel slot records, frame
// indices, w_sum and the resolve plane), argument validation, single-frame
// launches on a borrowed stream, state access, and the batched tick engine.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fwrs.h"
#include "fwrs_device.hpp"
#include "fwrs_internal.hpp"

using fwrs::FrameDesc;

namespace {

constexpr size_t kPitchAlign = 64;   // elements; planes start on 256-byte boundaries
constexpr size_t kStatBytes = 3 * sizeof(unsigned long long) * fwrs::kStatSlots;
constexpr int kDefaultTileX = 64, kDefaultTileY = 1;

// Frames of a context before its fused passes use the resolve plane.  While a
// store fills (the first frames after a reset), most pixels replace a slot every
// frame, so copying unchanged resolves from the plane saves little and keeping
// the plane costs a write per changed pixel; the frame before this one writes the
// plane densely (kOpFill) and later frames use it (kOpCached).  A launch-policy
// constant: it never changes results.
#ifndef FWRS_RES_FROM
#define FWRS_RES_FROM 32
#endif
constexpr uint32_t kResFrom = FWRS_RES_FROM;

size_t pitch_for(int width, int height)
{
    const size_t n = (size_t)width * (size_t)height;
    return (n + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
}

bool sizes_ok(int width, int height, int k)
{
    if (width <= 0 || height <= 0 || k < 1 || k > FWRS_MAX_K) return false;
    // pixel indices are 32-bit in the kernels and in the Philox counter
    return (long long)width * (long long)height < (1ll << 31);
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

bool params_ok(const fwrs_params* p)
{
    if (!p) return false;
    if (!finite_pos(p->fov_deg) || !finite_pos(p->fovea_radius_px)) return false;
    if (p->bias_mode > FWRS_AES) return false;
    if (!std::isfinite(p->lambda_decay) || p->lambda_decay < 0.0f) return false;
    if (!(p->a_k > 0.0f && p->a_k <= 1.0f)) return false;
    if ((p->flags & ~(uint32_t)(FWRS_FLAG_REPROJECT | FWRS_FLAG_NO_RESOLVE_PLANE)) != 0u) return false;
    return finite_pos(p->r_m) && finite_pos(p->r2k) && finite_pos(p->rek);
}

// Whether a context keeps the resolve plane: every mode with one w_sum per
// pixel, unless the caller opted out; not the per-slot modes (Eq. 7 reads every
// slot's colour each frame anyway) nor reprojecting contexts (dense passes).
bool keeps_res(uint32_t bias_mode, uint32_t flags)
{
    return !fwrs::per_slot_mode(bias_mode) && (flags & (FWRS_FLAG_REPROJECT | FWRS_FLAG_NO_RESOLVE_PLANE)) == 0u;
}

// Elements (4 bytes) of one bank of the store: w_sum (one per pixel, or one per
// slot under Eq. 7), the slot records, the slot frame indices, the resolve
// plane (3 per pixel) where kept, and for a reprojecting context the pixel
// counts and depths.
size_t bank_elems(size_t pitch, size_t k, uint32_t bias_mode, uint32_t flags)
{
    const size_t ws = fwrs::per_slot_mode(bias_mode) ? k : 1;
    const size_t extra = (flags & FWRS_FLAG_REPROJECT) ? 2 : (keeps_res(bias_mode, flags) ? 3 : 0);
    return pitch * (ws + 5 * k + extra);
}

// Per-context constants, derived with the same binary32 functions the kernels use.
fwrs::Consts derive(const fwrs_params& p, int width)
{
    fwrs::Consts c{};
    c.A = p.a_k;
    c.B = 1.0f - p.a_k;
    c.IR2 = 1.0f / p.r2k;
    c.IRM = 1.0f / p.r_m;
    c.C = 1.44269504088896341f / p.rek;
    const float ppd = (float)width / p.fov_deg;
    c.iPPD = 1.0f / ppd;
    c.rf = p.fovea_radius_px * c.iPPD;
    float num, den;
    fwrs::density_terms(c, c.rf, num, den);
    c.Drf = num / den;
    c.decay = fwrs::exp2_neg(-(p.lambda_decay * 1.44269504088896341f));   // exp(-lambda)
    return c;
}

int log2_exact(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return (1 << l) == v ? l : -1;
}

bool tile_ok(int tx, int ty)
{
    const int lx = log2_exact(tx), ly = log2_exact(ty);
    if (lx < 0 || ly < 0) return false;
    return lx + ly >= 6 && lx + ly <= 8;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

// Makes `waiter` wait for the work enqueued so far on `signaller` (nothing when
// they are one stream).  `ev` is created on first use; its owner destroys it.
hipError_t order_after(hipStream_t waiter, hipStream_t signaller, hipEvent_t& ev)
{
    if (waiter == signaller) return hipSuccess;
    if (!ev) {
        const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            ev = nullptr;
            return e;
        }
    }
    hipError_t e = hipEventRecord(ev, signaller);
    if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
    return e;
}

}  // namespace

struct fwrs_ctx {
    int width = 0, height = 0, k = 0, device = 0;
    fwrs_params prm{};
    fwrs::Consts c{};
    hipStream_t stream = nullptr;
    void* arena = nullptr;
    bool owns_arena = false;
    size_t pitch = 0;
    size_t wsum_slots = 1;   // 1: one w_sum per pixel; k under Eq. 7 (one per slot)
    // the current bank (the store the next frame reads)
    float* wsum = nullptr;
    float* rec = nullptr;
    uint32_t* idx = nullptr;
    // reprojecting contexts: two banks; bank[b] = {wsum, rec, idx, cnt, depth}
    bool reproject = false;
    int cur = 0;
    float* bank_wsum[2] = {nullptr, nullptr};
    float* bank_rec[2] = {nullptr, nullptr};
    uint32_t* bank_idx[2] = {nullptr, nullptr};
    uint32_t* bank_cnt[2] = {nullptr, nullptr};
    float* bank_depth[2] = {nullptr, nullptr};
    // the resolve plane (null if not kept) and whether it holds every pixel's
    // current resolve
    float* res = nullptr;
    bool res_valid = false;
    uint32_t res_from = kResFrom;    // first frame index whose fused pass may use the plane
    unsigned long long* stats = nullptr;
    uint32_t t = 0;
    uint64_t pixel_updates = 0;
    // `resolved_out` holds this context's resolve as of frame `resolved_at`
    // (valid only while `resolved` is set): the precondition of the
    // incremental entry point.
    const float* resolved_out = nullptr;
    uint32_t resolved_at = 0;
    bool resolved = false;
    int tile_x = kDefaultTileX, tile_y = kDefaultTileY;
    hipEvent_t order_ev = nullptr;   // marks this context's stream for work on other streams
    // batched ticks: the layout pass that last met this context, and its group there
    uint64_t tick_mark = 0;
    int tick_group = 0;
};

namespace {

int clear_store(fwrs_ctx* x)
{
    const size_t P = x->pitch, k = (size_t)x->k;
    // wsum and the slot records are contiguous and start out zero (A-ES keys:
    // -infinity); idx starts empty.
    const bool aes = x->prm.bias_mode == FWRS_AES;
    if (fwrs::launch_fill_u32(reinterpret_cast<uint32_t*>(x->wsum), P * x->wsum_slots, aes ? 0xFF800000u : 0u,
                              x->stream) != hipSuccess ||
        fwrs::launch_fill_u32(reinterpret_cast<uint32_t*>(x->rec), P * 4 * k, 0u, x->stream) != hipSuccess)
        return FWRS_E_HIP;
    if (fwrs::launch_fill_u32(x->idx, P * k, 0xFFFFFFFFu, x->stream) != hipSuccess) return FWRS_E_HIP;
    // the resolve of an empty reservoir is 0
    if (x->res && fwrs::launch_fill_u32(reinterpret_cast<uint32_t*>(x->res), P * 3, 0u, x->stream) != hipSuccess)
        return FWRS_E_HIP;
    x->res_valid = x->res != nullptr;
    if (x->reproject) {
        // counts 0; depths NaN: no previous frame, so the first reprojected frame flushes
        if (fwrs::launch_fill_u32(x->bank_cnt[x->cur], P, 0u, x->stream) != hipSuccess ||
            fwrs::launch_fill_u32(reinterpret_cast<uint32_t*>(x->bank_depth[x->cur]), P, 0x7FC00000u, x->stream) !=
                hipSuccess)
            return FWRS_E_HIP;
    }
    if (fwrs::launch_fill_u32(reinterpret_cast<uint32_t*>(x->stats), kStatBytes / 4, 0u, x->stream) != hipSuccess)
        return FWRS_E_HIP;
    x->t = 0;
    x->pixel_updates = 0;
    x->resolved = false;
    return FWRS_OK;
}

void fill_geometry(FrameDesc& d, int width, int height, int tx, int ty)
{
    d.tile_x_log2 = (uint32_t)log2_exact(tx);
    d.tile_y_log2 = (uint32_t)log2_exact(ty);
    const uint32_t tile_w = (uint32_t)tx;
    d.tiles_x = ((uint32_t)width + tile_w - 1) / tile_w;
    const uint32_t tiles_y = ((uint32_t)height + (uint32_t)ty - 1) / (uint32_t)ty;
    const uint32_t tiles_per_item = (uint32_t)fwrs::kBlock / (uint32_t)(tx * ty);
    d.items = (d.tiles_x * tiles_y + tiles_per_item - 1) / tiles_per_item;
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

FrameDesc make_desc(const fwrs_ctx* x, const float* color, const uint8_t* level, float gx, float gy, float* out,
                    int tx, int ty)
{
    FrameDesc d{};
    d.color = color;
    d.level = level;
    d.out = out;
    d.wsum = x->wsum;
    d.rec = x->rec;
    d.idx = x->idx;
    d.res = x->res;
    d.stats = x->stats;
    d.width = (uint32_t)x->width;
    d.height = (uint32_t)x->height;
    d.t = x->t;
    d.gx = gx;
    d.gy = gy;
    d.c = x->c;
    d.seed = x->prm.seed;
    d.stream_id = x->prm.stream_id;
    d.bias = x->prm.bias_mode;
    d.k = (uint32_t)x->k;
    fill_geometry(d, x->width, x->height, tx, ty);
    return d;
}

bool gaze_ok(float gx, float gy) { return std::isfinite(gx) && std::isfinite(gy); }

// The kernel op of a fused frame (update + resolve of every pixel) of context x
// at frame index t with the resolve plane valid or not (res_valid): from the
// resolve plane once it is valid and the store is past its filling frames,
// filling the plane on the frame before.
int fused_op_at(const fwrs_ctx* x, uint32_t t, bool res_valid)
{
    if (!x->res) return fwrs::kOpFused;
    if (res_valid && t >= x->res_from) return fwrs::kOpCached;
    return t + 1u >= x->res_from ? fwrs::kOpFill : fwrs::kOpFused;
}

int fused_op(const fwrs_ctx* x) { return fused_op_at(x, x->t, x->res_valid); }

// Whether the plane holds every pixel's resolve after a frame run as `op` on x.
bool plane_after(const fwrs_ctx* x, int op)
{
    // kOpPush, kOpFused and kOpIncremental change records without the plane;
    // a group leaves it whole wherever it is kept
    return op == fwrs::kOpCached || op == fwrs::kOpFill || (op == fwrs::kOpGroup && x->res);
}

// After a successful launch of `op` on x: the frame count, the record of the
// last resolve target and the validity of the resolve plane.  (A group of
// frames advances x once per frame, in order.)
void advance(fwrs_ctx* x, int op, const float* out)
{
    if (op != fwrs::kOpResolve) {
        x->t += 1u;
        x->pixel_updates += (uint64_t)x->width * (uint64_t)x->height;
        x->res_valid = plane_after(x, op);
    }
    if (op != fwrs::kOpPush && out) {   // every op that leaves `out` holding the resolve
        x->resolved_out = out;
        x->resolved_at = x->t;
        x->resolved = true;
    } else {
        x->resolved = false;
    }
}

int run_frame(fwrs_ctx* x, const float* color, const uint8_t* level, float gx, float gy, float* out, int op)
{
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    if (op == fwrs::kOpFused) op = fused_op(x);
    FrameDesc d = make_desc(x, color, level, gx, gy, out, x->tile_x, x->tile_y);
    if (fwrs::launch_frame(d, op, x->stream) != hipSuccess) return FWRS_E_HIP;
    advance(x, op, out);
    return FWRS_OK;
}

}  // namespace

extern "C" {

int fwrs_default_params(int width, fwrs_params* p)
{
    if (width <= 0 || !p) return FWRS_E_ARG;
    p->seed = 0;
    p->stream_id = 0;
    p->fov_deg = 70.0f;
    p->fovea_radius_px = 0.05f * (float)width;
    p->bias_mode = FWRS_BIAS_BERNOULLI;
    p->r_m = 41.03f;
    p->a_k = 0.9851f;
    p->r2k = 1.058f;
    p->rek = 22.14f;
    p->flags = 0u;
    p->lambda_decay = 0.0231f;
    return FWRS_OK;
}

size_t fwrs_state_bytes_params(int width, int height, int k, const fwrs_params* params)
{
    if (!sizes_ok(width, height, k) || !params_ok(params)) return 0;
    const size_t banks = (params->flags & FWRS_FLAG_REPROJECT) ? 2 : 1;
    return 4 * banks * bank_elems(pitch_for(width, height), (size_t)k, params->bias_mode, params->flags) + kStatBytes;
}

size_t fwrs_state_bytes(int width, int height, int k)
{
    fwrs_params p;
    if (fwrs_default_params(width > 0 ? width : 1, &p) != FWRS_OK) return 0;
    return fwrs_state_bytes_params(width, height, k, &p);
}

size_t fwrs_state_host_bytes(int width, int height, int k)
{
    if (!sizes_ok(width, height, k)) return 0;
    return (size_t)width * (size_t)height * (8 + 24 * (size_t)k);
}

int fwrs_create_ex(int width, int height, int k, const fwrs_params* params, void* hip_stream, void* arena,
                   size_t arena_bytes, fwrs_ctx** out)
{
    if (!out || !sizes_ok(width, height, k) || !params_ok(params)) return FWRS_E_ARG;
    *out = nullptr;
    const size_t need = fwrs_state_bytes_params(width, height, k, params);
    if (arena && (arena_bytes < need || !aligned(arena, 256))) return FWRS_E_ARG;
    fwrs_ctx* x = new (std::nothrow) fwrs_ctx();
    if (!x) return FWRS_E_NOMEM;
    if (hipGetDevice(&x->device) != hipSuccess) { delete x; return FWRS_E_HIP; }
    x->width = width;
    x->height = height;
    x->k = k;
    x->prm = *params;
    x->c = derive(*params, width);
    x->stream = (hipStream_t)hip_stream;
    x->pitch = pitch_for(width, height);
    x->wsum_slots = fwrs::per_slot_mode(params->bias_mode) ? (size_t)k : 1;
    x->reproject = (params->flags & FWRS_FLAG_REPROJECT) != 0u;
    if (arena) {
        x->arena = arena;
    } else {
        if (hipMalloc(&x->arena, need) != hipSuccess) {
            (void)hipGetLastError();
            delete x;
            return FWRS_E_NOMEM;
        }
        x->owns_arena = true;
    }
    const size_t P = x->pitch, kk = (size_t)k;
    const size_t ws = x->wsum_slots;
    const size_t bank = bank_elems(P, kk, params->bias_mode, params->flags);
    float* base = static_cast<float*>(x->arena);
    for (int b = 0; b < (x->reproject ? 2 : 1); ++b) {
        float* B = base + (size_t)b * bank;
        x->bank_wsum[b] = B;
        x->bank_rec[b] = B + ws * P;
        x->bank_idx[b] = reinterpret_cast<uint32_t*>(B + (ws + 4 * kk) * P);
        if (keeps_res(params->bias_mode, params->flags)) x->res = B + (ws + 5 * kk) * P;
        if (x->reproject) {
            x->bank_cnt[b] = reinterpret_cast<uint32_t*>(B + (ws + 5 * kk) * P);
            x->bank_depth[b] = B + (ws + 5 * kk + 1) * P;
        }
    }
    x->wsum = x->bank_wsum[0];
    x->rec = x->bank_rec[0];
    x->idx = x->bank_idx[0];
    x->stats = reinterpret_cast<unsigned long long*>(base + (x->reproject ? 2 : 1) * bank);
    const int rc = clear_store(x);
    if (rc != FWRS_OK) {
        if (x->owns_arena) (void)hipFree(x->arena);
        delete x;
        return rc;
    }
    *out = x;
    return FWRS_OK;
}

int fwrs_create(int width, int height, int k, fwrs_ctx** out)
{
    fwrs_params p;
    if (fwrs_default_params(width, &p) != FWRS_OK) return FWRS_E_ARG;
    return fwrs_create_ex(width, height, k, &p, nullptr, nullptr, 0, out);
}

int fwrs_destroy(fwrs_ctx* x)
{
    if (!x) return FWRS_OK;
    int rc = FWRS_OK;
    {
        DeviceGuard g(x->device);
        if (hipStreamSynchronize(x->stream) != hipSuccess) rc = FWRS_E_HIP;
        if (x->owns_arena && hipFree(x->arena) != hipSuccess) rc = FWRS_E_HIP;
        if (x->order_ev) (void)hipEventDestroy(x->order_ev);
    }
    delete x;
    return rc;
}

int fwrs_set_stream(fwrs_ctx* x, void* hip_stream)
{
    if (!x) return FWRS_E_ARG;
    if ((hipStream_t)hip_stream != x->stream) {
        // later calls and fwrs_destroy see only the new stream
        DeviceGuard g(x->device);
        if (!g.ok || hipStreamSynchronize(x->stream) != hipSuccess) return FWRS_E_HIP;
    }
    x->stream = (hipStream_t)hip_stream;
    return FWRS_OK;
}

int fwrs_reset(fwrs_ctx* x)
{
    if (!x) return FWRS_E_ARG;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    return clear_store(x);
}

int fwrs_push_frame(fwrs_ctx* x, const float* color, const uint8_t* level_map, float gaze_x, float gaze_y)
{
    if (!x || !color || !level_map || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    if (x->t == 0xFFFFFFFFu || x->reproject) return FWRS_E_STATE;
    return run_frame(x, color, level_map, gaze_x, gaze_y, nullptr, fwrs::kOpPush);
}

int fwrs_resolve(fwrs_ctx* x, float* out)
{
    if (!x || !out) return FWRS_E_ARG;
    return run_frame(x, nullptr, nullptr, 0.0f, 0.0f, out, fwrs::kOpResolve);
}

int fwrs_push_frame_resolve(fwrs_ctx* x, const float* color, const uint8_t* level_map, float gaze_x, float gaze_y,
                            float* out)
{
    if (!x || !color || !level_map || !out || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    if (x->t == 0xFFFFFFFFu || x->reproject) return FWRS_E_STATE;
    return run_frame(x, color, level_map, gaze_x, gaze_y, out, fwrs::kOpFused);
}

int fwrs_push_frame_resolve_incremental(fwrs_ctx* x, const float* color, const uint8_t* level_map, float gaze_x,
                                        float gaze_y, float* out)
{
    if (!x || !color || !level_map || !out || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    if (x->t == 0xFFFFFFFFu || x->reproject) return FWRS_E_STATE;
    if (!x->resolved || x->resolved_out != out || x->resolved_at != x->t) return FWRS_E_STATE;
    return run_frame(x, color, level_map, gaze_x, gaze_y, out, fwrs::kOpIncremental);
}

int fwrs_push_frame_reproject(fwrs_ctx* x, const float* color, const uint8_t* level_map, const float* motion,
                              const float* depth, float gaze_x, float gaze_y, float depth_tol, float* out)
{
    if (!x || !color || !level_map || !motion || !depth || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    if (!std::isfinite(depth_tol) || depth_tol < 0.0f || !aligned(motion, 8)) return FWRS_E_ARG;
    if (!x->reproject || x->t == 0xFFFFFFFFu) return FWRS_E_STATE;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    const int src = x->cur, dst = 1 - x->cur;
    fwrs::ReprojDesc r{};
    r.f = make_desc(x, color, level_map, gaze_x, gaze_y, out, x->tile_x, x->tile_y);
    r.f.wsum = x->bank_wsum[dst];
    r.f.rec = x->bank_rec[dst];
    r.f.idx = x->bank_idx[dst];
    r.motion = motion;
    r.depth = depth;
    r.src_wsum = x->bank_wsum[src];
    r.src_rec = x->bank_rec[src];
    r.src_idx = x->bank_idx[src];
    r.src_cnt = x->bank_cnt[src];
    r.src_depth = x->bank_depth[src];
    r.cnt = x->bank_cnt[dst];
    r.depth_out = x->bank_depth[dst];
    r.tol = depth_tol;
    if (fwrs::launch_reproject(r, x->stream) != hipSuccess) return FWRS_E_HIP;
    x->cur = dst;
    x->wsum = x->bank_wsum[dst];
    x->rec = x->bank_rec[dst];
    x->idx = x->bank_idx[dst];
    x->t += 1u;
    x->pixel_updates += (uint64_t)x->width * (uint64_t)x->height;
    x->resolved = false;
    return FWRS_OK;
}

int fwrs_frame_index(const fwrs_ctx* x, uint32_t* frame_index)
{
    if (!x || !frame_index) return FWRS_E_ARG;
    *frame_index = x->t;
    return FWRS_OK;
}

int fwrs_get_state(const fwrs_ctx* x, fwrs_state_view* v)
{
    if (!x || !v) return FWRS_E_ARG;
    v->width = x->width;
    v->height = x->height;
    v->k = x->k;
    v->frame_index = x->t;
    v->pitch = x->pitch;
    v->wsum_slots = (int)x->wsum_slots;
    v->cnt = x->reproject ? x->bank_cnt[x->cur] : nullptr;
    v->depth = x->reproject ? x->bank_depth[x->cur] : nullptr;
    v->wsum = x->wsum;
    v->rec = x->rec;
    v->idx = x->idx;
    v->res = x->res_valid ? x->res : nullptr;
    return FWRS_OK;
}

int fwrs_download_state(fwrs_ctx* x, void* host, size_t host_bytes)
{
    if (!x || !host || host_bytes != fwrs_state_host_bytes(x->width, x->height, x->k)) return FWRS_E_ARG;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    const size_t N = (size_t)x->width * (size_t)x->height, k = (size_t)x->k;
    const size_t ws = x->wsum_slots;
    std::vector<float> rec, sums;
    std::vector<uint32_t> idx;
    try {
        rec.resize(N * k * 4);
        idx.resize(N * k);
        sums.resize(N * ws);
    } catch (const std::bad_alloc&) {
        return FWRS_E_NOMEM;
    }
    char* h = static_cast<char*>(host);
    float* wsum = reinterpret_cast<float*>(h);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(h + 4 * N);
    float* wt = reinterpret_cast<float*>(h + 8 * N);
    uint32_t* hidx = reinterpret_cast<uint32_t*>(h + (8 + 4 * k) * N);
    float* col = reinterpret_cast<float*>(h + (8 + 8 * k) * N);
    float* wslot = reinterpret_cast<float*>(h + (8 + 20 * k) * N);
    if (hipMemcpyAsync(sums.data(), x->wsum, 4 * N * ws, hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
        hipMemcpyAsync(rec.data(), x->rec, 16 * N * k, hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
        hipMemcpyAsync(idx.data(), x->idx, 4 * N * k, hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
        hipStreamSynchronize(x->stream) != hipSuccess)
        return FWRS_E_HIP;
    // every pixel has seen one candidate per frame: m = frame count
    if (x->reproject) {
        // per-pixel m: a flush restarts it
        if (hipMemcpyAsync(cnt, x->bank_cnt[x->cur], 4 * N, hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
            hipStreamSynchronize(x->stream) != hipSuccess)
            return FWRS_E_HIP;
    } else {
        for (size_t p = 0; p < N; ++p) cnt[p] = x->t;
    }
    // per-slot sums [k][N]: Eq. 7's own ([N][k] on the device; the shared
    // w_sum is then 0), else the shared w_sum repeated for every slot
    const bool per_slot = fwrs::per_slot_mode(x->prm.bias_mode);
    for (size_t p = 0; p < N; ++p) wsum[p] = per_slot ? 0.0f : sums[p];
    for (size_t j = 0; j < k; ++j)
        for (size_t p = 0; p < N; ++p) wslot[j * N + p] = per_slot ? sums[p * k + j] : sums[p];
    // device records [N][k]{w, r, g, b} -> packed planes wt[k][N], idx[k][N], col[k][3][N]
    for (size_t p = 0; p < N; ++p)
        for (size_t j = 0; j < k; ++j) {
            const float* r = &rec[(p * k + j) * 4];
            wt[j * N + p] = r[0];
            col[(j * 3 + 0) * N + p] = r[1];
            col[(j * 3 + 1) * N + p] = r[2];
            col[(j * 3 + 2) * N + p] = r[3];
            hidx[j * N + p] = idx[p * k + j];
        }
    return FWRS_OK;
}

int fwrs_get_stats(fwrs_ctx* x, uint64_t* slot_takes, uint64_t* pixels_changed, uint64_t* pixel_updates,
                   uint64_t* pixels_flushed)
{
    if (!x) return FWRS_E_ARG;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    std::vector<unsigned long long> h(3 * fwrs::kStatSlots);
    if (hipMemcpyAsync(h.data(), x->stats, kStatBytes, hipMemcpyDeviceToHost, x->stream) != hipSuccess)
        return FWRS_E_HIP;
    if (hipStreamSynchronize(x->stream) != hipSuccess) return FWRS_E_HIP;
    uint64_t takes = 0, changed = 0, flushed = 0;
    for (int i = 0; i < fwrs::kStatSlots; ++i) {
        takes += h[3 * i];
        changed += h[3 * i + 1];
        flushed += h[3 * i + 2];
    }
    if (slot_takes) *slot_takes = takes;
    if (pixels_changed) *pixels_changed = changed;
    if (pixel_updates) *pixel_updates = x->pixel_updates;
    if (pixels_flushed) *pixels_flushed = flushed;
    return FWRS_OK;
}

int fwrs_set_resolve_plane_from(fwrs_ctx* x, uint32_t frame_index)
{
    if (!x) return FWRS_E_ARG;
    if (!x->res) return FWRS_E_STATE;
    x->res_from = frame_index;
    return FWRS_OK;
}

int fwrs_set_tile(fwrs_ctx* x, int tile_x, int tile_y)
{
    if (!x || !tile_ok(tile_x, tile_y)) return FWRS_E_ARG;
    x->tile_x = tile_x;
    x->tile_y = tile_y;
    return FWRS_OK;
}

int fwrs_sync(fwrs_ctx* x)
{
    if (!x) return FWRS_E_ARG;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    if (hipStreamSynchronize(x->stream) != hipSuccess) return FWRS_E_HIP;
    return hipGetLastError() == hipSuccess ? FWRS_OK : FWRS_E_HIP;
}

const char* fwrs_strerror(int status)
{
    switch (status) {
        case FWRS_OK: return "ok";
        case FWRS_E_ARG: return "invalid argument";
        case FWRS_E_NOMEM: return "out of memory";
        case FWRS_E_HIP: return "HIP runtime error";
        case FWRS_E_STATE: return "invalid state";
        default: return "unknown status";
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched ticks.  A tick's frame descriptors form a table that one launch of
// the batched kernel reads from device memory (one block per 256-pixel work
// item of all the tick's frames).  An engine keeps a ring of kRing tick slots
// -- a pinned host table, its device copy and an event marking the end of the
// tick that last used the slot -- so the host writes the next tick's table
// while earlier ticks run, and a slot is written again only after its event.
// A tick is the copy of its table (host to device, on the tick's stream) and
// the kernel; in graph mode each slot's copy and kernel are a HIP graph built
// on first use and replayed as it is, updating only the copy's byte count and
// the kernel's grid when the tick's frames change size.
// ---------------------------------------------------------------------------
namespace {

constexpr int kRing = 4;                // even: a slot always serves ticks of the same direction
constexpr int kTickMax = 4096;          // frames per tick (fwrs_tick; engines up to their max_frames)
constexpr int kMaxDevices = 64;

struct TileClass {
    long long min_pixels;
    int tx, ty;
};

// A slot's HIP graph for one of the batched kernels: the table's copy, then the kernel.
struct TickGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr;
    hipGraphNode_t kernel = nullptr;
    size_t copy_bytes = 0;              // bytes the copy node moves
    uint32_t grid = 0;                  // the kernel's grid
};

struct TickSlot {
    void* host = nullptr;               // pinned table
    void* dev = nullptr;                // device table
    hipEvent_t done = nullptr;          // end of the slot's latest tick
    bool pending = false;               // `done` recorded, not yet waited for
    TickGraph graph[fwrs::kTickKinds];  // one per kind of tick (the batched kernel's instantiations)
    const void* head_arg = nullptr;     // the kernel node's argument values
    const void* descs_arg = nullptr;
    void* kparams[2] = {nullptr, nullptr};
};

// The checks every batched call makes on each entry before any device work:
// FWRS_OK, or the status to return.  (A context's entries as a whole are
// checked when the tick is laid out.)
int check_tick(const fwrs_frame* frames, int n, int max_frames, int device)
{
    if (n < 0 || n > max_frames || (n > 0 && !frames)) return FWRS_E_ARG;
    for (int i = 0; i < n; ++i) {
        const fwrs_frame& f = frames[i];
        if (!f.ctx || !f.color || !f.level_map || !f.out || !gaze_ok(f.gaze_x, f.gaze_y)) return FWRS_E_ARG;
        if (f.ctx->device != device) return FWRS_E_ARG;
        if (f.ctx->t == 0xFFFFFFFFu || f.ctx->reproject) return FWRS_E_STATE;
    }
    return FWRS_OK;
}

// Scratch of the tick layout for up to m entries: kTickWorkInts * m ints.
constexpr size_t kTickWorkInts = 6;
struct TickWork {
    int* group;     // [entry] its context's group
    int* count;     // [group] entries
    int* pos;       // [group] entries laid out so far
    int* slot;      // [group] the leader's table index
    int* base;      // [group] table index of the group's second frame
    int* plane;     // [group] whether the resolve plane is whole before the entry being laid out
    TickWork(int* w, size_t m)
        : group(w), count(w + m), pos(w + 2 * m), slot(w + 3 * m), base(w + 4 * m), plane(w + 5 * m) {}
};

// Whether pixel_group runs x's groups: compile-time slot counts and one w_sum per pixel.
bool group_kernel(const fwrs_ctx* x)
{
    return (x->k == 1 || x->k == 2 || x->k == 4 || x->k == 8) && !fwrs::per_slot_mode(x->prm.bias_mode);
}

std::atomic<uint64_t> g_tick_marks{0};

// Lays out the tick of frames[0 .. n) (each entry checked by check_tick): the
// table's head and descriptors, the op each entry runs as (ops[i], the op its
// context then advances by) and the batched kernel's kind for the table.  The entries of one context are its
// consecutive frames in the order given and form one group; groups are
// visited in the order of their first entries, reversed (each group's items
// too) if `reverse`.  FWRS_E_STATE if a context's frames would run past the
// last frame index.
template <typename TileFn>
int layout_tick(const fwrs_frame* frames, int n, bool reverse, TileFn tile, TickWork w, fwrs::TickHead* head,
                FrameDesc* descs, int* ops, int& kind)
{
    kind = fwrs::kTickAlone;
    const uint64_t mark = g_tick_marks.fetch_add(1u, std::memory_order_relaxed) + 1u;
    int groups = 0;
    for (int i = 0; i < n; ++i) {
        fwrs_ctx* x = frames[i].ctx;
        if (x->tick_mark != mark) {
            x->tick_mark = mark;
            x->tick_group = groups;
            w.count[groups] = 0;
            w.pos[groups] = 0;
            w.plane[groups] = x->res_valid ? 1 : 0;
            ++groups;
        }
        w.group[i] = x->tick_group;
        w.count[x->tick_group] += 1;
        if ((uint64_t)x->t + (uint64_t)w.count[x->tick_group] > 0xFFFFFFFFull) return FWRS_E_STATE;
    }
    int later = groups;
    for (int s = 0; s < groups; ++s) {
        const int g = reverse ? groups - 1 - s : s;
        w.slot[g] = s;
        w.base[g] = later;
        later += w.count[g] - 1;
    }
    for (int i = 0; i < n; ++i) {
        const fwrs_frame& f = frames[i];
        fwrs_ctx* x = f.ctx;
        const int g = w.group[i];
        const int nf = w.count[g];
        const int at = w.pos[g]++;
        int tx, ty;
        tile(x, tx, ty);
        FrameDesc& d = descs[at == 0 ? w.slot[g] : w.base[g] + at - 1];
        d = make_desc(x, f.color, f.level_map, f.gaze_x, f.gaze_y, f.out, tx, ty);
        d.t = x->t + (uint32_t)at;
        const bool plane = w.plane[g] != 0;
        const int op = nf > 1 && group_kernel(x) ? fwrs::kOpGroup : fused_op_at(x, d.t, plane);
        w.plane[g] = plane_after(x, op) ? 1 : 0;
        if (nf > 1 && kind != fwrs::kTickGroups8)
            kind = op == fwrs::kOpGroup && x->k == 8 ? fwrs::kTickGroups8 : fwrs::kTickGroups;
        ops[i] = op;
        d.op = (uint32_t)op;
        d.res_ok = plane ? 1u : 0u;
        d.rev = reverse ? 1u : 0u;
        d.nf = at == 0 ? (uint32_t)nf : 1u;
        d.more = at == 0 ? (uint32_t)w.base[g] : 0u;
    }
    head->n = (uint32_t)groups;
    head->total = 0;
    head->pad0 = head->pad1 = 0;
    for (int s = 0; s < groups; ++s) {
        descs[s].first = head->total;
        head->total += descs[s].items;
    }
    return FWRS_OK;
}

}  // namespace

struct fwrs_engine {
    hipStream_t stream = nullptr;
    int device = 0;
    int max_frames = 0;
    int use_graph = 0;
    bool ctx_tiles = false;             // each context's own tile (fwrs_tick) instead of the class table
    size_t table_bytes = 0;
    std::vector<TileClass> classes;
    std::vector<int> ops;               // op of each frame of the tick being issued
    std::vector<int> work;              // the tick layout's scratch (TickWork)
    fwrs::TickArgs args;                // the table of a tick small enough for the kernel's arguments
    TickSlot slot[kRing];
    hipEvent_t done_ev = nullptr;       // end of the latest tick, for contexts on other streams
    uint32_t ticks = 0;                 // ticks issued (odd ticks run in reverse order)
};

namespace {

void graph_free(TickGraph& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = TickGraph{};
}

void engine_free(fwrs_engine* e)
{
    for (TickSlot& sl : e->slot) {
        for (TickGraph& g : sl.graph) graph_free(g);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    if (e->done_ev) (void)hipEventDestroy(e->done_ev);
    delete e;
}

// Allocates the ring; FWRS_OK or an error status (the caller frees e).
int engine_init(fwrs_engine* e, int max_frames)
{
    e->max_frames = max_frames;
    e->table_bytes = fwrs::tick_table_bytes((size_t)max_frames);
    try {
        e->ops.resize((size_t)max_frames);
        e->work.resize(kTickWorkInts * (size_t)max_frames);
    } catch (const std::bad_alloc&) {
        return FWRS_E_NOMEM;
    }
    for (TickSlot& sl : e->slot) {
        if (hipHostMalloc(&sl.host, e->table_bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&sl.dev, e->table_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return FWRS_E_NOMEM;
        }
        if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return FWRS_E_HIP;
        sl.head_arg = sl.dev;
        sl.descs_arg = static_cast<const char*>(sl.dev) + fwrs::kTickDescOffset;
        sl.kparams[0] = &sl.head_arg;
        sl.kparams[1] = &sl.descs_arg;
    }
    return FWRS_OK;
}

void engine_tile(const fwrs_engine* e, const fwrs_ctx* x, int& tx, int& ty)
{
    if (e->ctx_tiles) {
        tx = x->tile_x;
        ty = x->tile_y;
        return;
    }
    const long long pixels = (long long)x->width * x->height;
    tx = kDefaultTileX;
    ty = kDefaultTileY;
    long long best = -1;
    for (const TileClass& c : e->classes)
        if (pixels >= c.min_pixels && c.min_pixels > best) {
            best = c.min_pixels;
            tx = c.tx;
            ty = c.ty;
        }
}

hipKernelNodeParams tick_node(TickSlot& sl, int kind, uint32_t grid)
{
    hipKernelNodeParams kp{};
    kp.func = fwrs::tick_kernel_entry(kind);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(fwrs::kBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = sl.kparams;
    kp.extra = nullptr;
    return kp;
}

// The slot's graph for a kind of tick: the copy of `bytes` of its table, then
// the kernel on `grid` blocks.  A built graph is updated only where the tick's
// size differs from the one it holds.  On failure nothing is left half built.
hipError_t slot_graph(TickSlot& sl, int kind, size_t bytes, uint32_t grid)
{
    TickGraph& g = sl.graph[kind];
    if (g.exec) {
        hipError_t err = hipSuccess;
        if (g.copy_bytes != bytes) {
            err = hipGraphExecMemcpyNodeSetParams1D(g.exec, g.copy, sl.dev, sl.host, bytes, hipMemcpyHostToDevice);
            if (err == hipSuccess) g.copy_bytes = bytes;
        }
        if (err == hipSuccess && g.grid != grid) {
            hipKernelNodeParams kp = tick_node(sl, kind, grid);
            err = hipGraphExecKernelNodeSetParams(g.exec, g.kernel, &kp);
            if (err == hipSuccess) g.grid = grid;
        }
        return err;
    }
    hipError_t err = hipGraphCreate(&g.graph, 0);
    if (err == hipSuccess)
        err = hipGraphAddMemcpyNode1D(&g.copy, g.graph, nullptr, 0, sl.dev, sl.host, bytes, hipMemcpyHostToDevice);
    if (err == hipSuccess) {
        hipKernelNodeParams kp = tick_node(sl, kind, grid);
        err = hipGraphAddKernelNode(&g.kernel, g.graph, &g.copy, 1, &kp);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        graph_free(g);
        return err;
    }
    g.copy_bytes = bytes;
    g.grid = grid;
    return hipSuccess;
}

// One tick of n frames on `stream`: validation, the table, the launch, the
// contexts' frame counts.  Every context's frame enters the state of the
// tick's launch or of none: on FWRS_E_HIP no context has advanced, except that
// if only the final cross-stream ordering failed the tick ran and they did.
int engine_tick(fwrs_engine* e, const fwrs_frame* frames, int n, hipStream_t stream)
{
    const int rc = check_tick(frames, n, e->max_frames, e->device);
    if (rc != FWRS_OK) return rc;
    if (n == 0) return FWRS_OK;
    DeviceGuard g(e->device);
    if (!g.ok) return FWRS_E_HIP;
    // A tick of at most kArgFrames frames carries its table in the kernel's
    // arguments; a larger one copies it from the ring's pinned buffer.
    const bool in_args = n <= fwrs::kArgFrames;
    TickSlot& sl = e->slot[e->ticks % kRing];
    if (!in_args && sl.pending) {
        if (hipEventSynchronize(sl.done) != hipSuccess) return FWRS_E_HIP;
        sl.pending = false;
    }
    // Every other tick walks its work items last first (its frames in reverse
    // order, each frame's items in reverse), so a tick starts on the state the
    // previous one touched last, while it is still in the Infinity Cache.
    const bool reverse = (e->ticks & 1u) != 0u;
    fwrs::TickHead* head = in_args ? &e->args.head : static_cast<fwrs::TickHead*>(sl.host);
    FrameDesc* descs = in_args ? e->args.descs
                               : reinterpret_cast<FrameDesc*>(static_cast<char*>(sl.host) + fwrs::kTickDescOffset);
    int kind = fwrs::kTickAlone;
    const int lrc = layout_tick(frames, n, reverse, [e](const fwrs_ctx* x, int& tx, int& ty) { engine_tile(e, x, tx, ty); },
                                TickWork(e->work.data(), (size_t)e->max_frames), head, descs, e->ops.data(), kind);
    if (lrc != FWRS_OK) return lrc;
    // each context's earlier work on its own stream comes first
    hipError_t err = hipSuccess;
    bool foreign = false;
    for (int i = 0; i < n && err == hipSuccess; ++i) {
        fwrs_ctx* c = frames[i].ctx;
        if (c->stream != stream) {
            foreign = true;
            err = order_after(stream, c->stream, c->order_ev);
        }
    }
    const size_t bytes = fwrs::tick_table_bytes((size_t)n);
    if (err == hipSuccess && in_args) {
        err = fwrs::launch_tick_args(e->args, kind, stream);
    } else if (err == hipSuccess && e->use_graph) {
        err = slot_graph(sl, kind, bytes, head->total);
        if (err == hipSuccess) err = hipGraphLaunch(sl.graph[kind].exec, stream);
    } else if (err == hipSuccess) {
        err = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, stream);
        if (err == hipSuccess) err = fwrs::launch_tick(sl.dev, head->total, kind, stream);
    }
    if (err == hipSuccess && !in_args) err = hipEventRecord(sl.done, stream);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return FWRS_E_HIP;
    }
    if (!in_args) sl.pending = true;
    e->ticks += 1u;
    for (int i = 0; i < n; ++i) advance(frames[i].ctx, e->ops[i], frames[i].out);
    // ... and its later work (and fwrs_destroy) waits for this tick
    if (foreign) {
        if (!e->done_ev && hipEventCreateWithFlags(&e->done_ev, hipEventDisableTiming) != hipSuccess) {
            e->done_ev = nullptr;
            err = hipErrorOutOfMemory;
        }
        if (err == hipSuccess) err = hipEventRecord(e->done_ev, stream);
        for (int i = 0; i < n && err == hipSuccess; ++i)
            if (frames[i].ctx->stream != stream) err = hipStreamWaitEvent(frames[i].ctx->stream, e->done_ev, 0);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            return FWRS_E_HIP;
        }
    }
    return FWRS_OK;
}

// fwrs_tick's engines: one per device, made on first use, kept for the process.
std::mutex g_tick_mutex;
fwrs_engine* g_tick_engine[kMaxDevices] = {};

}  // namespace

extern "C" {

int fwrs_engine_create(void* hip_stream, int max_frames, int use_graph, fwrs_engine** out)
{
    if (!out || max_frames <= 0 || max_frames > kTickMax) return FWRS_E_ARG;
    *out = nullptr;
    fwrs_engine* e = new (std::nothrow) fwrs_engine();
    if (!e) return FWRS_E_NOMEM;
    e->stream = (hipStream_t)hip_stream;
    e->use_graph = use_graph ? 1 : 0;
    if (hipGetDevice(&e->device) != hipSuccess) {
        delete e;
        return FWRS_E_HIP;
    }
    const int rc = engine_init(e, max_frames);
    if (rc != FWRS_OK) {
        engine_free(e);
        return rc;
    }
    *out = e;
    return FWRS_OK;
}

int fwrs_engine_set_tile(fwrs_engine* e, long long min_pixels, int tile_x, int tile_y)
{
    if (!e || min_pixels < 0 || !tile_ok(tile_x, tile_y)) return FWRS_E_ARG;
    for (TileClass& c : e->classes)
        if (c.min_pixels == min_pixels) {
            c.tx = tile_x;
            c.ty = tile_y;
            return FWRS_OK;
        }
    if (e->classes.size() >= 8) return FWRS_E_ARG;
    e->classes.push_back(TileClass{min_pixels, tile_x, tile_y});
    return FWRS_OK;
}

int fwrs_engine_tick(fwrs_engine* e, const fwrs_frame* frames, int n)
{
    if (!e) return FWRS_E_ARG;
    return engine_tick(e, frames, n, e->stream);
}

int fwrs_engine_destroy(fwrs_engine* e)
{
    if (!e) return FWRS_OK;
    int rc = FWRS_OK;
    {
        DeviceGuard g(e->device);
        if (hipStreamSynchronize(e->stream) != hipSuccess) rc = FWRS_E_HIP;
        for (TickSlot& sl : e->slot)
            if (sl.pending && hipEventSynchronize(sl.done) != hipSuccess) rc = FWRS_E_HIP;
        engine_free(e);
    }
    return rc;
}

int fwrs_tick(const fwrs_frame* frames, int n, void* hip_stream)
{
    if (n < 0 || n > kTickMax || (n > 0 && (!frames || !frames[0].ctx))) return FWRS_E_ARG;
    if (n == 0) return FWRS_OK;
    const int dev = frames[0].ctx->device;
    if (dev < 0 || dev >= kMaxDevices) return FWRS_E_ARG;
    std::lock_guard<std::mutex> lock(g_tick_mutex);
    fwrs_engine*& e = g_tick_engine[dev];
    if (!e) {
        DeviceGuard g(dev);
        if (!g.ok) return FWRS_E_HIP;
        fwrs_engine* made = new (std::nothrow) fwrs_engine();
        if (!made) return FWRS_E_NOMEM;
        made->device = dev;
        made->ctx_tiles = true;
        const int rc = engine_init(made, kTickMax);
        if (rc != FWRS_OK) {
            engine_free(made);
            return rc;
        }
        e = made;
    }
    return engine_tick(e, frames, n, (hipStream_t)hip_stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// fwrs_tick_noalloc: fwrs_tick for callers that cannot allocate.  Its tick
// table lives in `scratch`, a file-scope device array (each GPU holds its own
// copy until the process ends), and is written by fill kernels whose
// arguments carry the descriptors, so a call allocates nothing and copies
// nothing from host memory.  In host code `scratch` names no device address:
// each device's address comes from hipGetSymbolAddress (once per device, with
// that device current) and only that address is used.
// ---------------------------------------------------------------------------
namespace {

constexpr int kStaticTickFrames = 256;
constexpr size_t kStaticTickBytes = fwrs::kTickDescOffset + kStaticTickFrames * sizeof(FrameDesc);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticTickBytes];

namespace {

std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};      // each device's address of `scratch`
uint32_t g_scratch_ticks[kMaxDevices] = {};

// The address of `scratch` on device `dev` (the current device): looked up on
// the first call on that device.
hipError_t scratch_table(int dev, void** out)
{
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return err != hipSuccess ? err : hipErrorInvalidSymbol;
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int fwrs_tick_noalloc(const fwrs_frame* frames, int n, void* hip_stream)
{
    if (n > kStaticTickFrames) return FWRS_E_ARG;
    if (n < 0 || (n > 0 && (!frames || !frames[0].ctx))) return FWRS_E_ARG;
    if (n == 0) return FWRS_OK;
    const int dev = frames[0].ctx->device;
    if (dev < 0 || dev >= kMaxDevices) return FWRS_E_ARG;
    const int rc = check_tick(frames, n, kStaticTickFrames, dev);
    if (rc != FWRS_OK) return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    DeviceGuard g(dev);
    if (!g.ok) return FWRS_E_HIP;
    void* table = nullptr;
    if (scratch_table(dev, &table) != hipSuccess) return FWRS_E_HIP;
    // the tick's layout (as in fwrs_tick: every other call on a device runs backwards)
    const bool reverse = (g_scratch_ticks[dev] & 1u) != 0u;
    auto ctx_tile = [](const fwrs_ctx* x, int& tx, int& ty) {
        tx = x->tile_x;
        ty = x->tile_y;
    };
    int ops[kStaticTickFrames];
    int work[kTickWorkInts * kStaticTickFrames];
    int kind = fwrs::kTickAlone;
    hipError_t err = hipSuccess;
    if (n <= fwrs::kArgFrames) {
        // the whole table in the kernel's arguments: the array is not needed
        fwrs::TickArgs args;
        const int lrc = layout_tick(frames, n, reverse, ctx_tile, TickWork(work, kStaticTickFrames), &args.head,
                                    args.descs, ops, kind);
        if (lrc != FWRS_OK) return lrc;
        err = fwrs::launch_tick_args(args, kind, stream);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            return FWRS_E_HIP;
        }
        g_scratch_ticks[dev] += 1u;
        for (int i = 0; i < n; ++i) advance(frames[i].ctx, ops[i], frames[i].out);
        return FWRS_OK;
    }
    FrameDesc descs[kStaticTickFrames];
    fwrs::TickFill fill{};
    const int lrc = layout_tick(frames, n, reverse, ctx_tile, TickWork(work, kStaticTickFrames), &fill.head, descs,
                                ops, kind);
    if (lrc != FWRS_OK) return lrc;
    // the descriptors, kFillFrames per fill launch, then the batched kernel
    for (int at = 0; at < n && err == hipSuccess; at += fwrs::kFillFrames) {
        fill.at = (uint32_t)at;
        fill.count = (uint32_t)std::min(fwrs::kFillFrames, n - at);
        fill.write_head = at == 0 ? 1u : 0u;
        std::memcpy(fill.descs, descs + at, fill.count * sizeof(FrameDesc));
        err = fwrs::launch_tick_fill(table, fill, stream);
    }
    if (err == hipSuccess) err = fwrs::launch_tick(table, fill.head.total, kind, stream);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return FWRS_E_HIP;
    }
    g_scratch_ticks[dev] += 1u;
    for (int i = 0; i < n; ++i) advance(frames[i].ctx, ops[i], frames[i].out);
    return FWRS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Foveation generator
// ---------------------------------------------------------------------------
struct fwrs_foveator {
    int width = 0, height = 0, device = 0;
    uint32_t mode = FWRS_FOV_MIP;
    float r0 = 0.f, r1 = 0.f;
    hipStream_t stream = nullptr;
    hipEvent_t order_ev = nullptr;         // marks `stream` for contexts on other streams
    float* buf = nullptr;                  // one allocation for the level images
    float* l1 = nullptr;
    float* l2 = nullptr;
    uint32_t w1 = 0, h1 = 0, w2 = 0, h2 = 0;
    int radius[2] = {0, 0};
    float wt[2][2 * fwrs::kMaxBlurRadius + 1] = {};
};

namespace {

// Normalised Gaussian weights for offsets -R..R, R = ceil(3 sigma), with the
// library's binary32 exp2; the sum is taken in offset order.
int gauss_weights(float sigma, float* w)
{
    const int R = (int)ceilf(3.0f * sigma);
    const float inv = 1.0f / (2.0f * sigma * sigma);
    float S = 0.0f;
    for (int d = -R; d <= R; ++d) {
        const float a = (float)(d * d) * inv;
        w[d + R] = fwrs::exp2_neg(-(a * 1.44269504088896341f));
        S = S + w[d + R];
    }
    for (int d = -R; d <= R; ++d) w[d + R] = w[d + R] / S;
    return R;
}

fwrs::FovSrc build_levels(fwrs_foveator* f, const float* full, float gaze_x, float gaze_y, hipStream_t stream,
                          hipError_t& err)
{
    fwrs::FovSrc s{};
    s.full = full;
    s.l1 = f->l1;
    s.l2 = f->l2;
    s.w1 = f->w1;
    s.h1 = f->h1;
    s.w2 = f->w2;
    s.h2 = f->h2;
    s.r0sq = f->r0 * f->r0;
    s.r1sq = f->r1 * f->r1;
    s.mode = f->mode;
    if (f->mode == FWRS_FOV_MIP) {
        err = fwrs::launch_mips(full, f->l1, f->l2, (uint32_t)f->width, (uint32_t)f->height, stream);
    } else {
        err = fwrs::launch_gauss_levels(full, f->l1, (uint32_t)f->width, (uint32_t)f->height, gaze_x, gaze_y, s.r0sq,
                                        s.r1sq, f->wt[0], f->wt[1], stream);
    }
    return s;
}

}  // namespace

extern "C" {

int fwrs_foveator_create(int width, int height, float fovea_radius_px, float ring_radius_px, uint32_t mode,
                         void* hip_stream, fwrs_foveator** out)
{
    if (!out || !sizes_ok(width, height, 1)) return FWRS_E_ARG;
    if (!std::isfinite(fovea_radius_px) || !std::isfinite(ring_radius_px) || fovea_radius_px < 0.0f ||
        ring_radius_px < fovea_radius_px)
        return FWRS_E_ARG;
    if (mode != FWRS_FOV_MIP && mode != FWRS_FOV_GAUSS) return FWRS_E_ARG;
    *out = nullptr;
    fwrs_foveator* f = new (std::nothrow) fwrs_foveator();
    if (!f) return FWRS_E_NOMEM;
    if (hipGetDevice(&f->device) != hipSuccess) { delete f; return FWRS_E_HIP; }
    f->width = width;
    f->height = height;
    f->mode = mode;
    f->r0 = fovea_radius_px;
    f->r1 = ring_radius_px;
    f->stream = (hipStream_t)hip_stream;
    f->w1 = ((uint32_t)width + 1) / 2;
    f->h1 = ((uint32_t)height + 1) / 2;
    f->w2 = (f->w1 + 1) / 2;
    f->h2 = (f->h1 + 1) / 2;
    const size_t n = (size_t)width * (size_t)height * 3;
    // level images at 256-byte boundaries
    auto up = [](size_t v) { return (v + 63) / 64 * 64; };
    size_t s1, s2;
    if (mode == FWRS_FOV_MIP) {
        s1 = up((size_t)f->w1 * f->h1 * 3);
        s2 = up((size_t)f->w2 * f->h2 * 3);
    } else {
        s1 = up(n);                        // one plane: each pixel at its own level
        s2 = 0;
        f->radius[0] = gauss_weights(1.0f, f->wt[0]);
        f->radius[1] = gauss_weights(2.0f, f->wt[1]);
        if (f->radius[0] != fwrs::kGaussR1 || f->radius[1] != fwrs::kGaussR2) {
            delete f;
            return FWRS_E_ARG;
        }
    }
    if (hipMalloc(&f->buf, 4 * (s1 + s2)) != hipSuccess) {
        (void)hipGetLastError();
        delete f;
        return FWRS_E_NOMEM;
    }
    f->l1 = f->buf;
    f->l2 = s2 ? f->buf + s1 : nullptr;
    *out = f;
    return FWRS_OK;
}

int fwrs_foveate(fwrs_foveator* f, const float* full, float gaze_x, float gaze_y, float* color, uint8_t* level_map)
{
    if (!f || !full || !color || !level_map || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    DeviceGuard g(f->device);
    if (!g.ok) return FWRS_E_HIP;
    hipError_t err = hipSuccess;
    const fwrs::FovSrc s = build_levels(f, full, gaze_x, gaze_y, f->stream, err);
    if (err != hipSuccess) return FWRS_E_HIP;
    if (fwrs::launch_foveate(s, color, level_map, (uint32_t)f->width, (uint32_t)f->height, gaze_x, gaze_y,
                             f->stream) != hipSuccess)
        return FWRS_E_HIP;
    return FWRS_OK;
}

int fwrs_push_frame_foveated(fwrs_ctx* x, fwrs_foveator* f, const float* full, float gaze_x, float gaze_y, float* out)
{
    if (!x || !f || !full || !gaze_ok(gaze_x, gaze_y)) return FWRS_E_ARG;
    if (f->width != x->width || f->height != x->height || f->device != x->device) return FWRS_E_ARG;
    if (x->t == 0xFFFFFFFFu || x->reproject) return FWRS_E_STATE;
    DeviceGuard g(x->device);
    if (!g.ok) return FWRS_E_HIP;
    // The level images are rebuilt on the context's stream: after the
    // foveator's earlier work, and before its later work and its destroy.
    if (order_after(x->stream, f->stream, f->order_ev) != hipSuccess) return FWRS_E_HIP;
    hipError_t err = hipSuccess;
    fwrs::FovDesc fd{};
    fd.s = build_levels(f, full, gaze_x, gaze_y, x->stream, err);
    if (err != hipSuccess) return FWRS_E_HIP;
    fd.f = make_desc(x, nullptr, nullptr, gaze_x, gaze_y, out, x->tile_x, x->tile_y);
    const int op = out ? fused_op(x) : fwrs::kOpPush;
    if (fwrs::launch_foveated(fd, op, x->stream) != hipSuccess) return FWRS_E_HIP;
    advance(x, op, out);
    if (order_after(f->stream, x->stream, x->order_ev) != hipSuccess) return FWRS_E_HIP;
    return FWRS_OK;
}

int fwrs_foveator_destroy(fwrs_foveator* f)
{
    if (!f) return FWRS_OK;
    int rc = FWRS_OK;
    {
        DeviceGuard g(f->device);
        if (hipStreamSynchronize(f->stream) != hipSuccess) rc = FWRS_E_HIP;
        if (f->buf && hipFree(f->buf) != hipSuccess) rc = FWRS_E_HIP;
        if (f->order_ev) (void)hipEventDestroy(f->order_ev);
    }
    delete f;
    return rc;
}

int fwrs_method_constants(int width, const fwrs_params* params, float* out)
{
    if (width <= 0 || !out || !params_ok(params)) return FWRS_E_ARG;
    const fwrs::Consts c = derive(*params, width);
    const float v[9] = {c.A, c.B, c.IR2, c.IRM, c.C, c.iPPD, c.rf, c.Drf, c.decay};
    for (int i = 0; i < 9; ++i) out[i] = v[i];
    return FWRS_OK;
}

int fwrs_gauss_weights(float sigma, float* out)
{
    if (!out || !std::isfinite(sigma) || sigma <= 0.0f || 3.0f * sigma > (float)fwrs::kMaxBlurRadius) return -1;
    return gauss_weights(sigma, out);
}

}  // extern "C"
