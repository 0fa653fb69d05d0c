/*
 * fwrs.h -- C ABI of the foveated weighted-reservoir-sampling library for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is the per-pixel weighted reservoir sampling of "Enhancing
 * Foveated Rendering with Weighted Reservoir Sampling" (MIG '25, arXiv
 * 2510.03964).  The problem statement (Sec. 4): every frame, each pixel is
 * handed a freshly rendered sample at some foveation level, and the question
 * is whether to keep that sample for display.  Each pixel location is an
 * independent stream (Sec. 4.1); the new sample is scored with the retinal
 * density weight of Eq. 3-4; the reservoir's running weight sum is biased by
 * the Bernoulli survival probability of Eq. 5-6 (Sec. 4.2); then the temporal
 * reservoir and the new sample are combined by Alg. 2 (Sec. 3.2).  This
 * library keeps k such n = 1 reservoirs ("slots") per pixel that see the same
 * candidates and w_sum and draw independent variates; k = 1 is exactly the
 * paper's reservoir.  The displayed colour is the combination of the slots
 * weighted by each kept sample's render-time weight (at k = 1: the kept sample,
 * R_out.x).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Images are row-major, pixel p = y * width + x.  `color` and `out` are
 *    [height][width][3] float32 (RGB, HWC); `level_map` is [height][width]
 *    uint8 with 0 = rendered at full resolution this frame, 1 and 2 = reduced.
 *  - Every buffer argument named color, level_map, out or arena is a DEVICE
 *    pointer on the context's device; `host` arguments are host pointers.
 *    Buffers are owned by the caller and must stay valid until the work
 *    enqueued on the context's stream has completed (stream-ordered use).
 *  - Gaze (gaze_x, gaze_y) is in continuous pixel coordinates of the same
 *    image (pixel centres are at x + 0.5, y + 0.5).
 *  - Calls that enqueue GPU work return as soon as it is enqueued.  An
 *    asynchronous failure is reported by fwrs_sync (FWRS_E_HIP).
 *  - Every call returns a status (FWRS_OK on success) except
 *    fwrs_state_bytes, fwrs_state_bytes_params and fwrs_strerror.  On FWRS_E_ARG nothing was enqueued and the context is
 *    unchanged.
 *  - A context is not thread-safe; distinct contexts are independent.
 *
 * Randomness: slot j of pixel p at frame t (t = 0, 1, ... counts the frames
 * pushed into the context) draws word j % 4 of the Philox4x32-10 block with
 * key (seed, stream_id) and counter (p, t, j / 4, 0) and reads it as
 * u = ((word >> 8) + 1) * 2^-24 in (0, 1].  Results therefore do not depend on
 * how frames are batched, on the launch configuration or on the device.
 *
 * Arithmetic: the weight, the biased weight sum and the keep/replace test are
 * IEEE binary32 operations in a fixed order, without contraction into fused
 * multiply-adds; the decisions (and so the kept frame indices and counts) are
 * reproducible bit for bit.  The resolve is a binary32 weighted mean.
 */
#ifndef FWRS_H
#define FWRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define FWRS_OK 0
#define FWRS_E_ARG 1     /* invalid argument; nothing enqueued */
#define FWRS_E_NOMEM 2   /* device or host allocation failed */
#define FWRS_E_HIP 3     /* a HIP runtime call failed (possibly asynchronously) */
#define FWRS_E_STATE 4   /* call not valid in the object's current state */

/* ---- temporal bias modes (Sec. 4.2) ------------------------------------- */
#define FWRS_BIAS_NONE 0u       /* plain Alg. 2: R1.w_sum is not biased */
#define FWRS_BIAS_BERNOULLI 1u  /* Eq. 6: R1.w_sum *= 1 - w / (R1.w_sum + w) */
/* Eq. 7: every slot keeps its own w_sum, which is scaled by (1 - |dL|) and
 * then by Eq. 6's factor before the slot's Alg. 2 decision; |dL| =
 * min(1, dE94 / 100) with dE94 the CIE94 difference (graphic-arts weights) in
 * CIE Lab (D65 white, linear sRGB primaries) between the slot's sample
 * (reference) and the new pixel. */
#define FWRS_BIAS_FULL 2u
/* Ablations the paper argues against (Sec. 3.1, 4.1, 4.2):
 * memory-less bias: every past candidate's weight decays by exp(-lambda) per
 * frame, i.e. R1.w_sum *= exp(-lambda_decay) before Alg. 2; */
#define FWRS_BIAS_MEMORYLESS 3u
/* A-ES (Efraimidis-Spirakis) instead of A-Chao: each slot keeps its sample's
 * key rand^(1/w), stored as log2(rand) / w (-infinity when empty), and the
 * candidate replaces it when its key is larger; there is no w_sum.  rand is
 * the slot's variate above; log2 is a fixed binary32 series, so keys are
 * reproducible bit for bit. */
#define FWRS_AES 4u

/* Largest slot count per pixel. */
#define FWRS_MAX_K 16

/* ---- context flags ------------------------------------------------------- */
/* The context follows a moving camera (Sec. 4.3): it keeps two banks of the
 * store and is updated only by fwrs_push_frame_reproject. */
#define FWRS_FLAG_REPROJECT 1u
/* The context keeps no resolve plane (12 bytes per pixel less).  By default a
 * context whose bias mode keeps one w_sum per pixel (NONE, BERNOULLI,
 * MEMORYLESS) also stores every pixel's resolve as of the last frame that
 * replaced one of its slots; a fused update + resolve then copies the
 * unchanged resolve of a pixel without a replacement instead of re-reading
 * its k slot records.  Results are identical either way. */
#define FWRS_FLAG_NO_RESOLVE_PLANE 2u

/* Method parameters.
 *   seed, stream_id   Philox key words.
 *   fov_deg           horizontal field of view spanned by `width` pixels; the
 *                     eccentricity of a pixel is its distance to the gaze in
 *                     pixels divided by ppd = width / fov_deg (degrees).
 *   fovea_radius_px   r_f in pixels; inside it the weight is 1 (Eq. 4).
 *   bias_mode         FWRS_BIAS_*.
 *   r_m, a_k, r2k, rek  parameters of the retinal density d(e) of Eq. 3
 *                     (Sec. 4.1 prints a_k = 0.9851, r_2,k = 1.058,
 *                     r_e,k = 22.14; r_m is not printed, default 41.03).
 *   flags             FWRS_FLAG_* (0 by default).
 *   lambda_decay      the memory-less bias rate per frame (FWRS_BIAS_MEMORYLESS;
 *                     not given in the paper; default 0.0231, a 30-frame
 *                     half-life).
 */
typedef struct fwrs_params {
    uint32_t seed;
    uint32_t stream_id;
    float fov_deg;
    float fovea_radius_px;
    uint32_t bias_mode;
    float r_m;
    float a_k;
    float r2k;
    float rek;
    uint32_t flags;
    float lambda_decay;
} fwrs_params;

typedef struct fwrs_ctx fwrs_ctx;

/* Device-side view of a context's reservoir store.  N = width * height,
 * p = y * width + x.
 *   wsum[p]                  float32  w_sum of the pixel's reservoir (Alg. 2);
 *                                     under FWRS_BIAS_FULL wsum[p*k + j] is
 *                                     slot j's own w_sum, under FWRS_AES its
 *                                     key (wsum_slots = k)
 *   rec[(p*k + j)*4 + 0]     float32  render-time weight of slot j's sample
 *   rec[(p*k + j)*4 + 1..3]  float32  its colour (r, g, b)
 *   idx[p*k + j]             uint32   frame index of slot j's sample
 *                                     (0xFFFFFFFF while empty)
 *   res[p*3 + c]             float32  the pixel's resolve (channel c), where
 *                                     the context keeps the resolve plane and
 *                                     it is current; NULL otherwise (before
 *                                     the frames that use it, after
 *                                     fwrs_push_frame or an incremental frame)
 * A pixel's k slots are one contiguous 16k-byte record, so a replacement
 * touches only that pixel's record.  `pitch` (>= N, a multiple of 64) times
 * `wsum_slots` is the element count reserved for the wsum plane.  Alg. 2's candidate count m is
 * the same for every pixel -- each pixel receives one candidate per frame --
 * so it is frame_index and has no plane -- except in a reprojecting context,
 * where a flush restarts a pixel's count: there
 *   cnt[p]                   uint32   m of the pixel's reservoir
 *   depth[p]                 float32  the pixel's depth in the last frame
 *                                     (NaN before the first frame)
 * describe the current bank (NULL otherwise).  The pointers are owned by the
 * context (or by the caller's arena); in a reprojecting context they change
 * with every frame (the banks alternate). */
typedef struct fwrs_state_view {
    int width, height, k;
    uint32_t frame_index;   /* frames pushed so far */
    size_t pitch;
    float* wsum;
    float* rec;
    uint32_t* idx;
    int wsum_slots;         /* 1, or k under FWRS_BIAS_FULL and FWRS_AES */
    uint32_t* cnt;
    float* depth;
    float* res;
} fwrs_state_view;

/* Fills `p` with the defaults for an image `width` pixels wide: seed 0,
 * stream 0, fov 70 degrees, fovea radius 5% of the width, BERNOULLI bias,
 * the Eq. 3 parameters above and no flags.  FWRS_E_ARG if width <= 0 or p is NULL. */
int fwrs_default_params(int width, fwrs_params* p);

/* Device bytes of the reservoir store for a width x height image with k
 * slots under the default parameters (FWRS_BIAS_BERNOULLI, with the resolve
 * plane): 4 * pitch * (1 + 5k + 3) plus a small statistics area, where pitch
 * is width * height rounded up to 64 (20 bytes per slot, 4 for w_sum and 12
 * for the resolve plane per pixel).  Use it for admission control and to size
 * a caller-provided arena.  Returns 0 for invalid sizes. */
size_t fwrs_state_bytes(int width, int height, int k);

/* As fwrs_state_bytes for given parameters: FWRS_BIAS_FULL and FWRS_AES keep
 * one value per slot and no resolve plane (4 * pitch * 6k),
 * FWRS_FLAG_NO_RESOLVE_PLANE drops the plane (4 * pitch * (1 + 5k)),
 * FWRS_FLAG_REPROJECT keeps two banks, each with a count and a depth per pixel
 * and no plane (2 * 4 * pitch * (s + 5k + 2), s = 1 or k), plus the
 * statistics area.  Returns 0 for invalid sizes or parameters. */
size_t fwrs_state_bytes_params(int width, int height, int k, const fwrs_params* params);

/* Host bytes written by fwrs_download_state: width * height * (8 + 24k). */
size_t fwrs_state_host_bytes(int width, int height, int k);

/* Creates a context with fwrs_default_params(width) on the null stream of the
 * current device.  The library allocates the reservoir store and clears it
 * to the empty state (w_sum = 0, wt = 0, col = 0, idx = 0xFFFFFFFF; m = 0).
 * FWRS_E_ARG: width or height <= 0, width * height >= 2^31, k outside
 * [1, FWRS_MAX_K], out NULL.  FWRS_E_NOMEM: allocation failed. */
int fwrs_create(int width, int height, int k, fwrs_ctx** out);

/* As fwrs_create with explicit parameters, a borrowed HIP stream (hipStream_t,
 * NULL = null stream) and an optional caller-owned device arena of
 * `arena_bytes` >= fwrs_state_bytes_params(width, height, k, params) bytes,
 * aligned to 256
 * bytes, that the library uses for the store and never frees.  With arena ==
 * NULL the library allocates.  The arena is cleared on the stream.
 * FWRS_E_ARG also for: params NULL, fov_deg or fovea_radius_px not finite and
 * > 0, bias_mode unknown, a_k outside (0, 1], r_m, r2k or rek not finite and
 * > 0, lambda_decay negative or not finite, unknown flags, arena too small or
 * misaligned. */
int fwrs_create_ex(int width, int height, int k, const fwrs_params* params, void* hip_stream, void* arena,
                   size_t arena_bytes, fwrs_ctx** out);

/* Waits for the context's stream, then frees library-owned memory.  A NULL
 * context is accepted. */
int fwrs_destroy(fwrs_ctx* ctx);

/* Changes the stream later calls enqueue on (borrowed, NULL = null stream).
 * Waits for the previous stream first, so later calls and fwrs_destroy need
 * only the new one.  FWRS_E_HIP if that wait fails (the stream is unchanged). */
int fwrs_set_stream(fwrs_ctx* ctx, void* hip_stream);

/* Enqueues a clear of the store to the empty state and sets the frame index
 * to 0. */
int fwrs_reset(fwrs_ctx* ctx);

/* One frame of the method for every pixel (Sec. 4.1-4.2): weight w from the
 * eccentricity to (gaze_x, gaze_y) (Eq. 3-4; level 0 scores 1), bias of the
 * pixel's w_sum by Eq. 6 (BERNOULLI), then Alg. 2 per slot: the slot takes
 * (color, w, frame index) when u * (W1' + w) > W1', and w_sum <- W1' + w,
 * m <- m + 1.  Under FWRS_BIAS_FULL each slot runs the same test on its own
 * w_sum, biased by Eq. 7 against its own sample.  Then the frame index
 * advances by 1.
 * FWRS_E_ARG: NULL pointers, non-finite gaze.  Level values above 2 are
 * treated like 2 (reduced resolution).  FWRS_E_STATE: 2^32 - 1 frames pushed,
 * or a reprojecting context (use fwrs_push_frame_reproject).  The same holds
 * for fwrs_push_frame_resolve, fwrs_push_frame_resolve_incremental and the
 * engine's ticks. */
int fwrs_push_frame(fwrs_ctx* ctx, const float* color, const uint8_t* level_map, float gaze_x, float gaze_y);

/* Enqueues the resolve into `out` ([height][width][3] float32): for each
 * pixel sum_j wt_j * col_j / sum_j wt_j over its slots; 0 before any frame. */
int fwrs_resolve(fwrs_ctx* ctx, float* out);

/* fwrs_push_frame followed by fwrs_resolve in one pass over memory; the
 * results are bit-identical to the two calls. */
int fwrs_push_frame_resolve(fwrs_ctx* ctx, const float* color, const uint8_t* level_map, float gaze_x,
                            float gaze_y, float* out);

/* fwrs_push_frame_resolve for a caller that keeps its output between frames:
 * writes `out` only at the pixels where some slot was replaced this frame,
 * because every other pixel's resolve is unchanged.  The result is
 * bit-identical to fwrs_push_frame_resolve.  Precondition, checked by the
 * library: `out` is the buffer this context last resolved into -- the `out`
 * of the previous fwrs_push_frame_resolve, fwrs_push_frame_resolve_incremental,
 * fwrs_resolve or batched tick of this context, with no fwrs_push_frame or
 * fwrs_reset since -- and the caller has not modified it.  FWRS_E_STATE if
 * the library's record of the last resolve does not match. */
int fwrs_push_frame_resolve_incremental(fwrs_ctx* ctx, const float* color, const uint8_t* level_map,
                                        float gaze_x, float gaze_y, float* out);

/* One frame of a reprojecting context (FWRS_FLAG_REPROJECT) with a moving
 * camera or moving objects (Sec. 4.3).  `motion` is [height][width][2]
 * float32, 8-byte aligned: the screen-space displacement in pixels of the
 * surface point seen at each pixel since the previous frame (current minus
 * previous position); `depth` is [height][width] float32, the point's depth
 * (> 0, any linear unit).  Reverse reprojection: pixel (x, y) continues the
 * reservoir of pixel (floor(x + 0.5 - mx), floor(y + 0.5 - my)) of the
 * previous frame, if that pixel is inside the image and
 * |depth - its previous depth| <= depth_tol * depth; otherwise (the point was
 * off-screen, occluded or just disoccluded) the pixel's history is flushed and
 * it starts from the empty reservoir (m = 0), so the new candidate fills every
 * slot -- the fall-back to plain foveated rendering of Sec. 6.  Then the
 * frame's update (weight, bias, Alg. 2 per slot) as in fwrs_push_frame, and
 * the resolve into `out` unless `out` is NULL.  Before the first frame there
 * is no previous depth: every pixel starts empty.  Pixels flushed are counted
 * by fwrs_get_stats.
 * FWRS_E_ARG: NULL color, level_map, motion or depth; motion misaligned;
 * non-finite gaze; depth_tol negative or not finite.  FWRS_E_STATE: the
 * context was not created with FWRS_FLAG_REPROJECT, or 2^32 - 1 frames. */
int fwrs_push_frame_reproject(fwrs_ctx* ctx, const float* color, const uint8_t* level_map, const float* motion,
                              const float* depth, float gaze_x, float gaze_y, float depth_tol, float* out);

/* Frames pushed so far (host-side counter; no synchronisation). */
int fwrs_frame_index(const fwrs_ctx* ctx, uint32_t* frame_index);

/* Device pointers and layout of the store (no synchronisation). */
int fwrs_get_state(const fwrs_ctx* ctx, fwrs_state_view* view);

/* Synchronises the stream and copies the store to host memory, packed
 * without padding in the order wsum[N], cnt[N], wt[k][N], idx[k][N],
 * col[k][3][N], wslot[k][N] (N = width * height; cnt[p] = m = frame_index;
 * wslot[j][p] = slot j's w_sum: its own under FWRS_BIAS_FULL, its key under
 * FWRS_AES -- in both wsum[p] is 0 -- else wsum[p] for every j).  `host_bytes` must equal
 * fwrs_state_host_bytes(...). */
int fwrs_download_state(fwrs_ctx* ctx, void* host, size_t host_bytes);

/* Synchronises the stream and returns, since creation or the last reset, the
 * number of slot replacements (takes), of pixel updates in which at least one
 * slot was replaced, of pixel updates, and of reprojected pixel updates whose
 * history was flushed.  Any pointer may be NULL. */
int fwrs_get_stats(fwrs_ctx* ctx, uint64_t* slot_takes, uint64_t* pixels_changed, uint64_t* pixel_updates,
                   uint64_t* pixels_flushed);

/* The frame index from which the context's fused passes (fwrs_push_frame_resolve,
 * batched ticks, fwrs_push_frame_foveated with an output) use the resolve
 * plane: the pass at frame index frame_index - 1 writes it for every pixel, and
 * the later passes read a pixel's slot records only where a slot was replaced
 * (default 32: while a store fills after a reset most pixels change every
 * frame).  0 uses it from the first frame.  A launch policy: results are
 * identical for every value.  FWRS_E_STATE if the context keeps no resolve
 * plane (FWRS_FLAG_NO_RESOLVE_PLANE, FWRS_BIAS_FULL, FWRS_AES, reprojecting). */
int fwrs_set_resolve_plane_from(fwrs_ctx* ctx, uint32_t frame_index);

/* Selects the thread-block tile: tile_x pixels by tile_y rows (one thread per
 * pixel), tile_x * tile_y in {64, 128, 256}, both powers of two.  It only
 * changes the launch shape, never the results. */
int fwrs_set_tile(fwrs_ctx* ctx, int tile_x, int tile_y);

/* Waits for the context's stream; reports asynchronous HIP failures. */
int fwrs_sync(fwrs_ctx* ctx);

/* Text for a status code (static storage). */
const char* fwrs_strerror(int status);

/* ---- batched form --------------------------------------------------------
 * One tick advances several contexts -- any mix of sizes, slot counts and bias
 * modes, on the same device -- by one frame each with a single kernel launch:
 * one block per 256-pixel work item of all the tick's frames, whose
 * descriptors the kernel reads from a table in device memory (copied there
 * from pinned host memory on the tick's stream).  Sec. 3.2 and 4.1 make every
 * pixel of every stream an independent reservoir, so the order in which a tick
 * visits them never changes a result: each entry's results are bit-identical
 * to calling fwrs_push_frame_resolve once per entry, in the entries' order.
 * A context may appear several times in one tick: its entries are its next
 * consecutive frames, in the order they appear (other contexts' entries may
 * come between them), and run as one group, in which each pixel reads its
 * stored state once, applies the frames in turn and writes each frame's
 * output to that entry's `out`, and writes its state back once (for slot
 * counts 1, 2, 4 and 8 with one w_sum per pixel; otherwise each frame passes
 * through the store in turn).  A serving loop that has fallen behind can so
 * run a session's overdue frames for much less memory traffic per frame.
 * A context's entries may share one `out`, which then ends up holding the last
 * one's output (each pixel's frames run in order in one thread); otherwise an
 * entry's buffers must not overlap another entry's `out` or any context's
 * store. */
typedef struct fwrs_frame {
    fwrs_ctx* ctx;
    const float* color;
    const uint8_t* level_map;
    float gaze_x;
    float gaze_y;
    float* out;
} fwrs_frame;

/* Enqueues one tick of the n entries of `frames` (0 <= n <= 4096) on the HIP
 * stream `hip_stream` (borrowed; NULL = null stream), each context tiled as
 * its fwrs_set_tile says.  A context whose own stream is another one is
 * ordered by events: the tick waits for the work already enqueued on that
 * stream, and later work there (fwrs_destroy's wait included) waits for the
 * tick.  A tick of at most 21 entries carries its descriptor table in the
 * kernel's arguments: one launch, nothing copied.  A larger tick's table
 * lives in a ring of pinned host and device buffers that the library
 * allocates for each device on first use and keeps until the process ends,
 * and is copied to the device on the stream before the launch; a call waits
 * (on the host) only if the ring's oldest such tick is still running.
 * Thread-safe.
 * FWRS_E_ARG: n outside [0, 4096], frames NULL with n > 0, a NULL field or
 * non-finite gaze, contexts on different devices.  FWRS_E_STATE: as
 * fwrs_push_frame, also if a context's entries would take its frame index
 * past 2^32 - 1.  On either no context advances.  FWRS_E_HIP: the copy of the table or the
 * launch failed (no context advanced), or only the final cross-stream
 * ordering failed (the tick ran and every context advanced). */
int fwrs_tick(const fwrs_frame* frames, int n, void* hip_stream);

/* fwrs_tick for callers that cannot allocate device or pinned memory (code
 * that must not call hipMalloc: under HIP graph capture, in tight serving
 * loops, or in harnesses that forbid it).  Same arguments and results as
 * fwrs_tick, for at most 256 entries (FWRS_E_ARG beyond, before any device
 * work).  The descriptor table lives in a fixed 46 KiB array in device memory
 * that the library holds for the process's lifetime -- one per GPU, shared by
 * every call on that GPU -- and is written by small kernels whose arguments
 * carry the descriptors, on hip_stream, before the batched kernel (a call of
 * at most 21 entries carries the table in the batched kernel's arguments and
 * does not touch the array): a call allocates nothing and copies nothing from
 * host memory.  Calls on one GPU
 * must not overlap: a call on another stream while an earlier one may still
 * run races on the shared table (calls on one stream are ordered by it).
 * Unlike fwrs_tick it does not order the tick against the contexts' own
 * streams: the caller does.  Other errors as fwrs_tick. */
int fwrs_tick_noalloc(const fwrs_frame* frames, int n, void* hip_stream);

/* An engine: fwrs_tick with its own ring, a fixed stream, a tile table per
 * resolution class and optionally HIP graphs. */
typedef struct fwrs_engine fwrs_engine;

/* Creates an engine for up to `max_frames` (1 .. 4096) entries per tick on a
 * borrowed HIP stream.  With use_graph != 0 each tick of more than 21 entries
 * is the replay of a HIP graph -- the copy of the descriptor table, then the
 * batched kernel -- built once per ring slot and kind of tick and updated only
 * when a tick's frames change size; the stream must then not be capturing.
 * Smaller ticks launch the kernel with the table in its arguments in either
 * mode (a graph would only add a copy).
 * FWRS_E_ARG, FWRS_E_NOMEM, FWRS_E_HIP. */
int fwrs_engine_create(void* hip_stream, int max_frames, int use_graph, fwrs_engine** out);

/* fwrs_tick on the engine's stream and ring, tiles from its class table.
 * FWRS_E_ARG also for n above the engine's max_frames. */
int fwrs_engine_tick(fwrs_engine* eng, const fwrs_frame* frames, int n);

/* Selects the tile shape the engine uses for contexts whose width * height is
 * at least `min_pixels` (class table of up to 8 entries, largest threshold
 * first wins); same constraints as fwrs_set_tile.  Results never change. */
int fwrs_engine_set_tile(fwrs_engine* eng, long long min_pixels, int tile_x, int tile_y);

/* Waits for the engine's stream and ticks, then frees the engine. */
int fwrs_engine_destroy(fwrs_engine* eng);

/* ---- foveation generator (Sec. 4.3) -------------------------------------
 * The paper simulates foveated rendering as a post-process on the full
 * frame: mipmapping with bilinear filtering, or a Gaussian blur that grows
 * with eccentricity.  A foveator turns a full-resolution frame ([height]
 * [width][3] float32, device) into the candidates of the reservoir pass: a
 * level per pixel by its distance d to the gaze (0 if d <= fovea_radius_px,
 * 1 if d <= ring_radius_px, 2 beyond; squared distances of pixel centres in
 * binary32) and a colour
 *   level 0: the frame's own pixel;
 *   FWRS_FOV_MIP:   level l samples mip l (mip l = 2x2 box mean of mip l-1;
 *                   edge texels average the texels that exist) bilinearly at
 *                   the pixel centre, texel centres at (i + 0.5) 2^l, clamp
 *                   to edge;
 *   FWRS_FOV_GAUSS: level l is the frame blurred by a separable Gaussian of
 *                   sigma 2^(l-1) pixels (radius ceil(3 sigma), weights
 *                   normalised, clamp to edge) at the pixel.
 * Every operation is binary32 in a fixed order, so results are reproducible
 * bit for bit.  The foveator owns the level images (mip: N/4 + N/16 texels;
 * Gaussian: N), reused by every call: fwrs_foveate runs on the foveator's
 * stream, and fwrs_push_frame_foveated orders itself against that stream. */
#define FWRS_FOV_MIP 0u
#define FWRS_FOV_GAUSS 1u

typedef struct fwrs_foveator fwrs_foveator;

/* FWRS_E_ARG: sizes as fwrs_create, radii not finite, fovea_radius_px < 0 or
 * ring_radius_px < fovea_radius_px, unknown mode.  FWRS_E_NOMEM. */
int fwrs_foveator_create(int width, int height, float fovea_radius_px, float ring_radius_px, uint32_t mode,
                         void* hip_stream, fwrs_foveator** out);

/* Enqueues the degraded frame into `color` ([height][width][3] float32) and
 * the level map into `level_map` ([height][width] uint8), on the foveator's
 * stream.  FWRS_E_ARG: NULL pointers, non-finite gaze. */
int fwrs_foveate(fwrs_foveator* fov, const float* full, float gaze_x, float gaze_y, float* color,
                 uint8_t* level_map);

/* fwrs_foveate followed by fwrs_push_frame_resolve (or fwrs_push_frame if
 * `out` is NULL) without the intermediate frame: the level images are built,
 * then one reservoir pass samples its candidates from them directly.  Runs on
 * the context's stream; if the foveator's stream is another one, the call
 * first waits (by an event) for the work enqueued there, and later work there
 * (fwrs_foveator_destroy's wait included) waits for this call.  Results are
 * bit-identical to the two calls.
 * FWRS_E_ARG: NULL ctx, fov or full, non-finite gaze, sizes differ.
 * FWRS_E_STATE: as fwrs_push_frame (a reprojecting context is refused). */
int fwrs_push_frame_foveated(fwrs_ctx* ctx, fwrs_foveator* fov, const float* full, float gaze_x, float gaze_y,
                             float* out);

/* Waits for the foveator's stream, then frees it.  NULL is accepted. */
int fwrs_foveator_destroy(fwrs_foveator* fov);

/* ---- the constants the kernels use (host only, no device work) ----------- */
/* The per-context constants derived from `params` for an image `width` pixels
 * wide, exactly as a context passes them to the kernels (Sec. 4.1, Eq. 3-4):
 * out[0..8] = a_k, 1 - a_k, 1 / r_2,k, 1 / r_m, log2(e) / r_e,k, degrees per
 * pixel (fov_deg / width as 1 / (width / fov_deg)), r_f in degrees, the
 * unnormalised density at r_f, and exp(-lambda_decay).  FWRS_E_ARG for
 * width <= 0, out NULL or invalid params. */
int fwrs_method_constants(int width, const fwrs_params* params, float* out);

/* The foveation generator's normalised Gaussian weights for `sigma` pixels:
 * writes 2R + 1 weights (offsets -R..R, R = ceil(3 sigma)) to `out` and returns
 * R; -1 if out is NULL, sigma is not finite and > 0, or R would exceed 32. */
int fwrs_gauss_weights(float sigma, float* out);

#ifdef __cplusplus
}
#endif

#endif /* FWRS_H */
