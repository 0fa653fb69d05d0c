/*
 * CPU oracle for per-pixel weighted reservoir sampling on foveated frames
 * (arXiv 2510.03964, Sec. 3.1, 3.2, 4.1, 4.2).  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU baseline, never
 * by the product path.  Shares nothing with the GPU library.
 *
 * Layout of the oracle's own state, N = width * height, p = y * width + x:
 *   wsum[p]              binary32, the reservoir's w_sum (Alg. 2)
 *   cnt[p]               uint32, candidates seen (Alg. 2's m)
 *   wt[j * N + p]        binary32, render-time weight of the sample in slot j
 *   idx[j * N + p]       uint32, frame index of the sample in slot j
 *                        (0xFFFFFFFF while empty)
 *   col[(j*3 + c)*N + p] binary32, channel c of the sample in slot j
 *   depth[p]             binary32, the depth the pixel had in the previous
 *                        reprojected frame (NaN before the first one)
 * Frames are [H][W][3] binary32 (HWC) with a [H][W] uint8 level map; motion
 * vectors are [H][W][2] binary32 in pixels (current minus previous screen
 * position of the surface point), depth [H][W] binary32 (> 0).
 */
#ifndef FWRS_ORACLE_H
#define FWRS_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWRS_ORACLE_BIAS_NONE 0u
#define FWRS_ORACLE_BIAS_BERNOULLI 1u
#define FWRS_ORACLE_BIAS_FULL 2u      /* Eq. 7: Eq. 6 times (1 - |dL|), per-slot w_sum */
#define FWRS_ORACLE_BIAS_MEMORYLESS 3u   /* Sec. 3.1 memory-less bias: w_sum * exp(-lambda) per frame */
#define FWRS_ORACLE_AES 4u            /* Sec. 3.1 A-ES: keys rand^(1/w), per-slot key, no w_sum */

typedef struct fwrs_oracle_params {
    uint32_t seed;            /* Philox key word 0 */
    uint32_t stream_id;       /* Philox key word 1 */
    float fov_deg;            /* horizontal field of view covered by `width` pixels */
    float fovea_radius_px;    /* r_f in pixels */
    uint32_t bias_mode;       /* FWRS_ORACLE_BIAS_* */
    float r_m, a_k, r2k, rek; /* Eq. 3 parameters */
    float lambda_decay;       /* memory-less bias rate per frame */
} fwrs_oracle_params;

typedef struct fwrs_oracle {
    int width, height, k;
    fwrs_oracle_params prm;
    uint32_t t;
    float A, B, IR2, IRM, C, ppd, iPPD, rf, Drf;
    float decay;    /* exp(-lambda_decay), the memory-less factor per frame */
    float* wsum;
    uint32_t* cnt;
    float* wt;
    uint32_t* idx;
    float* col;
    float* wslot;   /* [k][N] per-slot w_sum (BIAS_FULL) or log2 key (AES); NULL otherwise */
    float* depth;   /* [N] previous reprojected frame's depth */
    uint64_t flushes;   /* reprojected pixel-updates that started from an empty reservoir */
} fwrs_oracle;

void fwrs_oracle_default_params(int width, fwrs_oracle_params* p);
fwrs_oracle* fwrs_oracle_create(int width, int height, int k, const fwrs_oracle_params* p);
void fwrs_oracle_destroy(fwrs_oracle* o);
void fwrs_oracle_push(fwrs_oracle* o, const float* color, const uint8_t* level, float gx, float gy);
void fwrs_oracle_push_rows(fwrs_oracle* o, const float* color, const uint8_t* level, float gx, float gy, int y0,
                           int y1);
void fwrs_oracle_advance(fwrs_oracle* o);
void fwrs_oracle_resolve(const fwrs_oracle* o, double* out);
/* The same for rows [y0, y1) of out only (independent rows: callers may run bands in parallel). */
void fwrs_oracle_resolve_rows(const fwrs_oracle* o, double* out, int y0, int y1);
uint32_t fwrs_oracle_frame_index(const fwrs_oracle* o);
void fwrs_oracle_constants(const fwrs_oracle* o, float out[9]);
void fwrs_oracle_state(const fwrs_oracle* o, float* wsum, uint32_t* cnt, float* wt, uint32_t* idx, float* col);
void fwrs_oracle_slot_sums(const fwrs_oracle* o, float* wslot);
int fwrs_oracle_push_reproject(fwrs_oracle* o, const float* color, const uint8_t* level, const float* motion,
                               const float* depth, float gx, float gy, float depth_tol);
void fwrs_oracle_depth(const fwrs_oracle* o, float* depth);
uint64_t fwrs_oracle_flushes(const fwrs_oracle* o);

#define FWRS_ORACLE_FOV_MIP 0u     /* mipmap + bilinear filtering */
#define FWRS_ORACLE_FOV_GAUSS 1u   /* Gaussian blur growing with the level */
int fwrs_oracle_foveate(const float* full, int width, int height, float gx, float gy, float r0, float r1,
                        uint32_t mode, float* color, uint8_t* level);
void fwrs_oracle_mip_down(const float* src, int width, int height, float* dst);
int fwrs_oracle_gauss_weights(float sigma, float* w);
void fwrs_oracle_blur(const float* src, int width, int height, float sigma, float* tmp, float* dst);
float fwrs_oracle_log2u(uint32_t bits);
void fwrs_oracle_log2u_many(const uint32_t* bits, float* out, size_t count);
float fwrs_oracle_decay(const fwrs_oracle* o);
float fwrs_oracle_cbrt(float t);
void fwrs_oracle_lab(float r, float g, float b, float lab[3]);
float fwrs_oracle_de94(const float ref[3], const float x[3]);
float fwrs_oracle_delta_l(const float rgb_ref[3], const float rgb_x[3]);
void fwrs_oracle_cbrt_many(const float* t, float* out, size_t count);
void fwrs_oracle_lab_many(const float* rgb, float* lab, size_t count);
void fwrs_oracle_de94_many(const float* ref, const float* x, float* out, size_t count);

void fwrs_oracle_philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);
void fwrs_oracle_philox_many(const uint32_t* keys, const uint32_t* ctrs, uint32_t* out, size_t count);
float fwrs_oracle_exp2p(float y);
void fwrs_oracle_exp2p_many(const float* y, float* out, size_t count);
float fwrs_oracle_density(const fwrs_oracle* o, float e);
void fwrs_oracle_density_many(const fwrs_oracle* o, const float* e, float* out, size_t count);
float fwrs_oracle_eccentricity(const fwrs_oracle* o, int x, int y, float gx, float gy);
float fwrs_oracle_weight(const fwrs_oracle* o, int x, int y, uint8_t level, float gx, float gy);
void fwrs_oracle_weight_image(const fwrs_oracle* o, const uint8_t* level, float gx, float gy, float* out);
int fwrs_oracle_trials(int width, int height, int k, const fwrs_oracle_params* p, int px, int py,
                       uint32_t seed0, int n_trials, int n_frames, const float* rgb, const uint8_t* lev,
                       const float* gaze, uint32_t* idx_out, float* wsum_out);

#ifdef __cplusplus
}
#endif

#endif
