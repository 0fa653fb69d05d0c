/*
 * CPU oracle for per-pixel weighted reservoir sampling on foveated frames.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path never
 * links, imports or calls it; it shares no code, header, constant or table
 * with the GPU library.
 *
 * Paper: "Enhancing Foveated Rendering with Weighted Reservoir Sampling"
 * (MIG '25, arXiv 2510.03964).  Section / equation / algorithm numbers below
 * are the paper's:
 *   Sec. 3.1, Eq. 1      A-Chao selection probability w_i / sum_{j<=i} w_j
 *   Sec. 3.1, Alg. 1     A-Chao update of an n = 1 reservoir
 *   Sec. 3.2, Alg. 2     Combine Reservoirs (keep R1 iff rand*(W1+W2) <= W1)
 *   Sec. 4.1             one independent stream per pixel; one new candidate
 *                        per frame; combine temporal reservoir R1 with R2 =
 *                        the new candidate
 *   Sec. 4.1, Eq. 3      Watson retinal density d(e)
 *   Sec. 4.1, Eq. 4      weight w(e) = 1 inside the fovea, d(e)/d(r_f) outside
 *   Sec. 4.2, Eq. 5, 6   Bernoulli survival bias applied to R1.w_sum before
 *                        the combine
 *   Sec. 4.3, Eq. 7      full temporal bias: Eq. 6 additionally scaled by
 *                        (1 - |dL|), dL from the CIE94 colour difference in Lab
 *   Sec. 3.1             A-ES (Efraimidis and Spirakis): key rand^(1/w), the
 *                        largest key is kept; the memory-less temporal bias
 *                        f(j, i) = exp(-lambda (i - j)) (Aggarwal), both as
 *                        the ablations Sec. 4.1 and 4.2 argue against
 *   Sec. 4.3             foveated rendering simulated as a post-process on the
 *                        full frame: mipmapping with bilinear filtering, or a
 *                        Gaussian blur that grows with eccentricity
 *   Sec. 4.3             temporal reprojection by motion vectors; a depth
 *                        disagreement between frames (occlusion or
 *                        disocclusion) flushes the reservoir's history
 *                        (Sec. 6: the pixel falls back to the new sample)
 *
 * Precision.  Every quantity that decides which sample a slot keeps (the
 * weight, the biased weight sum, the uniform variate and the comparison) is
 * evaluated in IEEE binary32, round-to-nearest-even, one operation at a time
 * (build with -ffp-contract=off -fno-fast-math).  The decision is an integer
 * result, so it is taken in the precision the GPU kernel uses.  The resolve
 * (the weighted mean of the slots) has a plain definition and is evaluated in
 * binary64.
 *
 * Readings of the paper that this file fixes (the paper does not state them):
 *   - k slots per pixel are k independent n = 1 A-Chao reservoirs that see the
 *     same candidate stream and share w_sum; each slot draws its own variate.
 *     At k = 1 this is exactly the paper's reservoir.
 *   - rand is uniform on (0, 1] with 24 bits: u = ((bits >> 8) + 1) * 2^-24,
 *     so an empty reservoir always takes its first candidate.
 *   - rand comes from Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11),
 *     key = (seed, stream_id), counter = (pixel, frame, block, 0); slot j
 *     uses word j % 4 of block j / 4.
 *   - eccentricity e (degrees) = pixel-centre distance to the gaze point
 *     divided by ppd = width / fov_deg; r_f = fovea_radius_px / ppd.
 *   - r_m (not printed in the paper) defaults to 41.03 degrees.
 *   - level 0 ("rendered at full fidelity") has weight 1.
 *   - the stored w_sum after a frame is biased W1 + w (Alg. 2 sums the
 *     biased R1.w_sum and R2.w_sum).
 *   - resolve: out = sum_j wt_j * col_j / sum_j wt_j over the slots, with the
 *     render-time weights; 0 before the first frame.
 *   - Eq. 7 (BIAS_FULL): dL compares the new pixel with the slot's sample, so
 *     every slot keeps its own w_sum; |dL| = min(1, dE94 / 100) with dE94 the
 *     CIE94 difference (graphic-arts weights, the slot's sample as reference)
 *     of the two colours in CIE Lab (D65), the colours read as linear RGB.
 *     The factors apply left to right: (W1 * (1 - |dL|)) * (1 - w / (W1 + w)).
 *   - memory-less bias (MEMORYLESS): every past candidate's weight decays by
 *     exp(-lambda) per frame, so the accumulated w_sum is multiplied by
 *     exp(-lambda) before the combine: W1' = W1 * exp(-lambda).
 *   - A-ES (AES): each slot keeps the log2 of its sample's key,
 *     log2(rand) / w (the logarithm orders keys like rand^(1/w) and does not
 *     underflow); the candidate replaces the sample iff its key is larger; an
 *     empty slot has key -infinity.  log2(rand) uses the rand of the slot's
 *     Philox word, computed by the series below.
 *   - foveation levels are rings around the gaze: level 0 within r0 (full
 *     resolution), 1 within r1, 2 beyond (squared distance of the pixel centre
 *     in binary32).  MIP: mip l is the 2x2 box mean of mip l-1 (edge texels
 *     average the texels that exist); level l samples mip l bilinearly at the
 *     pixel centre (texel centres at (i + 0.5) 2^l, clamp to edge, a + f (b - a)
 *     interpolation).  GAUSS: level l is the frame blurred by a separable
 *     Gaussian of sigma 2^(l-1) pixels, radius ceil(3 sigma), weights
 *     normalised to sum 1, clamp to edge.
 *   - reprojection is reverse and nearest: pixel (x, y) continues the
 *     reservoir of the pixel that contains its centre moved back by its motion
 *     vector, (floor(x + 0.5 - mx), floor(y + 0.5 - my)); that history is kept
 *     when the point is inside the image and |depth - previous depth there| <=
 *     depth_tol * depth, otherwise the pixel starts from an empty reservoir
 *     (m = 0, w_sum = 0, slots empty) before the frame's update.  Before the
 *     first reprojected frame no depth exists, so every pixel starts empty.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fwrs_oracle.h"

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon et al., SC'11: a 4-word counter and a  */
/* 2-word key; each round multiplies words 0 and 2 by fixed odd constants,    */
/* takes the high and low halves of the 64-bit products, xors the high halves */
/* with the other two words and the round key, and permutes; the key is       */
/* advanced by the two Weyl constants between rounds.                         */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void fwrs_oracle_philox(const uint32_t key_in[2], const uint32_t ctr_in[4], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* 2^y for y <= 0: exact range reduction y = n + f with n = rint(y) and       */
/* |f| <= 1/2, then the degree-7 Taylor polynomial of 2^f = exp(f ln 2) in    */
/* Horner form (one multiply and one add per step), then scaling by 2^n.      */
/* Coefficient i is the binary32 rounding of (ln 2)^i / i!.                   */
/* ------------------------------------------------------------------------ */
static float exp2_coef[8];

static void init_exp2_coef(void)
{
    /* (ln 2)^i / i! accumulated in binary64, then rounded once to binary32. */
    const double ln2 = 0.69314718055994530942;
    double c = 1.0;
    for (int i = 0; i < 8; ++i) {
        if (i > 0) c = c * ln2 / (double)i;
        exp2_coef[i] = (float)c;
    }
}

float fwrs_oracle_exp2p(float y)
{
    if (exp2_coef[0] != 1.0f) init_exp2_coef();
    float n = rintf(y);
    float f = y - n;
    float p = exp2_coef[7];
    for (int i = 6; i >= 0; --i) {
        p = p * f;
        p = p + exp2_coef[i];
    }
    return ldexpf(p, (int)n);
}

/* ------------------------------------------------------------------------ */
/* Eq. 3 multiplied through by (1 + e/r_2k)^2; the 2 d_c(0) factor cancels in */
/* Eq. 4 and is dropped:                                                      */
/*   d(e) ~ num(e) / den(e),                                                  */
/*   num(e) = a_k + (1 - a_k) exp(-e / r_ek) (1 + e/r_2k)^2,                  */
/*   den(e) = (1 + e/r_2k)^2 (1 + e/r_m).                                     */
/* exp(-e / r_ek) = 2^(-e log2(e) / r_ek).                                    */
/* ------------------------------------------------------------------------ */
static void density_terms(const fwrs_oracle* o, float e, float* num, float* den)
{
    float t1 = 1.0f + e * o->IRM;
    float t2 = 1.0f + e * o->IR2;
    float T = t2 * t2;
    float E = fwrs_oracle_exp2p(-(e * o->C));
    *num = o->A + (o->B * E) * T;
    *den = T * t1;
}

float fwrs_oracle_density(const fwrs_oracle* o, float e)
{
    float num, den;
    density_terms(o, e, &num, &den);
    return num / den;
}

float fwrs_oracle_eccentricity(const fwrs_oracle* o, int x, int y, float gx, float gy)
{
    float dx = ((float)x + 0.5f) - gx;
    float dy = ((float)y + 0.5f) - gy;
    return sqrtf(dx * dx + dy * dy) * o->iPPD;
}

/* Eq. 4, with level 0 (a pixel rendered at full fidelity this frame) scored 1. */
float fwrs_oracle_weight(const fwrs_oracle* o, int x, int y, uint8_t level, float gx, float gy)
{
    float e = fwrs_oracle_eccentricity(o, x, y, gx, gy);
    if (level == 0 || e <= o->rf) return 1.0f;
    float num, den;
    density_terms(o, e, &num, &den);
    return fminf(1.0f, num / (den * o->Drf));
}

/* ------------------------------------------------------------------------ */
/* log2 of the uniform variate u = ((bits >> 8) + 1) * 2^-24, for A-ES keys:   */
/* the binary32 value nearest to the real number log2(u) = log2(m) - 24,       */
/* m = (bits >> 8) + 1 in 1 .. 2^24.  log2(m) is an integer when m is a power  */
/* of two and irrational otherwise, so it is never halfway between two        */
/* binary32 values and the nearest one is unique.  It is found from the        */
/* extended-precision log2l (64-bit significand): rounding that value to       */
/* binary32 gives the nearest binary32 unless it lies within a few of its own  */
/* ulps of a binary32 midpoint, which the function reports by returning NaN    */
/* (a test evaluates all 2^24 variates and finds none).                        */
/* ------------------------------------------------------------------------ */
float fwrs_oracle_log2u(uint32_t bits)
{
    const uint32_t m = (bits >> 8) + 1u;                 /* 1 .. 2^24 */
    const long double v = log2l((long double)m) - 24.0L;
    if (v == 0.0L) return 0.0f;
    const float f = (float)v;
    /* the binary32 neighbours of v and the midpoint between them (exact in long double) */
    const float lo = (long double)f <= v ? f : nextafterf(f, -INFINITY);
    const float hi = nextafterf(lo, INFINITY);
    const long double mid = ((long double)lo + (long double)hi) * 0.5L;
    const long double guard = fabsl(v) * 0x1p-58L;       /* a few ulps of the 64-bit significand */
    if (fabsl(v - mid) <= guard) return NAN;
    return f;
}

float fwrs_oracle_decay(const fwrs_oracle* o) { return o->decay; }

/* ------------------------------------------------------------------------ */
/* Foveation generator (Sec. 4.3).  The paper renders the full frame and then */
/* degrades it away from the gaze, either by mipmapping with bilinear         */
/* filtering or by a progressively stronger Gaussian blur; the degraded frame */
/* and its level map are the candidates of the reservoir pass.                */
/* ------------------------------------------------------------------------ */
/* One mip level down: dst[(j * ceil(W/2) + i) * 3 + c] = mean of the texels  */
/* (2i + dx, 2j + dy), dx, dy in {0, 1}, that lie in the source, summed in    */
/* row-major order.                                                           */
void fwrs_oracle_mip_down(const float* src, int width, int height, float* dst)
{
    const int w2 = (width + 1) / 2, h2 = (height + 1) / 2;
    for (int j = 0; j < h2; ++j)
        for (int i = 0; i < w2; ++i)
            for (int c = 0; c < 3; ++c) {
                float s = 0.0f;
                int n = 0;
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const int x = 2 * i + dx, y = 2 * j + dy;
                        if (x < width && y < height) {
                            s = s + src[((size_t)y * (size_t)width + (size_t)x) * 3 + (size_t)c];
                            n = n + 1;
                        }
                    }
                dst[((size_t)j * (size_t)w2 + (size_t)i) * 3 + (size_t)c] = s / (float)n;
            }
}

/* Bilinear sample of channel c of a w x h level at the centre of full-res */
/* pixel (x, y), the level being 1/scale of the full resolution.           */
static float bilinear(const float* lv, int w, int h, int x, int y, float inv_scale, int c)
{
    const float u = ((float)x + 0.5f) * inv_scale - 0.5f;
    const float v = ((float)y + 0.5f) * inv_scale - 0.5f;
    const float fu = floorf(u), fv = floorf(v);
    const float fx = u - fu, fy = v - fv;
    int i0 = (int)fu, j0 = (int)fv;
    int i1 = i0 + 1, j1 = j0 + 1;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > w - 1) i1 = w - 1;
    if (j1 > h - 1) j1 = h - 1;
    if (i0 > w - 1) i0 = w - 1;
    if (j0 > h - 1) j0 = h - 1;
    const float t00 = lv[((size_t)j0 * (size_t)w + (size_t)i0) * 3 + (size_t)c];
    const float t10 = lv[((size_t)j0 * (size_t)w + (size_t)i1) * 3 + (size_t)c];
    const float t01 = lv[((size_t)j1 * (size_t)w + (size_t)i0) * 3 + (size_t)c];
    const float t11 = lv[((size_t)j1 * (size_t)w + (size_t)i1) * 3 + (size_t)c];
    const float top = t00 + fx * (t10 - t00);
    const float bot = t01 + fx * (t11 - t01);
    return top + fy * (bot - top);
}

/* Normalised Gaussian weights w[0 .. 2R] for offsets -R .. R, R = ceil(3 sigma): */
/* g(d) = exp(-d^2 / (2 sigma^2)) by the project's exp2, divided by their sum     */
/* taken in offset order.  Returns R, or -1 if R exceeds 32.                      */
int fwrs_oracle_gauss_weights(float sigma, float* w)
{
    const int R = (int)ceilf(3.0f * sigma);
    if (R < 0 || R > 32) return -1;
    const float inv = 1.0f / (2.0f * sigma * sigma);
    float S = 0.0f;
    for (int d = -R; d <= R; ++d) {
        const float a = (float)(d * d) * inv;
        w[d + R] = fwrs_oracle_exp2p(-(a * 1.44269504088896341f));
        S = S + w[d + R];
    }
    for (int d = -R; d <= R; ++d) w[d + R] = w[d + R] / S;
    return R;
}

/* Separable Gaussian blur, clamp to edge: a horizontal pass into tmp, then a */
/* vertical pass into dst; each output accumulates w[d] * sample in offset    */
/* order from 0.                                                              */
void fwrs_oracle_blur(const float* src, int width, int height, float sigma, float* tmp, float* dst)
{
    float w[65];
    const int R = fwrs_oracle_gauss_weights(sigma, w);
    if (R < 0) return;
    for (int y = 0; y < height; ++y)
        for (int x = 0; x < width; ++x)
            for (int c = 0; c < 3; ++c) {
                float acc = 0.0f;
                for (int d = -R; d <= R; ++d) {
                    int xx = x + d;
                    if (xx < 0) xx = 0;
                    if (xx > width - 1) xx = width - 1;
                    acc = acc + w[d + R] * src[((size_t)y * (size_t)width + (size_t)xx) * 3 + (size_t)c];
                }
                tmp[((size_t)y * (size_t)width + (size_t)x) * 3 + (size_t)c] = acc;
            }
    for (int y = 0; y < height; ++y)
        for (int x = 0; x < width; ++x)
            for (int c = 0; c < 3; ++c) {
                float acc = 0.0f;
                for (int d = -R; d <= R; ++d) {
                    int yy = y + d;
                    if (yy < 0) yy = 0;
                    if (yy > height - 1) yy = height - 1;
                    acc = acc + w[d + R] * tmp[((size_t)yy * (size_t)width + (size_t)x) * 3 + (size_t)c];
                }
                dst[((size_t)y * (size_t)width + (size_t)x) * 3 + (size_t)c] = acc;
            }
}

/* The foveated frame and its level map from the full frame and the gaze.     */
/* Returns 0, 1 for an unknown mode, 2 if memory is short.                    */
int fwrs_oracle_foveate(const float* full, int width, int height, float gx, float gy, float r0, float r1,
                        uint32_t mode, float* color, uint8_t* level)
{
    if (mode != FWRS_ORACLE_FOV_MIP && mode != FWRS_ORACLE_FOV_GAUSS) return 1;
    const size_t n = (size_t)width * (size_t)height;
    const int w1 = (width + 1) / 2, h1 = (height + 1) / 2;
    const int w2 = (w1 + 1) / 2, h2 = (h1 + 1) / 2;
    float *a = NULL, *b = NULL, *tmp = NULL;
    if (mode == FWRS_ORACLE_FOV_MIP) {
        a = (float*)malloc((size_t)w1 * (size_t)h1 * 3 * sizeof(float));
        b = (float*)malloc((size_t)w2 * (size_t)h2 * 3 * sizeof(float));
        if (!a || !b) { free(a); free(b); return 2; }
        fwrs_oracle_mip_down(full, width, height, a);
        fwrs_oracle_mip_down(a, w1, h1, b);
    } else {
        a = (float*)malloc(n * 3 * sizeof(float));
        b = (float*)malloc(n * 3 * sizeof(float));
        tmp = (float*)malloc(n * 3 * sizeof(float));
        if (!a || !b || !tmp) { free(a); free(b); free(tmp); return 2; }
        fwrs_oracle_blur(full, width, height, 1.0f, tmp, a);
        fwrs_oracle_blur(full, width, height, 2.0f, tmp, b);
    }
    const float r0sq = r0 * r0, r1sq = r1 * r1;
    for (int y = 0; y < height; ++y)
        for (int x = 0; x < width; ++x) {
            const size_t p = (size_t)y * (size_t)width + (size_t)x;
            const float dx = ((float)x + 0.5f) - gx;
            const float dy = ((float)y + 0.5f) - gy;
            const float d2 = dx * dx + dy * dy;
            const uint8_t lv = d2 <= r0sq ? 0 : (d2 <= r1sq ? 1 : 2);
            level[p] = lv;
            for (int c = 0; c < 3; ++c) {
                float v;
                if (lv == 0) v = full[p * 3 + (size_t)c];
                else if (mode == FWRS_ORACLE_FOV_GAUSS) v = (lv == 1 ? a : b)[p * 3 + (size_t)c];
                else if (lv == 1) v = bilinear(a, w1, h1, x, y, 0.5f, c);
                else v = bilinear(b, w2, h2, x, y, 0.25f, c);
                color[p * 3 + (size_t)c] = v;
            }
        }
    free(a); free(b); free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Colour difference for Eq. 7.                                               */
/* ------------------------------------------------------------------------ */
/* Cube root: the binary32 value nearest to the real number t^(1/3).  For a  */
/* binary32 y = M 2^E (M a 24-bit integer) the midpoint to the next binary32   */
/* above is (2M + 1) 2^(E-1), a 25-bit significand, whose cube has 75 bits and */
/* is never a binary32; so the real cube root of t is never halfway and the   */
/* nearest binary32 is unique: it is the y whose lower midpoint cubed is below */
/* t and whose upper midpoint cubed is above t.  Those cubes are compared with */
/* t exactly in 128-bit integer arithmetic, starting from libm's binary64     */
/* cube root rounded to binary32 and stepping to a neighbour while a           */
/* comparison fails.  cbrt(0) = 0, cbrt(inf) = inf, NaN stays NaN, and         */
/* cbrt(-t) = -cbrt(t).                                                        */
typedef unsigned __int128 u128;

static int bit_length(u128 v)
{
    int n = 0;
    while (v) { v >>= 1; ++n; }
    return n;
}

/* Sign of a 2^ea - b 2^eb for a, b > 0. */
static int compare_scaled(u128 a, int ea, u128 b, int eb)
{
    const int la = bit_length(a) + ea, lb = bit_length(b) + eb;
    if (la != lb) return la < lb ? -1 : 1;
    /* same binade: align the exponents (the shifted value keeps the other's bit length) */
    if (ea > eb) a <<= (unsigned)(ea - eb);
    else b <<= (unsigned)(eb - ea);
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* A finite binary32 x > 0 as an integer significand times a power of two. */
static void split_float(float x, u128* sig, int* ex)
{
    int e;
    const float f = frexpf(x, &e);                       /* x = f 2^e, f in [1/2, 1) */
    *sig = (u128)(uint32_t)ldexpf(f, 24);                /* exact: 24 bits */
    *ex = e - 24;
}

/* Sign of m^3 - t, m the midpoint between y > 0 and the next binary32 above it. */
static int midpoint_cube_vs(float y, float t)
{
    u128 M, T;
    int E, Et;
    split_float(y, &M, &E);
    split_float(t, &T, &Et);
    const u128 m = 2 * M + 1;                            /* midpoint = m 2^(E-1) */
    return compare_scaled(m * m * m, 3 * (E - 1), T, Et);
}

float fwrs_oracle_cbrt(float t)
{
    if (t != t || t == 0.0f || t == INFINITY || t == -INFINITY) return t;
    if (t < 0.0f) return -fwrs_oracle_cbrt(-t);
    float y = (float)cbrt((double)t);
    /* libm's binary64 cube root rounded to binary32 is within one ulp, so a step or two at most:
     * up while the cube root lies above the upper midpoint, down while it lies below the lower
     * midpoint (the upper midpoint of the binary32 below y).  NaN if that does not settle. */
    for (int step = 0; step < 4; ++step) {
        if (midpoint_cube_vs(y, t) < 0) y = nextafterf(y, INFINITY);
        else if (midpoint_cube_vs(nextafterf(y, 0.0f), t) > 0) y = nextafterf(y, 0.0f);
        else return y;
    }
    return NAN;
}

/* CIE Lab f(): cube root above (6/29)^3, the linear segment below. */
static float lab_f(float t)
{
    const float eps = 216.0f / 24389.0f;         /* (6/29)^3 */
    const float slope = 841.0f / 108.0f;         /* 1 / (3 (6/29)^2) */
    const float off = 4.0f / 29.0f;
    if (t > eps) return fwrs_oracle_cbrt(t);
    return t * slope + off;
}

/* Linear RGB (sRGB primaries) -> XYZ -> Lab, D65 white. */
void fwrs_oracle_lab(float r, float g, float b, float lab[3])
{
    float X = (0.4124564f * r + 0.3575761f * g) + 0.1804375f * b;
    float Y = (0.2126729f * r + 0.7151522f * g) + 0.0721750f * b;
    float Z = (0.0193339f * r + 0.1191920f * g) + 0.9503041f * b;
    float fx = lab_f(X / 0.95047f);
    float fy = lab_f(Y / 1.0f);
    float fz = lab_f(Z / 1.08883f);
    lab[0] = 116.0f * fy - 16.0f;
    lab[1] = 500.0f * (fx - fy);
    lab[2] = 200.0f * (fy - fz);
}

/* CIE94, graphic-arts weights (k_L = k_C = k_H = 1, K1 = 0.045, K2 = 0.015),
 * `ref` is the reference colour whose chroma scales S_C and S_H. */
float fwrs_oracle_de94(const float ref[3], const float x[3])
{
    float dL = ref[0] - x[0];
    float C1 = sqrtf(ref[1] * ref[1] + ref[2] * ref[2]);
    float C2 = sqrtf(x[1] * x[1] + x[2] * x[2]);
    float dC = C1 - C2;
    float da = ref[1] - x[1];
    float db = ref[2] - x[2];
    float dH2 = (da * da + db * db) - dC * dC;
    if (dH2 < 0.0f) dH2 = 0.0f;                  /* rounding can leave it slightly negative */
    float SC = 1.0f + 0.045f * C1;
    float SH = 1.0f + 0.015f * C1;
    float tC = dC / SC;
    float sum = dL * dL + tC * tC + dH2 / (SH * SH);
    return sqrtf(sum);
}

/* |dL| of Eq. 7 between a reservoir sample (reference) and a new pixel. */
float fwrs_oracle_delta_l(const float rgb_ref[3], const float rgb_x[3])
{
    float a[3], b[3];
    fwrs_oracle_lab(rgb_ref[0], rgb_ref[1], rgb_ref[2], a);
    fwrs_oracle_lab(rgb_x[0], rgb_x[1], rgb_x[2], b);
    return fminf(1.0f, fwrs_oracle_de94(a, b) / 100.0f);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                    */
/* ------------------------------------------------------------------------ */
void fwrs_oracle_default_params(int width, fwrs_oracle_params* p)
{
    p->seed = 0;
    p->stream_id = 0;
    p->fov_deg = 70.0f;
    p->fovea_radius_px = 0.05f * (float)width;
    p->bias_mode = FWRS_ORACLE_BIAS_BERNOULLI;
    p->r_m = 41.03f;       /* not printed in the paper; Watson (2014) */
    p->a_k = 0.9851f;      /* Sec. 4.1, parameters of Eq. 3 */
    p->r2k = 1.058f;
    p->rek = 22.14f;
    p->lambda_decay = 0.0231f;   /* not given in the paper: a 30-frame half-life */
}

static void derive_constants(fwrs_oracle* o)
{
    const fwrs_oracle_params* p = &o->prm;
    o->A = p->a_k;
    o->B = 1.0f - p->a_k;
    o->IR2 = 1.0f / p->r2k;
    o->IRM = 1.0f / p->r_m;
    o->C = 1.44269504088896341f / p->rek;   /* log2(e) / r_ek */
    o->ppd = (float)o->width / p->fov_deg;
    o->iPPD = 1.0f / o->ppd;
    o->rf = p->fovea_radius_px * o->iPPD;
    float num, den;
    density_terms(o, o->rf, &num, &den);
    o->Drf = num / den;
    o->decay = fwrs_oracle_exp2p(-(p->lambda_decay * 1.44269504088896341f));   /* exp(-lambda) */
}

/* The per-slot value of an empty slot: w_sum 0 (Eq. 7), key -infinity (A-ES). */
static float empty_slot_sum(const fwrs_oracle* o)
{
    return o->prm.bias_mode == FWRS_ORACLE_AES ? -INFINITY : 0.0f;
}

fwrs_oracle* fwrs_oracle_create(int width, int height, int k, const fwrs_oracle_params* p)
{
    if (width <= 0 || height <= 0 || k < 1 || k > 16) return NULL;
    fwrs_oracle* o = (fwrs_oracle*)calloc(1, sizeof(fwrs_oracle));
    if (!o) return NULL;
    o->width = width;
    o->height = height;
    o->k = k;
    if (p) o->prm = *p; else fwrs_oracle_default_params(width, &o->prm);
    size_t n = (size_t)width * (size_t)height;
    o->wsum = (float*)calloc(n, sizeof(float));
    o->cnt = (uint32_t*)calloc(n, sizeof(uint32_t));
    o->wt = (float*)calloc(n * (size_t)k, sizeof(float));
    o->idx = (uint32_t*)malloc(n * (size_t)k * sizeof(uint32_t));
    o->col = (float*)calloc(n * (size_t)k * 3, sizeof(float));
    const int per_slot = o->prm.bias_mode == FWRS_ORACLE_BIAS_FULL || o->prm.bias_mode == FWRS_ORACLE_AES;
    if (per_slot) o->wslot = (float*)malloc(n * (size_t)k * sizeof(float));
    o->depth = (float*)malloc(n * sizeof(float));
    if (!o->wsum || !o->cnt || !o->wt || !o->idx || !o->col || !o->depth ||
        (per_slot && !o->wslot)) {
        fwrs_oracle_destroy(o);
        return NULL;
    }
    for (size_t i = 0; i < n * (size_t)k; ++i) o->idx[i] = 0xFFFFFFFFu;   /* empty slot */
    for (size_t i = 0; i < n; ++i) o->depth[i] = NAN;                     /* no previous frame */
    if (per_slot)
        for (size_t i = 0; i < n * (size_t)k; ++i) o->wslot[i] = empty_slot_sum(o);
    derive_constants(o);
    return o;
}

void fwrs_oracle_destroy(fwrs_oracle* o)
{
    if (!o) return;
    free(o->wsum); free(o->cnt); free(o->wt); free(o->idx); free(o->col); free(o->wslot); free(o->depth);
    free(o);
}

/* ------------------------------------------------------------------------ */
/* One frame of one pixel stream (Sec. 4.1, 4.2):                             */
/*   R2 = {x_new, w} (Eq. 4);                                                 */
/*   bias R1.w_sum by the survival probability of Eq. 5 (Eq. 6), BERNOULLI;   */
/*   combine per Alg. 2, independently in every slot;                         */
/*   R_out.w_sum = biased R1.w_sum + w, R_out.m = R1.m + 1.                   */
/* The pixel's state lives at stride `n` (pixels per plane) from wsum/cnt.    */
/* ------------------------------------------------------------------------ */
static void update_pixel(const fwrs_oracle* o, int x, int y, uint32_t p, uint32_t t,
                         const float rgb[3], uint8_t level, float gx, float gy,
                         float* wsum, uint32_t* cnt, float* wt, uint32_t* idx, float* col, float* wslot, size_t n)
{
    const int k = o->k;
    float w = fwrs_oracle_weight(o, x, y, level, gx, gy);
    if (o->prm.bias_mode == FWRS_ORACLE_AES) {
        /* A-ES per slot: the larger key rand^(1/w) wins, compared as log2(rand) / w. */
        uint32_t key[2] = {o->prm.seed, o->prm.stream_id};
        uint32_t words[4];
        int have_block = -1;
        for (int j = 0; j < k; ++j) {
            int b = j / 4;
            if (b != have_block) {
                uint32_t ctr[4] = {p, t, (uint32_t)b, 0u};
                fwrs_oracle_philox(key, ctr, words);
                have_block = b;
            }
            float kn = fwrs_oracle_log2u(words[j % 4]) / w;
            if (kn > wslot[(size_t)j * n]) {
                col[((size_t)j * 3 + 0) * n] = rgb[0];
                col[((size_t)j * 3 + 1) * n] = rgb[1];
                col[((size_t)j * 3 + 2) * n] = rgb[2];
                wt[(size_t)j * n] = w;
                idx[(size_t)j * n] = t;
                wslot[(size_t)j * n] = kn;
            }
        }
        *wsum = 0.0f;
        *cnt = *cnt + 1u;
        return;
    }
    if (o->prm.bias_mode == FWRS_ORACLE_BIAS_FULL) {
        /* Eq. 7 per slot: the slot's own w_sum, biased by its colour difference
         * to the new pixel and by the survival probability; then Alg. 2. */
        uint32_t key[2] = {o->prm.seed, o->prm.stream_id};
        uint32_t words[4];
        int have_block = -1;
        for (int j = 0; j < k; ++j) {
            int b = j / 4;
            if (b != have_block) {
                uint32_t ctr[4] = {p, t, (uint32_t)b, 0u};
                fwrs_oracle_philox(key, ctr, words);
                have_block = b;
            }
            float kept[3] = {col[((size_t)j * 3 + 0) * n], col[((size_t)j * 3 + 1) * n],
                             col[((size_t)j * 3 + 2) * n]};
            float dl = fwrs_oracle_delta_l(kept, rgb);
            float W1 = wslot[(size_t)j * n];
            float total = W1 + w;
            float q = w / total;
            float survive = 1.0f - q;
            float W1b = (W1 * (1.0f - dl)) * survive;   /* Eq. 7 */
            float s = W1b + w;
            float u = (float)((words[j % 4] >> 8) + 1u) * 0x1p-24f;
            if (u * s > W1b) {
                col[((size_t)j * 3 + 0) * n] = rgb[0];
                col[((size_t)j * 3 + 1) * n] = rgb[1];
                col[((size_t)j * 3 + 2) * n] = rgb[2];
                wt[(size_t)j * n] = w;
                idx[(size_t)j * n] = t;
            }
            wslot[(size_t)j * n] = s;
        }
        *wsum = 0.0f;
        *cnt = *cnt + 1u;
        return;
    }
    float W1 = *wsum;
    float W1b = W1;
    if (o->prm.bias_mode == FWRS_ORACLE_BIAS_BERNOULLI) {
        float total = W1 + w;          /* R1.w_sum + R2.w_sum */
        float q = w / total;           /* chance that R2 replaces R1, Eq. 5 */
        float survive = 1.0f - q;      /* Eq. 5 */
        W1b = W1 * survive;            /* Eq. 6 */
    } else if (o->prm.bias_mode == FWRS_ORACLE_BIAS_MEMORYLESS) {
        W1b = W1 * o->decay;           /* every past weight times exp(-lambda) */
    }
    float s = W1b + w;                 /* Alg. 2: R_out.w_sum */

    uint32_t key[2] = {o->prm.seed, o->prm.stream_id};
    uint32_t words[4];
    int have_block = -1;
    for (int j = 0; j < k; ++j) {
        int b = j / 4;
        if (b != have_block) {
            uint32_t ctr[4] = {p, t, (uint32_t)b, 0u};
            fwrs_oracle_philox(key, ctr, words);
            have_block = b;
        }
        float u = (float)((words[j % 4] >> 8) + 1u) * 0x1p-24f;   /* rand in (0, 1] */
        /* Alg. 2 keeps R1 when rand * (W1 + W2) <= W1; otherwise R2 wins. */
        if (u * s > W1b) {
            col[((size_t)j * 3 + 0) * n] = rgb[0];
            col[((size_t)j * 3 + 1) * n] = rgb[1];
            col[((size_t)j * 3 + 2) * n] = rgb[2];
            wt[(size_t)j * n] = w;
            idx[(size_t)j * n] = t;
        }
    }
    *wsum = s;
    *cnt = *cnt + 1u;
}

/* Rows y0 <= y < y1 of one frame; the frame index does not advance.  Lets a
 * test follow a band of a large image without updating the rest. */
void fwrs_oracle_push_rows(fwrs_oracle* o, const float* color, const uint8_t* level, float gx, float gy, int y0,
                           int y1)
{
    const size_t n = (size_t)o->width * (size_t)o->height;
    for (int y = y0; y < y1 && y < o->height; ++y) {
        for (int x = 0; x < o->width; ++x) {
            size_t p = (size_t)y * (size_t)o->width + (size_t)x;
            update_pixel(o, x, y, (uint32_t)p, o->t, color + 3 * p, level[p], gx, gy,
                         o->wsum + p, o->cnt + p, o->wt + p, o->idx + p, o->col + p,
                         o->wslot ? o->wslot + p : NULL, n);
        }
    }
}

void fwrs_oracle_advance(fwrs_oracle* o) { o->t += 1u; }

void fwrs_oracle_push(fwrs_oracle* o, const float* color, const uint8_t* level, float gx, float gy)
{
    const size_t n = (size_t)o->width * (size_t)o->height;
    for (int y = 0; y < o->height; ++y) {
        for (int x = 0; x < o->width; ++x) {
            size_t p = (size_t)y * (size_t)o->width + (size_t)x;
            update_pixel(o, x, y, (uint32_t)p, o->t, color + 3 * p, level[p], gx, gy,
                         o->wsum + p, o->cnt + p, o->wt + p, o->idx + p, o->col + p,
                         o->wslot ? o->wslot + p : NULL, n);
        }
    }
    o->t += 1u;
}

/* ------------------------------------------------------------------------ */
/* One frame with camera or object motion (Sec. 4.3).  Reverse reprojection:  */
/* every pixel looks up where its surface point was in the previous frame     */
/* (its centre minus its motion vector) and continues the reservoir of the    */
/* pixel containing that point.  A point outside the previous image, or one   */
/* whose stored depth disagrees with the current depth (the point was hidden  */
/* or has just become visible), has no usable history: the reservoir is       */
/* flushed to the empty state, and the frame's candidate then fills it, so    */
/* the pixel falls back to plain foveated rendering (Sec. 6).  The frame's    */
/* update (Eq. 4, the bias, Alg. 2 per slot) follows as in oracle push.       */
/* Returns 0, or 1 if memory for the new state cannot be allocated.          */
/* ------------------------------------------------------------------------ */
int fwrs_oracle_push_reproject(fwrs_oracle* o, const float* color, const uint8_t* level, const float* motion,
                               const float* depth, float gx, float gy, float depth_tol)
{
    const int W = o->width, H = o->height, k = o->k;
    const size_t n = (size_t)W * (size_t)H;
    float* wsum = (float*)malloc(n * sizeof(float));
    uint32_t* cnt = (uint32_t*)malloc(n * sizeof(uint32_t));
    float* wt = (float*)malloc(n * (size_t)k * sizeof(float));
    uint32_t* idx = (uint32_t*)malloc(n * (size_t)k * sizeof(uint32_t));
    float* col = (float*)malloc(n * (size_t)k * 3 * sizeof(float));
    float* wslot = o->wslot ? (float*)malloc(n * (size_t)k * sizeof(float)) : NULL;
    float* dnew = (float*)malloc(n * sizeof(float));
    if (!wsum || !cnt || !wt || !idx || !col || !dnew || (o->wslot && !wslot)) {
        free(wsum); free(cnt); free(wt); free(idx); free(col); free(wslot); free(dnew);
        return 1;
    }
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * (size_t)W + (size_t)x;
            /* where this pixel's centre was in the previous frame */
            const float sx = ((float)x + 0.5f) - motion[2 * p + 0];
            const float sy = ((float)y + 0.5f) - motion[2 * p + 1];
            int keep = 0;
            size_t q = 0;
            if (sx >= 0.0f && sx < (float)W && sy >= 0.0f && sy < (float)H) {
                const int qx = (int)floorf(sx);
                const int qy = (int)floorf(sy);
                q = (size_t)qy * (size_t)W + (size_t)qx;
                const float dc = depth[p];
                const float dp = o->depth[q];
                /* the same surface within the tolerance; NaN compares false */
                if (fabsf(dc - dp) <= depth_tol * dc) keep = 1;
            }
            if (keep) {
                wsum[p] = o->wsum[q];
                cnt[p] = o->cnt[q];
                for (int j = 0; j < k; ++j) {
                    wt[(size_t)j * n + p] = o->wt[(size_t)j * n + q];
                    idx[(size_t)j * n + p] = o->idx[(size_t)j * n + q];
                    for (int c = 0; c < 3; ++c)
                        col[((size_t)j * 3 + c) * n + p] = o->col[((size_t)j * 3 + c) * n + q];
                    if (wslot) wslot[(size_t)j * n + p] = o->wslot[(size_t)j * n + q];
                }
            } else {
                /* flush: the empty reservoir */
                wsum[p] = 0.0f;
                cnt[p] = 0u;
                for (int j = 0; j < k; ++j) {
                    wt[(size_t)j * n + p] = 0.0f;
                    idx[(size_t)j * n + p] = 0xFFFFFFFFu;
                    for (int c = 0; c < 3; ++c) col[((size_t)j * 3 + c) * n + p] = 0.0f;
                    if (wslot) wslot[(size_t)j * n + p] = empty_slot_sum(o);
                }
                o->flushes += 1u;
            }
            dnew[p] = depth[p];
        }
    }
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * (size_t)W + (size_t)x;
            update_pixel(o, x, y, (uint32_t)p, o->t, color + 3 * p, level[p], gx, gy,
                         wsum + p, cnt + p, wt + p, idx + p, col + p, wslot ? wslot + p : NULL, n);
        }
    }
    free(o->wsum); free(o->cnt); free(o->wt); free(o->idx); free(o->col); free(o->wslot); free(o->depth);
    o->wsum = wsum; o->cnt = cnt; o->wt = wt; o->idx = idx; o->col = col; o->wslot = wslot; o->depth = dnew;
    o->t += 1u;
    return 0;
}

void fwrs_oracle_depth(const fwrs_oracle* o, float* depth)
{
    memcpy(depth, o->depth, (size_t)o->width * (size_t)o->height * sizeof(float));
}

uint64_t fwrs_oracle_flushes(const fwrs_oracle* o) { return o->flushes; }

/* Weighted combination of the k slots (the k-slot resolve; at k = 1 it is the
 * paper's output R_out.x).  Binary64 from the stored binary32 values; rows
 * [y0, y1) of `out` ([H][W][3]) only. */
void fwrs_oracle_resolve_rows(const fwrs_oracle* o, double* out, int y0, int y1)
{
    const size_t n = (size_t)o->width * (size_t)o->height;
    if (y0 < 0) y0 = 0;
    if (y1 > o->height) y1 = o->height;
    for (size_t p = (size_t)y0 * (size_t)o->width; p < (size_t)(y1 > y0 ? y1 : y0) * (size_t)o->width; ++p) {
        if (o->cnt[p] == 0) {
            out[3 * p + 0] = 0.0; out[3 * p + 1] = 0.0; out[3 * p + 2] = 0.0;
            continue;
        }
        double total = 0.0;
        for (int j = 0; j < o->k; ++j) total += (double)o->wt[(size_t)j * n + p];
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int j = 0; j < o->k; ++j)
                acc += (double)o->wt[(size_t)j * n + p] * (double)o->col[((size_t)j * 3 + c) * n + p];
            out[3 * p + c] = acc / total;
        }
    }
}

void fwrs_oracle_resolve(const fwrs_oracle* o, double* out) { fwrs_oracle_resolve_rows(o, out, 0, o->height); }

/* ------------------------------------------------------------------------ */
/* Accessors and vector helpers for the tests.                                */
/* ------------------------------------------------------------------------ */
uint32_t fwrs_oracle_frame_index(const fwrs_oracle* o) { return o->t; }

/* Per-slot w_sum [k][N]: BIAS_FULL's own sums, else the shared w_sum k times. */
void fwrs_oracle_slot_sums(const fwrs_oracle* o, float* wslot)
{
    const size_t n = (size_t)o->width * (size_t)o->height;
    for (int j = 0; j < o->k; ++j)
        memcpy(wslot + (size_t)j * n, o->wslot ? o->wslot + (size_t)j * n : o->wsum, n * sizeof(float));
}

void fwrs_oracle_constants(const fwrs_oracle* o, float out[9])
{
    out[0] = o->A; out[1] = o->B; out[2] = o->IR2; out[3] = o->IRM; out[4] = o->C;
    out[5] = o->ppd; out[6] = o->iPPD; out[7] = o->rf; out[8] = o->Drf;
}

void fwrs_oracle_state(const fwrs_oracle* o, float* wsum, uint32_t* cnt, float* wt, uint32_t* idx, float* col)
{
    const size_t n = (size_t)o->width * (size_t)o->height;
    const size_t k = (size_t)o->k;
    if (wsum) memcpy(wsum, o->wsum, n * sizeof(float));
    if (cnt) memcpy(cnt, o->cnt, n * sizeof(uint32_t));
    if (wt) memcpy(wt, o->wt, n * k * sizeof(float));
    if (idx) memcpy(idx, o->idx, n * k * sizeof(uint32_t));
    if (col) memcpy(col, o->col, n * k * 3 * sizeof(float));
}

void fwrs_oracle_philox_many(const uint32_t* keys, const uint32_t* ctrs, uint32_t* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) fwrs_oracle_philox(keys + 2 * i, ctrs + 4 * i, out + 4 * i);
}

void fwrs_oracle_cbrt_many(const float* t, float* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) out[i] = fwrs_oracle_cbrt(t[i]);
}

void fwrs_oracle_lab_many(const float* rgb, float* lab, size_t count)
{
    for (size_t i = 0; i < count; ++i) fwrs_oracle_lab(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], lab + 3 * i);
}

void fwrs_oracle_de94_many(const float* ref, const float* x, float* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) out[i] = fwrs_oracle_de94(ref + 3 * i, x + 3 * i);
}

void fwrs_oracle_log2u_many(const uint32_t* bits, float* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) out[i] = fwrs_oracle_log2u(bits[i]);
}

void fwrs_oracle_exp2p_many(const float* y, float* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) out[i] = fwrs_oracle_exp2p(y[i]);
}

void fwrs_oracle_density_many(const fwrs_oracle* o, const float* e, float* out, size_t count)
{
    for (size_t i = 0; i < count; ++i) out[i] = fwrs_oracle_density(o, e[i]);
}

void fwrs_oracle_weight_image(const fwrs_oracle* o, const uint8_t* level, float gx, float gy, float* out)
{
    for (int y = 0; y < o->height; ++y)
        for (int x = 0; x < o->width; ++x) {
            size_t p = (size_t)y * (size_t)o->width + (size_t)x;
            out[p] = fwrs_oracle_weight(o, x, y, level[p], gx, gy);
        }
}

/* Many independent runs of the single stream at pixel (px, py) of a
 * width x height context, differing only in the Philox seed (seed0 + trial).
 * Frame f supplies colour rgb[3f..3f+2], level lev[f] and gaze gaze[2f..2f+1].
 * Writes the final frame index of every slot to idx_out[trial * k + j] and the
 * final w_sum to wsum_out[trial] (if not NULL). */
int fwrs_oracle_trials(int width, int height, int k, const fwrs_oracle_params* p, int px, int py,
                       uint32_t seed0, int n_trials, int n_frames, const float* rgb, const uint8_t* lev,
                       const float* gaze, uint32_t* idx_out, float* wsum_out)
{
    if (px < 0 || py < 0 || px >= width || py >= height) return 1;
    fwrs_oracle* o = fwrs_oracle_create(1, 1, k, p);   /* scratch holder for one pixel's state */
    if (!o) return 2;
    /* The per-pixel math uses the full context's geometry. */
    o->width = width;
    o->height = height;
    derive_constants(o);
    const uint32_t pix = (uint32_t)((size_t)py * (size_t)width + (size_t)px);
    for (int trial = 0; trial < n_trials; ++trial) {
        o->prm.seed = seed0 + (uint32_t)trial;
        o->wsum[0] = 0.0f;
        o->cnt[0] = 0u;
        for (int j = 0; j < k; ++j) {
            if (o->wslot) o->wslot[j] = empty_slot_sum(o);
            o->wt[j] = 0.0f;
            o->idx[j] = 0xFFFFFFFFu;
            o->col[3 * j + 0] = o->col[3 * j + 1] = o->col[3 * j + 2] = 0.0f;
        }
        for (int f = 0; f < n_frames; ++f)
            update_pixel(o, px, py, pix, (uint32_t)f, rgb + 3 * f, lev[f], gaze[2 * f], gaze[2 * f + 1],
                         o->wsum, o->cnt, o->wt, o->idx, o->col, o->wslot, 1);
        for (int j = 0; j < k; ++j) idx_out[(size_t)trial * (size_t)k + (size_t)j] = o->idx[j];
        if (wsum_out) wsum_out[trial] = o->wslot ? o->wslot[0] : o->wsum[0];
    }
    o->width = 1;
    o->height = 1;
    fwrs_oracle_destroy(o);
    return 0;
}
