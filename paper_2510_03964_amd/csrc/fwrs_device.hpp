// Device-side building blocks of the weighted-reservoir-sampling pass for
// gfx950: the per-frame descriptor, the method constants, Philox4x32-10, the
// base-2 exponential, the Eq. 3-4 weight and the Eq. 5-6 bias.
//
// Every binary32 operation here is written out in the order the method fixes
// and the library is built with -ffp-contract=off and correctly rounded
// division and square root, so the weight, the biased w_sum and the keep /
// replace decisions are reproducible bit for bit on any IEEE binary32 target
// (the same functions run on the host to derive the per-context constants).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fwrs {

// Method constants derived once per context from its parameters (Sec. 4.1).
struct Consts {
    float A;     // a_k
    float B;     // 1 - a_k
    float IR2;   // 1 / r_2,k
    float IRM;   // 1 / r_m
    float C;     // log2(e) / r_e,k: exp(-e / r_e,k) = 2^(-e C)
    float iPPD;  // degrees per pixel = fov_deg / width (as 1 / (width / fov_deg))
    float rf;    // foveal radius in degrees = fovea_radius_px / ppd
    float Drf;   // density at r_f (normalisation of Eq. 4)
    float decay; // exp(-lambda): the memory-less bias factor per frame
};

// Everything one frame of one context needs on the device.  Passed by value
// to the single-frame kernels and stored in a device table for batched ticks
// (where `first` is the tick's first work item of the frame).  In a batched
// tick the consecutive frames of one context form a group: the table holds the
// group's first frame (the leader, which owns the work items) among the other
// leaders and its nf - 1 later frames after all the leaders, from index `more`
// on; each pixel then runs all nf frames in order.
struct alignas(8) FrameDesc {
    const float* color;         // [H][W][3] f32, the new candidates
    const uint8_t* level;       // [H][W] u8 foveation level
    float* out;                 // [H][W][3] f32 resolve target (null for update-only)
    float* wsum;                // [N] w_sum per pixel; [N][k] per slot under Eq. 7
    float* rec;                 // [N][k][4] slot records {w, r, g, b}
    uint32_t* idx;              // [N][k] frame index of each slot's sample
    float* res;                 // [N][3] each pixel's resolve as of its last change (resolve plane), or null
    unsigned long long* stats;  // [kStatSlots][3] counters (slots replaced, pixels changed, flushed), or null
    uint32_t width, height, t, k;
    float gx, gy;
    Consts c;
    uint32_t seed, stream_id, bias;
    uint32_t op;                // what the batched kernel runs for this frame (an Op of the kernels)
    uint32_t tile_x_log2, tile_y_log2, tiles_x, items;  // launch geometry
    uint32_t first;             // batched ticks: the frame's first work item in the tick
    uint32_t rev;               // batched ticks: the frame's items are visited last first
    uint32_t nf;                // batched ticks, leaders: frames in the group (1: the frame alone)
    uint32_t more;              // batched ticks, leaders: table index of the group's second frame
    uint32_t res_ok;            // the resolve plane holds every pixel's resolve before this frame
    uint32_t pad_;
};

// Reprojected frame (Sec. 4.3): the reservoirs are gathered from the previous
// bank at each pixel's motion-compensated source and written densely to the
// other bank (f's wsum / rec / idx), with the pixel counts and depths.
struct alignas(8) ReprojDesc {
    FrameDesc f;
    const float* motion;        // [H][W][2] f32 pixels, current minus previous position
    const float* depth;         // [H][W] f32 current depth (> 0)
    const float* src_wsum;      // previous bank (layout as f's)
    const float* src_rec;
    const uint32_t* src_idx;
    const uint32_t* src_cnt;    // [N] candidates seen (Alg. 2's m)
    const float* src_depth;     // [N] depth of the previous frame (NaN: none)
    uint32_t* cnt;              // this frame's bank
    float* depth_out;
    float tol;                  // relative depth tolerance
};

// Foveation generator sources (Sec. 4.3): the full frame and the reduced
// levels -- mip 1 and mip 2 (bilinear sampling), or one plane holding at every
// pixel of level l >= 1 the frame blurred with sigma 2^(l-1) px (sampled at the
// pixel; level-0 pixels are not written) -- and the rings that pick a level.
constexpr uint32_t kFovMip = 0u;
constexpr uint32_t kFovGauss = 1u;
struct FovSrc {
    const float* full;          // [H][W][3]
    const float* l1;            // mip 1 [h1][w1][3], or the Gaussian plane [H][W][3]
    const float* l2;            // mip 2 [h2][w2][3] (Gaussian: unused)
    uint32_t w1, h1, w2, h2;
    float r0sq, r1sq;           // squared ring radii (level 0 within r0, 1 within r1)
    uint32_t mode;              // kFovMip / kFovGauss
};

struct alignas(8) FovDesc {
    FrameDesc f;
    FovSrc s;
};

constexpr int kBlock = 256;             // threads per block
constexpr int kStatSlots = 1024;        // spread of the slot-take counters
constexpr uint32_t kBiasNone = 0u;
constexpr uint32_t kBiasBernoulli = 1u;
constexpr uint32_t kBiasFull = 2u;      // Eq. 7: per-slot w_sum scaled by (1 - |dL|) and Eq. 6
constexpr uint32_t kBiasMemoryless = 3u;  // w_sum * exp(-lambda) per frame (Sec. 3.1)
constexpr uint32_t kAes = 4u;           // A-ES keys (Sec. 3.1), one per slot, no w_sum

// Modes that keep one value per slot instead of one w_sum per pixel.
__host__ __device__ __forceinline__ bool per_slot_mode(uint32_t mode)
{
    return mode == kBiasFull || mode == kAes;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  Counter (x0..x3),
// key (k0, k1); per round: (hi, lo) of M_A * x0 and M_B * x2, new words
// (hi_B ^ x1 ^ k0, lo_B, hi_A ^ x3 ^ k1, lo_A); the key advances by the Weyl
// constants between rounds.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit multiply per product (v_mad_u64_u32) gives both halves
        const uint64_t pa = (uint64_t)kPhiloxMulA * (uint64_t)x0;
        const uint64_t pb = (uint64_t)kPhiloxMulB * (uint64_t)x2;
        const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        const uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        x0 = hi_b ^ x1 ^ k0;
        x1 = lo_b;
        x2 = hi_a ^ x3 ^ k1;
        x3 = lo_a;
        k0 += kPhiloxWeylA;
        k1 += kPhiloxWeylB;
    }
    return make_uint4(x0, x1, x2, x3);
}

// Variate in (0, 1] from the top 24 bits of a Philox word.
__device__ __forceinline__ float unit_variate(uint32_t word)
{
    return (float)((word >> 8) + 1u) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// 2^y for y <= 0: y = n + f, n = rint(y), |f| <= 1/2 (exact), degree-7 Taylor
// polynomial of 2^f = exp(f ln 2) in Horner form, scaled by 2^n.  The
// coefficients are the binary32 roundings of (ln 2)^i / i!.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ float exp2_neg(float y)
{
    const float n = rintf(y);
    const float f = y - n;
    float p = 0x1.ffcbfcp-17f;        // (ln 2)^7 / 7!
    p = p * f; p = p + 0x1.430912p-13f;   // (ln 2)^6 / 6!
    p = p * f; p = p + 0x1.5d87fep-10f;   // (ln 2)^5 / 5!
    p = p * f; p = p + 0x1.3b2ab6p-7f;    // (ln 2)^4 / 4!
    p = p * f; p = p + 0x1.c6b08ep-5f;    // (ln 2)^3 / 3!
    p = p * f; p = p + 0x1.ebfbe0p-3f;    // (ln 2)^2 / 2!
    p = p * f; p = p + 0x1.62e430p-1f;    // ln 2
    p = p * f; p = p + 1.0f;
    return ldexpf(p, (int)n);
}

// Eq. 3 multiplied through by (1 + e / r_2,k)^2, without the 2 d_c(0) factor
// that cancels in Eq. 4:  d(e) ~ num / den with
//   num = a_k + (1 - a_k) exp(-e / r_e,k) (1 + e / r_2,k)^2,
//   den = (1 + e / r_2,k)^2 (1 + e / r_m).
__host__ __device__ __forceinline__ void density_terms(const Consts& c, float e, float& num, float& den)
{
    const float t1 = 1.0f + e * c.IRM;
    const float t2 = 1.0f + e * c.IR2;
    const float T = t2 * t2;
    const float E = exp2_neg(-(e * c.C));
    num = c.A + (c.B * E) * T;
    den = T * t1;
}

// Eq. 4 for a pixel whose centre lies `dist2` squared pixels from the gaze,
// in two parts so that the arithmetic can run before the level is loaded:
// outside(...) is d(e) / d(r_f) (clamped to 1) and sets the eccentricity e;
// select_eq4(...) scores level 0 (full fidelity this frame) and e <= r_f as 1.
__device__ __forceinline__ float weight_outside(const Consts& c, float dist2, float& e)
{
    e = sqrtf(dist2) * c.iPPD;
    float num, den;
    density_terms(c, e, num, den);
    return fminf(1.0f, num / (den * c.Drf));
}

__device__ __forceinline__ float select_eq4(const Consts& c, float outside, float e, uint32_t level)
{
    return (level == 0u || e <= c.rf) ? 1.0f : outside;
}

__device__ __forceinline__ float weight_eq4(const Consts& c, float dist2, uint32_t level)
{
    float e;
    const float o = weight_outside(c, dist2, e);
    return select_eq4(c, o, e, level);
}

// The bias of a shared w_sum: Eq. 5-6 scale R1.w_sum by the survival
// probability 1 - w / (R1.w_sum + w) (BERNOULLI); the memory-less bias by
// exp(-lambda) (MEMORYLESS); NONE leaves it.
__device__ __forceinline__ float bias_shared(float W1, float w, uint32_t mode, float decay)
{
    if (mode == kBiasMemoryless) return W1 * decay;
    const float total = W1 + w;
    const float q = w / total;
    const float survive = 1.0f - q;
    return mode == kBiasBernoulli ? W1 * survive : W1;
}

// log2 of the variate ((bits >> 8) + 1) 2^-24 for A-ES keys, correctly rounded to
// binary32.  m = (bits >> 8) + 1 = 2^e f with f in [sqrt(1/2), sqrt(2)):
// log2 u = (e - 24) + log2 f and log2 f = (2 / ln 2) atanh(s), s = (f - 1) / (f + 1),
// |s| < 0.172, summed as the odd series to s^21 in binary64 (truncation below
// 2^-60 relative); the binary64 value is then rounded once to binary32.  That
// this is the nearest binary32 for every one of the 2^24 variates is checked
// exhaustively on the host.
__host__ __device__ __forceinline__ float log2_unit(uint32_t bits)
{
    const uint32_t m = (bits >> 8) + 1u;
    int e = 31 - __builtin_clz(m);
    double f = ldexp((double)m, -e);                 // exact, [1, 2)
    if (f >= 1.4142135623730951) {
        f = f * 0.5;
        e = e + 1;
    }
    const double s = (f - 1.0) / (f + 1.0);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    const double two_over_ln2 = 2.8853900817779268;   // 2 / ln 2
    return (float)((double)(e - 24) + (two_over_ln2 * s) * p);
}

// ---------------------------------------------------------------------------
// Foveation: the level ring of a pixel and its degraded colour.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ring_level(float r0sq, float r1sq, float gx, float gy, uint32_t x, uint32_t y)
{
    const float dx = ((float)x + 0.5f) - gx;
    const float dy = ((float)y + 0.5f) - gy;
    const float d2 = dx * dx + dy * dy;
    return d2 <= r0sq ? 0u : (d2 <= r1sq ? 1u : 2u);
}

__device__ __forceinline__ uint32_t fov_level(const FovSrc& s, float gx, float gy, uint32_t x, uint32_t y)
{
    return ring_level(s.r0sq, s.r1sq, gx, gy, x, y);
}

// Bilinear sample of a w x h level (1/scale of full resolution) at the centre
// of full-resolution pixel (x, y): texel centres at (i + 0.5) scale, clamp to
// edge, interpolation a + f (b - a) along x, then along y.
__device__ __forceinline__ float3 bilinear(const float* lv, uint32_t w, uint32_t h, uint32_t x, uint32_t y,
                                           float inv_scale)
{
    const float u = ((float)x + 0.5f) * inv_scale - 0.5f;
    const float v = ((float)y + 0.5f) * inv_scale - 0.5f;
    const float fu = floorf(u), fv = floorf(v);
    const float fx = u - fu, fy = v - fv;
    const int iw = (int)w - 1, ih = (int)h - 1;
    const int i0 = min(max((int)fu, 0), iw), j0 = min(max((int)fv, 0), ih);
    const int i1 = min((int)fu + 1, iw), j1 = min((int)fv + 1, ih);
    const float* r0 = lv + (size_t)j0 * w * 3;
    const float* r1 = lv + (size_t)j1 * w * 3;
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float t00 = r0[3 * i0 + c], t10 = r0[3 * i1 + c];
        const float t01 = r1[3 * i0 + c], t11 = r1[3 * i1 + c];
        const float top = t00 + fx * (t10 - t00);
        const float bot = t01 + fx * (t11 - t01);
        out[c] = top + fy * (bot - top);
    }
    return make_float3(out[0], out[1], out[2]);
}

__device__ __forceinline__ float3 fov_colour(const FovSrc& s, uint32_t x, uint32_t y, uint32_t p, uint32_t level)
{
    const float* src = level == 0u ? s.full : s.l1;
    if (level == 0u || s.mode == kFovGauss) {
        const float* c = src + 3 * (size_t)p;
        return make_float3(c[0], c[1], c[2]);
    }
    return level == 1u ? bilinear(s.l1, s.w1, s.h1, x, y, 0.5f) : bilinear(s.l2, s.w2, s.h2, x, y, 0.25f);
}

// ---------------------------------------------------------------------------
// Eq. 7's colour difference: both colours (linear RGB, sRGB primaries) to CIE
// Lab (D65 white), then the CIE94 difference with graphic-arts weights and the
// reservoir sample as the reference; |dL| = min(1, dE94 / 100).
// ---------------------------------------------------------------------------
// Cube root of t, correctly rounded to binary32 (t > 0 normal; zero, +inf and
// NaN pass through).
//
// The estimate y0 = 2^(log2(t) / 3) comes from the device's base-2 logarithm
// and exponential instructions (libm's on the host) and is within about 2^-19
// of the cube root.  One Newton step in binary64 follows:
// y1 = y0 + (t - y0^3) / (3 y0^2), with y0^2 exact, and the division taken as a
// product with the binary32 reciprocal of 3 y0^2.  y1 is within about 2^-36 of
// the cube root, so rounding it to binary32 gives the nearest binary32, unless
// y1 lies within kCbrtGuard (2^-34 relative) of a midpoint between two
// binary32 values.
//
// Those rare inputs take the exact decision in cube_root_nearest.  There
// y = RN(y1) is within one ulp of the cube root.  The real cube root lies above
// the midpoint m between y and the binary32 above it iff m^3 < t, and below the
// midpoint under y iff t < m^3.  A midpoint has 25 significant bits, so m^2 is
// exact in binary64 and m^3 is exactly hi + lo, with hi = m^2 m rounded and
// lo = fma(m^2, m, -hi).  hi is within a few ulps of t, so t - hi is exact, and
// t - m^3 has the sign of (t - hi) - lo.
//
// That the result equals the oracle's (the binary32 nearest to the real cube
// root) is checked on every t in [(6/29)^3, 2^8) and on every 61st positive
// normal binary32 beyond: on the GPU for the device code, and on the host for
// the host build.
__host__ __device__ __forceinline__ bool cube_below(double m, double t)     // m^3 < t, exactly
{
    const double m2 = m * m;
    const double hi = m2 * m;
    const double lo = fma(m2, m, -hi);
    return (t - hi) > lo;
}

// The binary32 nearest to t^(1/3), given y within one ulp of it.
__host__ __device__ __forceinline__ float cube_root_nearest(float t, float y)
{
    const uint32_t yb = __builtin_bit_cast(uint32_t, y);
    const float up = __builtin_bit_cast(float, yb + 1u);
    const float dn = __builtin_bit_cast(float, yb - 1u);
    const double td = (double)t;
    if (cube_below(0.5 * ((double)y + (double)up), td)) return up;
    if (!cube_below(0.5 * ((double)dn + (double)y), td)) return dn;
    return y;
}

// Distance from a binary32 midpoint below which the exact decision is taken, in
// units of 2^-52 of the binade (29 bits lie below binary32 precision): 2^-34.
constexpr int32_t kCbrtGuard = 1 << 18;

__host__ __device__ __forceinline__ float cube_root(float t)
{
    if (!(t < INFINITY) || t == 0.0f) return t;     // +inf, NaN, zero
#if defined(__HIP_DEVICE_COMPILE__)
    const float y0 = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(t) * 0x1.555556p-2f);
    const float r3 = __builtin_amdgcn_rcpf(3.0f * (y0 * y0));
#else
    const float y0 = exp2f(log2f(t) * 0x1.555556p-2f);
    const float r3 = 1.0f / (3.0f * (y0 * y0));
#endif
    const double yd = (double)y0;
    const double y1 = yd + ((double)t - (yd * yd) * yd) * (double)r3;
    const float y = (float)y1;
    const int32_t off = (int32_t)((uint32_t)__builtin_bit_cast(uint64_t, y1) & 0x1FFFFFFFu) - 0x10000000;
    if (off > -kCbrtGuard && off < kCbrtGuard) return cube_root_nearest(t, y);
    return y;
}

// x / c for a constant divisor c given rc = RN(1 / c): the product x rc corrected
// by one fused multiply-add of its residual (Markstein's method).  For each of the
// divisors below (0.95047, 1.08883, 100) this equals the correctly rounded x / c for
// every binary32 x with 2^-100 <= |x| <= 2^126 (checked exhaustively); other x
// take the division, so the result is always the correctly rounded quotient.
__host__ __device__ __forceinline__ float div_const(float x, float c, float rc)
{
    const float ax = fabsf(x);
    if (ax >= 0x1p-100f && ax <= 0x1p126f) {
        const float q = x * rc;
        const float r = fmaf(-q, c, x);
        return fmaf(r, rc, q);
    }
    return x / c;
}

__host__ __device__ __forceinline__ float lab_curve(float t)
{
    // t^(1/3) above (6/29)^3, the linear segment t / (3 (6/29)^2) + 4/29 below
    const float lin = t * (841.0f / 108.0f) + 4.0f / 29.0f;
    return t > 216.0f / 24389.0f ? cube_root(t) : lin;
}

__host__ __device__ __forceinline__ float3 rgb_to_lab(float r, float g, float b)
{
    const float X = (0.4124564f * r + 0.3575761f * g) + 0.1804375f * b;
    const float Y = (0.2126729f * r + 0.7151522f * g) + 0.0721750f * b;
    const float Z = (0.0193339f * r + 0.1191920f * g) + 0.9503041f * b;
    const float fx = lab_curve(div_const(X, 0.95047f, 0x1.0d5728p+0f));   // X / X_n
    const float fy = lab_curve(Y);
    const float fz = lab_curve(div_const(Z, 1.08883f, 0x1.d63ac2p-1f));   // Z / Z_n
    return make_float3(116.0f * fy - 16.0f, 500.0f * (fx - fy), 200.0f * (fy - fz));
}

__host__ __device__ __forceinline__ float cie94(const float3& ref, const float3& x)
{
    const float dL = ref.x - x.x;
    const float C1 = sqrtf(ref.y * ref.y + ref.z * ref.z);
    const float C2 = sqrtf(x.y * x.y + x.z * x.z);
    const float dC = C1 - C2;
    const float da = ref.y - x.y;
    const float db = ref.z - x.z;
    const float dH2 = fmaxf((da * da + db * db) - dC * dC, 0.0f);
    const float SC = 1.0f + 0.045f * C1;
    const float SH = 1.0f + 0.015f * C1;
    const float tC = dC / SC;
    return sqrtf((dL * dL + tC * tC) + dH2 / (SH * SH));
}

// A sample whose colour compares equal to the new pixel's, component by
// component, has the same Lab triple: the inputs are the same binary32 values
// up to the sign of a zero, and a zero component leaves the same Lab (a zero
// product adds nothing to a non-zero sum, and a zero X, Y or Z lands on the
// linear segment's 4/29).  CIE94 of a colour with itself is then exactly 0
// (dL, dC, da, db and dH2 are 0, so is the root), and so is |dL|.  This needs
// L* and the chroma finite, which components of magnitude below 2^24 ensure
// (a* and b* stay below 2^40, their squares far from overflow); other colours,
// and NaN, which compares unequal, take the full evaluation.
__host__ __device__ __forceinline__ bool lab_bounded(float c0, float c1, float c2)
{
    return fabsf(c0) < 0x1p24f && fabsf(c1) < 0x1p24f && fabsf(c2) < 0x1p24f;
}

__host__ __device__ __forceinline__ bool same_colour(const float4& s, float c0, float c1, float c2)
{
    return s.y == c0 && s.z == c1 && s.w == c2;
}

// Eq. 7: (W1 (1 - |dL|)) (1 - w / (W1 + w)).
__device__ __forceinline__ float bias_eq7(float W1, float w, float dl)
{
    const float total = W1 + w;
    const float q = w / total;
    const float survive = 1.0f - q;
    return (W1 * (1.0f - dl)) * survive;
}

// |dL| = min(1, dE94 / 100) of a sample of colour (r, g, b) against the new
// pixel, given the new pixel's Lab.
__device__ __forceinline__ float delta_l(float r, float g, float b, const float3& lab_new)
{
    return fminf(1.0f, div_const(cie94(rgb_to_lab(r, g, b), lab_new), 100.0f, 0x1.47ae14p-7f));
}

}  // namespace fwrs
