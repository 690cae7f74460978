// Device building blocks of the prior-predictive sampler (gfx950):
// counter-based random streams, prior draws and the per-draw simulators.
// One lane owns one draw; all model state lives in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pps_internal.hpp"

namespace pps {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the two Philox multipliers, swaps the halves and
// xors in the key; the key advances by the Weyl increments between rounds.
// The key is the seed and is wave-uniform, so its schedule lives in SGPRs.
// Each widening product is written as one 64-bit multiply, which gfx950
// issues as a single v_mad_u64_u32 (both halves at once; measured 18 % faster
// for the whole simulation than separate v_mul_hi_u32 / v_mul_lo_u32).  The
// three-way xors of rounds 1..9 (all operands per lane but the key) are one
// gfx950 v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c); round 0, whose
// counter words 1 and 3 are often wave-uniform, is left to the compiler.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        if (r == 0) {
            c0 = hi1 ^ c1 ^ k0;
            c2 = hi0 ^ c3 ^ k1;
        } else {
            c0 = xor3(hi1, c1, k0);
            c2 = xor3(hi0, c3, k1);
        }
        c1 = lo1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Stream purposes: prior draws, the path of a one-lane model, and cell c of a
// multi-cell model (the toggle switch) as PURPOSE_CELL0 + c.
enum : uint32_t {
    PURPOSE_PRIOR = 0,
    PURPOSE_PATH = 1,
    PURPOSE_CELL0 = 2,
    PURPOSE_TB_EVENT = 0x90000000u,   // tuberculosis: event e uses block e/2
    PURPOSE_TB_SAMPLE = 0x90000001u,  // tuberculosis: sampled case s uses block s/4
};

struct StreamKey {
    uint32_t k0, k1;  // (lo32 seed, hi32 seed)
};

__device__ __forceinline__ StreamKey make_key(uint64_t seed)
{
    return {static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
}

__device__ __forceinline__ Words4 stream_block(StreamKey key, uint64_t draw, uint32_t block,
                                               uint32_t purpose)
{
    return philox4x32_10(block, purpose, static_cast<uint32_t>(draw),
                         static_cast<uint32_t>(draw >> 32), key.k0, key.k1);
}

// ---------------------------------------------------------------------------
// Uniforms on the open unit interval: the top 23 bits pick the cell midpoint
// (2k+1) 2^-24; exact in FP32 and FP64.
// ---------------------------------------------------------------------------
// Two instruction sequences give the same value.  FUNNEL: 0x3F800000 | (w >>
// 9) is 1 + k 2^-23, k = w >> 9 (one funnel shift of the pair 0x7F:w by 9
// bits), and subtracting 1 - 2^-24 leaves (2k+1) 2^-24 exactly (the operands
// lie within a factor 2 of each other): two instructions.  Otherwise shift,
// convert and FMA: three, which the GARCH kernel's schedule has run faster.
template <bool FUNNEL = true>
__device__ __forceinline__ float uniform_f32(uint32_t w)
{
    if constexpr (FUNNEL) {
        const uint32_t one_k = __builtin_amdgcn_alignbit(0x7Fu, w, 9u);
        return __builtin_bit_cast(float, one_k) - 0x1.fffffep-1f;
    } else {
        return __builtin_fmaf(static_cast<float>(w >> 9), 0x1p-23f, 0x1p-24f);
    }
}

__device__ __forceinline__ double uniform_f64(uint32_t w)
{
    return static_cast<double>(w >> 9) * 0x1p-23 + 0x1p-24;
}

// FP64 Box-Muller (prior draws only: once per parameter per draw);
// cos(2 pi u1) is evaluated as cospi(2 u1), which needs no range reduction.
__device__ __forceinline__ double box_muller_f64_first(uint32_t w0, uint32_t w1)
{
    const double u0 = uniform_f64(w0);
    const double u1 = uniform_f64(w1);
    return sqrt(-2.0 * log(u0)) * cospi(2.0 * u1);
}

// Box-Muller in FP32 with the hardware transcendentals: v_log_f32 is log2,
// v_sin_f32 / v_cos_f32 take their argument in revolutions (x -> sin(2 pi x)),
// so the angle 2 pi u1 needs no range reduction.
// The six normals z_{6b..6b+5} of stream block b = (x, y, z, w): three
// Box-Muller pairs.  Pair i takes its radius uniform from word i (x, y, z)
// as uniform_f32 does (top 23 bits) and its angle from 19 more bits, the low
// 9 bits of word i followed by bits [22 - 10i, 32 - 10i) of w, as u1 = m
// 2^-19 (2^19 equally spaced angles from 0); the 126 bits used are disjoint,
// so one Philox call serves six normals.  The angle is built in place: a
// funnel shift of (word i : w << 10i) by 18 bits puts the 9 bits at [14, 23)
// and the 10 bits of w at [4, 14), and one and-or with the bits of 1.0 (an
// inline constant) gives 1 + u1 exactly; v_sin / v_cos are periodic in
// revolutions, so 1 + u1 is used as it is.
constexpr int NORMALS_PER_BLOCK = 6;

template <bool FUNNEL = true>
__device__ __forceinline__ void normals6(const Words4 &w, float (&z)[NORMALS_PER_BLOCK])
{
    const uint32_t rw[3] = {w.x, w.y, w.z};
    const uint32_t sw[3] = {w.w, w.w << 10, w.w << 20};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float u0 = uniform_f32<FUNNEL>(rw[i]);
        const uint32_t t = __builtin_amdgcn_alignbit(rw[i], sw[i], 18u);
        const float a1 = __builtin_bit_cast(float, (t & 0x007FFFF0u) | 0x3F800000u);  // 1 + u1
        // -2 ln u0 = log2(u0) * (-2 ln 2)
        const float r = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(u0) * -1.38629436111989061883f);
        z[2 * i] = r * __builtin_amdgcn_cosf(a1);
        z[2 * i + 1] = r * __builtin_amdgcn_sinf(a1);
    }
}

// Normals z_{6b..6b+5} of a draw's path.
template <bool FUNNEL = true>
__device__ __forceinline__ void path_normals6(StreamKey key, uint64_t draw, uint32_t block,
                                              float (&z)[NORMALS_PER_BLOCK])
{
    normals6<FUNNEL>(stream_block(key, draw, block, PURPOSE_PATH), z);
}

// Normals z_{6b..6b+5} of cell `cell` of a draw.
__device__ __forceinline__ void cell_normals6(StreamKey key, uint64_t draw, uint32_t cell,
                                              uint32_t block, float (&z)[NORMALS_PER_BLOCK])
{
    normals6(stream_block(key, draw, block, PURPOSE_CELL0 + cell), z);
}

// ---------------------------------------------------------------------------
// Prior draws (FP64).  Parameter j of attempt t uses PRIOR block 8t + j:
// uniform from word 0, normal / log-normal from words (0, 1).  The uniform
// transform is written with explicit round-to-nearest operations so that the
// GARCH constraint is decided exactly as an unfused IEEE evaluation.
// Kept out of line: the FP64 log / cospi / exp would otherwise set the
// register budget of the whole simulation loop (117 vs 58 VGPRs).
// ---------------------------------------------------------------------------
// The value of a prior from its attempt's variates: u = uniform of word 0,
// z = the first FP64 Box-Muller normal of words (0, 1).
__device__ __forceinline__ double prior_transform(const PriorDev &p, double u, double z)
{
    if (p.family == PPS_POINT)
        return p.a;
    if (p.family == PPS_UNIFORM)
        return __dadd_rn(p.a, __dmul_rn(__dsub_rn(p.b, p.a), u));
    const double v = __dadd_rn(p.a, __dmul_rn(p.b, z));
    return p.family == PPS_LOGNORMAL ? exp(v) : v;
}

__device__ __attribute__((noinline)) double prior_value(const PriorDev &p, StreamKey key, uint64_t draw,
                                              int j, int attempt)
{
    if (p.family == PPS_POINT)
        return p.a;
    const Words4 w = stream_block(key, draw, static_cast<uint32_t>(8 * attempt + j), PURPOSE_PRIOR);
    const double u = uniform_f64(w.x);
    if (p.family == PPS_UNIFORM)
        return prior_transform(p, u, 0.0);
    return prior_transform(p, u, box_muller_f64_first(w.x, w.y));
}

// The variates u and z of parameter j, attempt 0 (the lambda-group kernel
// applies every member's prior to one set).
__device__ __attribute__((noinline)) void prior_variates(StreamKey key, uint64_t draw, int j,
                                                         double &u, double &z)
{
    const Words4 w = stream_block(key, draw, static_cast<uint32_t>(j), PURPOSE_PRIOR);
    u = uniform_f64(w.x);
    z = box_muller_f64_first(w.x, w.y);
}

constexpr int MAX_PRIOR_ATTEMPTS = 32;

// theta ~ pi(theta); with the GARCH constraint, attempts whose
// theta[1] + theta[2] >= 1 are redrawn, with the tuberculosis constraint
// those with theta[0] <= theta[1] or theta[2] <= 0 (the last attempt is kept
// after 32).
// MAXP is the size of `theta` (the parameters a kernel holds in registers).
template <int MAXP>
__device__ __forceinline__ void prior_draw(const PriorDev *prior, int n_params, int constraint,
                                           StreamKey key, uint64_t draw, double *theta)
{
    for (int attempt = 0;; ++attempt) {
#pragma unroll
        for (int j = 0; j < MAXP; ++j)
            if (j < n_params)
                theta[j] = prior_value(prior[j], key, draw, j, attempt);
        if (constraint == PPS_GARCH_STATIONARY) {
            if (__dadd_rn(theta[1], theta[2]) < 1.0 || attempt + 1 == MAX_PRIOR_ATTEMPTS)
                return;
        } else if (constraint == PPS_TB_SUPERCRITICAL) {
            if ((theta[0] > theta[1] && theta[2] > 0.0) || attempt + 1 == MAX_PRIOR_ATTEMPTS)
                return;
        } else {
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Compensated (Kahan) FP32 accumulation: sum = s - c.
// ---------------------------------------------------------------------------
struct Kahan {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const
    {
        return static_cast<double>(s) - static_cast<double>(c);
    }
};

}  // namespace pps
