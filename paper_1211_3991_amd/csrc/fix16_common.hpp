// Device helpers shared by the fixed-point kernels: (cos, sin) of a 16-bit
// angle, the over-relaxation axis, the FP64 unit vector of a measurement and
// the exact Metropolis acceptance.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace xy {
namespace {

constexpr float kTwoPhiScale = 20860.756700940907f;   // 2^16 / pi: 2*phi in angle units
constexpr float kAngle = 9.587379924285257e-05f;      // 2 pi / 2^16

// (cos, sin) of a 16-bit angle in FP32.  The three forms are different
// deterministic functions of the angle (each within a few ulp of the exact
// value); whichever is compiled in defines the energy the sweep samples.
//   0: two-level table, (cos, sin)(256 a) rotated by (cos, sin)(b), 2 x 256 entries
//   1: 2048-entry table of (cos, sin)(32 a), rotated by the small angle of the
//      low 5 bits, delta <= 3.1e-3, with cos = 1 - delta^2/2 and sin = delta
//      (truncation errors 4e-12 and 5e-9)
//   2: the hardware sine/cosine of theta / 2^16 revolutions (no table)
// unit takes a 16-bit angle; unit_lo and unit_hi the angle in the low or the
// high half of a 32-bit word (two slots' angles).
template <int kTrig> struct Trig;

template <int kTrig> struct TrigHalves {
    static __device__ __forceinline__ float2 unit_lo(uint32_t w, const float2 *t) { return Trig<kTrig>::unit(w & 0xFFFFu, t); }
    static __device__ __forceinline__ float2 unit_hi(uint32_t w, const float2 *t) { return Trig<kTrig>::unit(w >> 16, t); }
};

template <> struct Trig<0> : TrigHalves<0> {
    static constexpr size_t kBytes = 512 * 8;
    static __device__ __forceinline__ void load(float2 *t, const DevBatch &b, int tid, int stride)
    {
        for (int k = tid; k < 512; k += stride) t[k] = b.tab32[k];
    }
    static __device__ __forceinline__ float2 unit(uint32_t th, const float2 *t)
    {
        const float2 a = t[th >> 8], c = t[256 + (th & 255u)];
        return make_float2(a.x * c.x - a.y * c.y, a.y * c.x + a.x * c.y);
    }
};

template <> struct Trig<1> : TrigHalves<1> {
    static constexpr size_t kBytes = 2048 * 8;
    static __device__ __forceinline__ void load(float2 *t, const DevBatch &b, int tid, int stride)
    {
        for (int k = tid; k < 2048; k += stride) t[k] = b.tab2k[k];
    }
    static __device__ __forceinline__ float2 unit(uint32_t th, const float2 *t)
    {
        const float2 a = t[th >> 5];
        const float d = (float)(th & 31u) * kAngle;
        const float c = 1.0f - 0.5f * d * d;
        return make_float2(a.x * c - a.y * d, a.y * c + a.x * d);
    }
};

template <> struct Trig<2> {
    static constexpr size_t kBytes = 0;
    static __device__ __forceinline__ void load(float2 *, const DevBatch &, int, int) {}
    // The input is 128 + theta / 2^16 revolutions: the float of exponent 7
    // (ulp 2^-16) whose low 16 mantissa bits are theta, exact and built from
    // the bits in one instruction; sine and cosine see only its fraction
    // theta / 2^16 (the 128 whole turns are invisible to them, and the results
    // equal those for 1 + theta / 2^16 bit for bit).
    static __device__ __forceinline__ float2 at(float r)
    {
        return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
    static __device__ __forceinline__ float2 unit(uint32_t th, const float2 *)
    {
        return at(__uint_as_float(0x43000000u | th));
    }
    // bits of w above the sixteenth are ignored (one v_and_or_b32)
    static __device__ __forceinline__ float2 unit_lo(uint32_t w, const float2 *)
    {
        return at(__uint_as_float(0x43000000u | (w & 0xFFFFu)));
    }
    // (one v_or_b32 with the high half selected by SDWA)
    static __device__ __forceinline__ float2 unit_hi(uint32_t w, const float2 *)
    {
        return at(__uint_as_float(0x43000000u | (w >> 16)));
    }
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96), all operands per lane
__device__ __forceinline__ uint32_t xor3_v(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// 2 phi in units of 2pi/2^16, rounded, for phi = atan2(hy, hx): the axis of
// the over-relaxation reflection, in the low 16 bits of the result (the
// higher bits are not part of it; callers reduce mod 2^16).  atan on [0, 1]
// by an odd polynomial of degree 9, least-squares fitted on 4000 Chebyshev
// nodes (|error| < 1.3e-5 rad in FP32, an eighth of the angle quantum
// 2pi/2^16), of t = min(|hx|, |hy|) / max(|hx|, |hy|) (0 for a zero field).
// The octant is restored on the doubled angle, where it is a sign and a half
// turn: with a = atan(t), phi is +-phi0 or +-(pi - phi0) for phi0 = a, or
// pi/2 - a when |hy| > |hx| ("swapped"), so 2 phi = +-2 phi0 (mod 2 pi), +
// when hx and hy have equal signs; that is 2 phi = sigma 2a, plus pi when
// swapped, where sigma's sign bit is the XOR of those of hx, hy and
// |hx| - |hy| (negative exactly when swapped; the sign of a zero component
// does not matter, as a = 0 then).  The rounding adds 1.5 * 2^23 (+ 2^15 for
// the half turn) in the same fused multiply-add that scales the angle: the
// sum's ulp is 1, so it is the scaled angle rounded to the nearest integer
// (ties to even), and for |x| < 2^22 the float's low mantissa bits hold that
// integer mod 2^16.  The accuracy only affects the acceptance rate of the
// reflection, not the detailed balance (the reflection is accepted by a
// Metropolis test).
__device__ __forceinline__ uint32_t field_axis2(float hx, float hy)
{
    const float ax = fabsf(hx), ay = fabsf(hy);
    // the floor keeps t = 0 for a zero field; the median of (ax, ay, 0) is the
    // smaller magnitude (one v_med3_f32 with the absolute values as modifiers)
    const float mx = fmaxf(fmaxf(ax, ay), 1e-30f), mn = __builtin_amdgcn_fmed3f(ax, ay, 0.0f);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float t2 = t * t;
    float p = 0.02093181200325489f;
    p = fmaf(p, t2, -0.08540830761194229f);
    p = fmaf(p, t2, 0.1804126799106598f);
    p = fmaf(p, t2, -0.3304055631160736f);
    p = fmaf(p, t2, 0.9998787641525269f);
    float a = p * t;                                   // atan(t), t in [0, 1]
    const float d = ax - ay;                           // negative: swapped
    a = copysignf(a, __uint_as_float(xor3_v(__float_as_uint(hx), __float_as_uint(hy), __float_as_uint(d))));
    return __float_as_uint(fmaf(a, kTwoPhiScale, d < 0.f ? 12615680.0f : 12582912.0f));
}

__device__ __forceinline__ double2 unit64(uint32_t th, const double2 *t64)
{
    const double2 a = t64[th >> 8], c = t64[256 + (th & 255u)];
    return make_double2(a.x * c.x - a.y * c.y, a.y * c.x + a.x * c.y);
}

// Metropolis acceptance with probability min(1, exp(-beta dE)) for the FP32
// exp p (the hardware 2^x of dE * accept_factor(beta); p >= 1 when dE <= 0).
// The uniform is U = (u + V) / 2^16 with u the top 16 bits of `word` and V a
// further uniform, drawn only when needed: with q = p 2^16 - u (exact in one
// fused multiply-add), U < p holds for every V when q >= 1, for none when
// q < 0, and else (probability 2^-16) iff V < q, V from 32 more bits of the
// counter (site, sweep, slot, purpose 4 | sub).  So the test is exact.
__device__ __forceinline__ bool accept_move(float dE, float factor, uint32_t word, uint32_t site, uint32_t sweep,
                                            uint32_t slot, uint32_t sub, const SampleDesc &d)
{
    const float p = __builtin_amdgcn_exp2f(dE * factor);
    const float q = fmaf(p, 65536.0f, -(float)(word >> 16));
    if (q >= 1.0f) return true;
    if (q < 0.0f) return false;
    // (an empty volatile asm on the counter words: the compiler may not start
    // this rare draw's rounds ahead of the branch)
    asm volatile("" : "+v"(site), "+v"(slot));
    const U4 x = philox4x32_10({site, sweep, slot, tag(kMetAcc, sub)}, d.seed_lo, d.seed_hi);
    return (double)x.x < (double)q * 4294967296.0;
}

// Over-relaxation: true when the Metropolis test of the reflection accepts
// for certain, so that its energy change need not be evaluated.  The
// reflection theta' = 2 phi~ - theta about the computed axis changes the
// energy by dE = h . (s(theta) - s(theta')), s(x) = (cos x, sin x); with the
// axis 2 phi~ = 2 atan2(h_y, h_x) + delta it equals |h| (cos x - cos(x - delta))
// for x = theta - atan2(h_y, h_x), so |dE| <= |h| |delta| exactly, where
// |delta| <= 2 x 1.3e-5 (the atan polynomial) + 2pi / 2^17 (the rounding of
// 2 phi~ to the grid; the ratio's reciprocal and the scale add under 1e-6
// grid units) < 7.44e-5 rad.  The FP32 (cos, sin) of the 2^16 grid angles are
// within kTrigErr of the exact values (the largest error over all of them,
// measured on the GPU, is 1.2e-7), and the FP32 evaluation of dE adds under
// 4e-7 (|h_x| + |h_y|), so |dE| <= kDeltaE (|h_x| + |h_y|).  accept_move
// accepts when p 2^16 - u >= 1 for p = 2^(dE factor) (factor = -beta log2 e):
// with 2^(-y) >= 1 - y ln 2 and the hardware 2^x within kExp2Err (relative)
// for the arguments where this matters (|y| < 1.5; measured on [-2, 0.5]),
// u + 2^16 ln 2 kDeltaE |factor| (|h_x| + |h_y|) + 2^16 kExp2Err <= 65535
// suffices.  The test below uses a coefficient and a bound with margin over
// these; a move it does not clear takes the full test.
constexpr float kTrigErr = 2e-7f;
constexpr float kExp2Err = 2e-7f;
constexpr float kDeltaE = 7.44e-5f + 2.0f * kTrigErr + 4e-7f;
constexpr float kOrSureCoef = 4.0f;                            // > 2^16 ln 2 kDeltaE = 3.42

__device__ __forceinline__ bool or_accepts_surely(float hx, float hy, float factor, uint32_t word)
{
    return fmaf(-kOrSureCoef * factor, fabsf(hx) + fabsf(hy), (float)(word >> 16)) <= 65534.0f;
}

// Philox4x32-10 as philox4x32_10, for keys that are the same in every lane
// of the wave (scalar registers): each round's two three-input XORs are one
// v_bitop3_b32 each (truth table 0x96, a ^ b ^ c) instead of two v_xor_b32.
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ U4 philox4x32_10_uniform_key(U4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    const uint32_t kBumpA = 0x9E3779B9u, kBumpB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c.x;
        const uint64_t pb = (uint64_t)kMulB * c.z;
        U4 n;
        n.x = xor3_sk((uint32_t)(pb >> 32), c.y, k0);
        n.y = (uint32_t)pb;
        n.z = xor3_sk((uint32_t)(pa >> 32), c.w, k1);
        n.w = (uint32_t)pa;
        c = n;
        k0 += kBumpA;
        k1 += kBumpB;
    }
    return c;
}

// Phase form: threads per workgroup of the colour-phase kernel
constexpr int kPhaseBlock = 256;

}  // namespace
}  // namespace xy
