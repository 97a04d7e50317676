// Device-side helpers of libpdv: counter-based random numbers, uniform
// mapping, precision-specific math and wavefront utilities (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdv {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  A 128-bit counter is
// mixed with a 64-bit key by ten rounds; each round multiplies words 0 and 2
// by fixed 32-bit constants, keeps the low halves as the new words 3 and 1,
// and xors the high halves with the other two words and the round key.  The
// key advances by two Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct Block4 { uint32_t x, y, z, w; };

// a ^ b ^ c in one instruction: gfx950's three-input bit operation with the
// truth table of a three-way exclusive or (0x96); the compiler does not form
// it from two xors by itself
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The transport draws the block with counter (k, pid low, pid high, stream)
// for event k of a packet.  Counter words 1 and 2 (the packet id) are fixed
// for a packet, so the first round's product of word 2 and the words it
// feeds are formed once per packet (philox_packet_words); per event only the
// first-round product of the event counter k remains (philox10_event,
// s3 = stream ^ k1).  Each product is one 32x32->64 multiply
// (v_mad_u64_u32).
__device__ __forceinline__ void philox_packet_words(uint32_t pid_lo, uint32_t pid_hi, uint32_t k0, uint32_t& q0,
                                                    uint32_t& q1) {
    const uint64_t pb = (uint64_t)0xCD9E8D57u * pid_hi;
    q0 = (uint32_t)(pb >> 32) ^ pid_lo ^ k0;
    q1 = (uint32_t)pb;
}

__device__ __forceinline__ Block4 philox10_event(uint32_t k, uint32_t q0, uint32_t q1, uint32_t s3, uint32_t k0,
                                                 uint32_t k1) {
    constexpr uint32_t MUL_A = 0xD2511F53u, MUL_B = 0xCD9E8D57u;
    constexpr uint32_t BUMP_A = 0x9E3779B9u, BUMP_B = 0xBB67AE85u;
    const uint64_t p1 = (uint64_t)MUL_A * k;
    uint32_t c0 = q0, c1 = q1, c2 = (uint32_t)(p1 >> 32) ^ s3, c3 = (uint32_t)p1;
    k0 += BUMP_A;
    k1 += BUMP_B;
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        const uint64_t pa = (uint64_t)MUL_A * c0;
        const uint64_t pb = (uint64_t)MUL_B * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c0 = n0; c1 = (uint32_t)pb; c2 = n2; c3 = (uint32_t)pa;
        k0 += BUMP_A; k1 += BUMP_B;
    }
    return Block4{c0, c1, c2, c3};
}

// A 32-bit word to an odd multiple of 2^-24 in (0,1): exact in binary32 and
// binary64, so both precisions see the same uniform.
template <typename Real>
__device__ __forceinline__ Real unit_open(uint32_t x) {
    if constexpr (sizeof(Real) == 4) {
        // 1 + m 2^-23 from the top 23 bits as the mantissa, minus (1 - 2^-24):
        // exact (Sterbenz), and equal to (2m + 1) 2^-24.  The exponent bits
        // 0x3f800000 = 0x7f << 23 come in with the shift as the high word of
        // a funnel shift (one v_alignbit_b32).
        const uint32_t bits = __builtin_amdgcn_alignbit(0x7fu, x, 9u);
        return __uint_as_float(bits) - 0.99999994039535522461f;
    } else {
        return (Real)(((x >> 9) << 1) | 1u) * (Real)5.9604644775390625e-08;
    }
}

// ---------------------------------------------------------------------------
// Precision-specific math.  FP32 uses the hardware transcendental units with
// arguments in revolutions (v_sin/v_cos take x and return sin/cos(2 pi x));
// FP64 uses the correctly rounded library forms in the same expression
// order as a plain scalar evaluation.
// ---------------------------------------------------------------------------
template <typename Real> struct M;

template <> struct M<float> {
    // a * b + c with one rounding; the transport is compiled without
    // implicit contraction, so every fused operation is written out and the
    // arithmetic does not depend on how the compiler arranges the code
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float neg_log(float u) {
        return -0.693147180559945309f * __builtin_amdgcn_logf(u);
    }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // cos(2 pi r), sin(2 pi r) for |r| <= 1
    static __device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }
    static __device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
    // x clamped to [-1, 1] (one v_med3_f32)
    static __device__ __forceinline__ float clamp1(float x) { return __builtin_amdgcn_fmed3f(x, -1.0f, 1.0f); }
    // exp(-x) through the base-2 exponential unit
    static __device__ __forceinline__ float exp_neg(float x) {
        return __builtin_amdgcn_exp2f(-x * 1.44269504088896341f);
    }
    static __device__ __forceinline__ float acos(float x) { return ::acosf(x); }
};

template <> struct M<double> {
    static constexpr double PI = 3.14159265358979323846;
    // the FP64 kernels are compiled with contraction, which fuses this (an
    // explicit ::fma call there cost scalar registers and spills)
    static __device__ __forceinline__ double fma(double a, double b, double c) { return a * b + c; }
    static __device__ __forceinline__ double neg_log(double u) { return -::log(u); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double cos_rev(double r) { return ::cos(2.0 * PI * r); }
    static __device__ __forceinline__ double sin_rev(double r) { return ::sin(2.0 * PI * r); }
    static __device__ __forceinline__ double clamp1(double x) { return x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x); }
    static __device__ __forceinline__ double exp_neg(double x) { return ::exp(-x); }
    static __device__ __forceinline__ double acos(double x) { return ::acos(x); }
};

template <typename Real>
__device__ __forceinline__ uint64_t to_fixed32(Real w) {
    // w * 2^32 rounded to nearest; w in [0, 1]
    if constexpr (sizeof(Real) == 4) {
        // below 1 the scaled value fits 32 bits (and is exact for w >= 2^-8)
        const uint32_t lo = (uint32_t)__builtin_rintf(w * 4294967296.0f);
        return w >= 1.0f ? 4294967296ull : (uint64_t)lo;
    } else {
        return __double2ull_rn(w * 4294967296.0);
    }
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace pdv
