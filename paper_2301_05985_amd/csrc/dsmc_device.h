// dsmc_device.h -- device-side building blocks of the DSMC hot path (gfx950).
//
// Everything here is written for CDNA wave64: lane-level votes (__ballot
// returns a 64-bit mask), cross-lane shuffles, and LDS atomics.  All
// floating-point expressions are written in the exact evaluation order that
// defines the method's arithmetic; the library is compiled with
// -ffp-contract=off so no multiply-add is fused behind the code's back, and
// with correctly rounded FP32 division and square root.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsmc {

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0,c1,c2,c3) -> (hi(B*c2)^c1^k0, lo(B*c2), hi(A*c0)^c3^k1, lo(A*c0))
// with A = 0xD2511F53, B = 0xCD9E8D57; the key advances by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) between rounds.
struct u32x4 { uint32_t v[4]; };

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = 0xD2511F53u * c0, hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2, hi_b = __umulhi(0xCD9E8D57u, c2);
        c0 = hi_b ^ c1 ^ k0;
        c1 = lo_b;
        c2 = hi_a ^ c3 ^ k1;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    u32x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Stream keying: counter word 0 = sub-index (candidate / wall hit), word 1 =
// tag << 24 | block, word 2 = cell, instance or particle id, word 3 = step.
enum : uint32_t { kTagNcand = 1u, kTagPair = 2u, kTagWall = 3u };

__device__ __forceinline__ u32x4 draw(uint32_t sub, uint32_t tag, uint32_t block, uint32_t who,
                                      uint32_t step, uint32_t k0, uint32_t k1) {
    return philox10(sub, (tag << 24) | block, who, step, k0, k1);
}

// Uniform on [0,1): 53 bits (32 from a, 21 from the top of b) or 24 bits.
__device__ __forceinline__ double unif53(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * 0x1.0p-53;
}
__device__ __forceinline__ float unif24(uint32_t a) { return (float)(a >> 8) * 0x1.0p-24f; }

// Index in [0, n) from a 32-bit word by multiply-shift (no rejection).
__device__ __forceinline__ uint32_t scale_index(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// ----------------------------------------------------------------- wave ops
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wave-aggregated counter increment: lanes with equal `key` share one
// atomic; returns the value each lane would have obtained from its own
// atomicAdd(&ctr[key], 1) in some order.  The loop runs once per distinct
// key in the wave, which after the first step is a handful, because the
// particle arrays arrive sorted by cell.
__device__ __forceinline__ uint32_t wave_aggregated_inc(uint32_t *ctr, uint32_t key, bool active) {
    const int lane = lane_id();
    unsigned long long rem = __ballot(active);
    uint32_t slot = 0;
    while (rem) {
        const int leader = __ffsll((long long)rem) - 1;
        const uint32_t lk = __shfl(key, leader, 64);
        const unsigned long long same = __ballot(active && key == lk) & rem;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[lk], (uint32_t)__popcll(same));
        base = __shfl(base, leader, 64);
        if ((same >> lane) & 1ull) slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        rem &= ~same;
    }
    return slot;
}

}  // namespace dsmc
