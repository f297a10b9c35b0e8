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
        // the round keys are recomputed (two scalar adds) rather than kept:
        // hoisted out of the callers' loops they would hold 20 scalar
        // registers for the whole kernel
        asm volatile("" : "+s"(k0), "+s"(k1));
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

// x^a for x >= 0, 0 <= a <= 1, as 2^(a log2 x) in a fixed sequence of IEEE
// double operations (the variable-hard-sphere acceptance takes a decision on
// it, so the sequence is part of the method's definition here).
//   log2: x = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) with
//         s = (m - 1)/(m + 1) by its odd series through s^27 (Horner in s^2).
//   exp2: y = n + f, n = floor(y); 2^f = e^(f ln 2) by its Taylor series
//         through degree 18, Horner on the coefficients 1/k! (one multiply
//         and one add per degree, no division); scaled by 2^n exactly.
__device__ __forceinline__ double vhs_log2(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double sv = (m - 1.0) / (m + 1.0);
    const double s2 = sv * sv;
    double t = 1.0 / 27.0;
#pragma unroll
    for (int k = 25; k >= 1; k -= 2) t = t * s2 + 1.0 / (double)k;
    const double lnm = (2.0 * sv) * t;
    return (double)e + lnm * 1.44269504088896340736;
}
// 1/k! for k = 0..18, each the correctly rounded quotient of 1 and the
// exact integer k! (below 2^53), evaluated at compile time.
struct InvFactorials {
    double c[19];
};
constexpr InvFactorials inv_factorials() {
    InvFactorials r{};
    double f = 1.0;
    for (int k = 0; k <= 18; ++k) {
        if (k > 0) f *= (double)k;
        r.c[k] = 1.0 / f;
    }
    return r;
}
__device__ __forceinline__ double vhs_exp2(double y) {
    constexpr InvFactorials kC = inv_factorials();
    const double n = floor(y);
    const double f = (y - n) * 0.69314718055994530942;
    double t = kC.c[18];
#pragma unroll
    for (int k = 17; k >= 0; --k) t = t * f + kC.c[k];
    return ldexp(t, (int)n);
}
__device__ __forceinline__ double vhs_pow(double x, double a) {
    if (a == 0.0) return 1.0;
    if (!(x > 0.0)) return 0.0;
    if (x == 1.0) return 1.0;
    const double y = a * vhs_log2(x);
    if (y < -1000.0) return 0.0;
    return vhs_exp2(y);
}

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

// Wave-aggregated counter increment.  Lanes with equal `key` form a group;
// each group's first lane (its leader) adds the group size with a single
// atomic, all groups' atomics being issued by one instruction.  Returns the
// value each lane would have obtained from its own atomicAdd(&ctr[key], 1) in
// some order (or nothing, for the counting-only variant).  The grouping loop
// runs once per distinct key in the wave: a handful, because the particle
// arrays arrive sorted by cell after the first step.
struct WaveGroup {
    int leader;       // lane that carries the group's atomic
    uint32_t rank;    // position of this lane inside its group
    uint32_t size;    // group size (valid on the leader)
};

__device__ __forceinline__ WaveGroup wave_group(uint32_t key, bool active) {
    const int lane = lane_id();
    const unsigned long long lt = (1ull << lane) - 1ull;
    unsigned long long rem = __ballot(active);
    WaveGroup g{lane, 0u, 0u};
    while (rem) {
        const int leader = __ffsll((long long)rem) - 1;
        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const unsigned long long same = __ballot(active && key == lk) & rem;
        if ((same >> lane) & 1ull) {
            g.leader = leader;
            g.rank = (uint32_t)__popcll(same & lt);
        }
        if (lane == leader) g.size = (uint32_t)__popcll(same);
        rem &= ~same;
    }
    return g;
}

__device__ __forceinline__ void wave_aggregated_add(uint32_t *ctr, uint32_t key, bool active) {
    const WaveGroup g = wave_group(key, active);
    if (active && g.leader == lane_id()) atomicAdd(&ctr[key], g.size);  // result unused: no-return atomic
}

__device__ __forceinline__ uint32_t wave_aggregated_inc(uint32_t *ctr, uint32_t key, bool active) {
    const WaveGroup g = wave_group(key, active);
    uint32_t base = 0;
    if (active && g.leader == lane_id()) base = atomicAdd(&ctr[key], g.size);
    base = __shfl(base, g.leader, 64);
    return base + g.rank;
}

// Sum K per-lane values (K a power of two, at most 32) over the wave by
// recursive halving: at stride 32 each half of the wave keeps half of the
// values and receives the partner's copy of them, and so on until one value
// per lane is left; the remaining strides add it up.  K + log2(64/K) - 1
// shuffles instead of 6 K.  On return lane L holds the total of value index
// L >> log2(64/K).
template <int K, int HALF, int OFF>
struct HalvingStep {
    // one level: keep HALF values, receive the partner's copy of them
    static __device__ __forceinline__ void run(double (&v)[K], int lane) {
        if constexpr (OFF == 32 || OFF == 16) {
            // gfx950 lane swaps: v_permlane32_swap exchanges the upper half
            // of the first register with the lower half of the second
            // (v_permlane16_swap the odd rows of 16 with the even ones), so
            // the lower half of each 2 OFF lanes ends with (own v[k],
            // partner's v[k]) and the upper half with (partner's v[HALF + k],
            // own v[HALF + k]): the same two terms as the select-and-shuffle
            // form, without the selects
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                const uint64_t a = (uint64_t)__double_as_longlong(v[k]);
                const uint64_t b = (uint64_t)__double_as_longlong(v[HALF + k]);
                uint32_t xl, yl, xh, yh;
                if constexpr (OFF == 32) {
                    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
                    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false,
                                                                     false);
                    xl = lo[0]; yl = lo[1]; xh = hi[0]; yh = hi[1];
                } else {
                    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
                    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false,
                                                                     false);
                    xl = lo[0]; yl = lo[1]; xh = hi[0]; yh = hi[1];
                }
                const double x = __longlong_as_double((long long)(((uint64_t)xh << 32) | xl));
                const double y = __longlong_as_double((long long)(((uint64_t)yh << 32) | yl));
                v[k] = x + y;
            }
        } else if constexpr (OFF == 8 || OFF == 4) {
            // inside rows of 16 lanes: a row rotation by 8 (or by 12 and 4)
            // brings the partner's value; the bank mask (groups of 4 lanes)
            // lets only the lower (upper) lanes take it, the others keep
            // their own register, so x + y is (own, partner's) v[k] on the
            // lower lanes and v[HALF + k] on the upper ones
            constexpr int kLowBanks = OFF == 8 ? 0x3 : 0x5, kHighBanks = OFF == 8 ? 0xC : 0xA;
            constexpr int kRorLow = OFF == 8 ? 0x128 : 0x12C, kRorHigh = OFF == 8 ? 0x128 : 0x124;
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                const uint64_t a = (uint64_t)__double_as_longlong(v[k]);
                const uint64_t b = (uint64_t)__double_as_longlong(v[HALF + k]);
                const uint32_t xl = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)b, (int)(uint32_t)a, kRorLow,
                                                                          0xF, kLowBanks, false);
                const uint32_t xh = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(b >> 32),
                                                                          (int)(uint32_t)(a >> 32), kRorLow, 0xF,
                                                                          kLowBanks, false);
                const uint32_t yl = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)a, (int)(uint32_t)b,
                                                                          kRorHigh, 0xF, kHighBanks, false);
                const uint32_t yh = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(a >> 32),
                                                                          (int)(uint32_t)(b >> 32), kRorHigh, 0xF,
                                                                          kHighBanks, false);
                const double x = __longlong_as_double((long long)(((uint64_t)xh << 32) | xl));
                const double y = __longlong_as_double((long long)(((uint64_t)yh << 32) | yl));
                v[k] = x + y;
            }
        } else {
            const bool upper = (lane & OFF) != 0;
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                const double keep = upper ? v[HALF + k] : v[k];
                const double send = upper ? v[k] : v[HALF + k];
                v[k] = keep + __shfl_xor(send, OFF, 64);
            }
        }
        HalvingStep<K, HALF / 2, OFF / 2>::run(v, lane);
    }
};
template <int K, int OFF>
struct HalvingStep<K, 0, OFF> {
    static __device__ __forceinline__ void run(double (&)[K], int) {}
};

template <int K>
__device__ __forceinline__ double wave_sum_many(double (&v)[K]) {
    static_assert(K >= 1 && K <= 32 && (K & (K - 1)) == 0, "K must be a power of two <= 32");
    const int lane = lane_id();
    HalvingStep<K, K / 2, 32>::run(v, lane);
    double r = v[0];
#pragma unroll
    for (int o = 64 / (2 * K); o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
    return r;
}

// DPP wave reductions (GFX9 data-parallel moves): row shifts by 1, 2, 4, 8
// combine each row of 16 lanes into its lane 15, then the row broadcasts 15
// and 31 carry rows into lane 63, whose value is read as a scalar.  These
// are VALU moves, not LDS-crossbar permutes.  `id` is the identity of the
// operation (lanes without a source keep it).
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v, int ctrl, int row_mask) {
    switch (ctrl) {  // the DPP control must be a compile-time constant
        case 0x111: return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x111, 0xF, 0xF, false);
        case 0x112: return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x112, 0xF, 0xF, false);
        case 0x114: return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x114, 0xF, 0xF, false);
        case 0x118: return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x118, 0xF, 0xF, false);
        case 0x142: return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x142, 0xA, 0xF, false);
        default:    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x143, 0xC, 0xF, false);
    }
}
__device__ __forceinline__ float dpp_f32(float old, float v, int ctrl) {
    return __uint_as_float(dpp_u32(__float_as_uint(old), __float_as_uint(v), ctrl, 0));
}
__device__ __forceinline__ double dpp_f64(double old, double v, int ctrl) {
    const uint64_t o = (uint64_t)__double_as_longlong(old), x = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = dpp_u32((uint32_t)o, (uint32_t)x, ctrl, 0);
    const uint32_t hi = dpp_u32((uint32_t)(o >> 32), (uint32_t)(x >> 32), ctrl, 0);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Value of another lane of the same quad (DPP quad permutation CTRL; every
// source lane is valid, so no identity is needed).
template <int CTRL>
__device__ __forceinline__ double quad_perm_f64(double v) {
    const uint64_t x = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Sum over the four lanes of each quad, the same in all four.
__device__ __forceinline__ double quad_sum_f64(double v) {
    v += quad_perm_f64<0xB1>(v);  // lanes (0,1)(2,3) swapped
    return v + quad_perm_f64<0x4E>(v);  // pairs swapped
}
__device__ __forceinline__ uint32_t dpp_any(uint32_t old, uint32_t v, int ctrl) { return dpp_u32(old, v, ctrl, 0); }
__device__ __forceinline__ float dpp_any(float old, float v, int ctrl) { return dpp_f32(old, v, ctrl); }
__device__ __forceinline__ double dpp_any(double old, double v, int ctrl) { return dpp_f64(old, v, ctrl); }

__device__ __forceinline__ uint32_t read_lane63(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ float read_lane63(float v) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(v), 63));
}
__device__ __forceinline__ double read_lane63(double v) {
    const uint64_t x = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce_dpp(T v, T id, Op op) {
    v = op(v, dpp_any(id, v, 0x111));
    v = op(v, dpp_any(id, v, 0x112));
    v = op(v, dpp_any(id, v, 0x114));
    v = op(v, dpp_any(id, v, 0x118));
    v = op(v, dpp_any(id, v, 0x142));
    v = op(v, dpp_any(id, v, 0x143));
    return read_lane63(v);
}

// Wave minimum of an unsigned value (uniform result).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    return wave_reduce_dpp(v, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
}

template <typename T>
__device__ __forceinline__ T wave_min_t(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max_t(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace dsmc
