// dsmc_collide.h -- per-cell NTC collisions, importance weights and moment
// sampling, one 64-lane wave per cell (or a workgroup of waves for large
// homogeneous instances).
//
// Method (Bird 1994, no-time-counter scheme): a cell of N particles takes
//   M = floor( 1/2 N (N-1) F_N sigma g_max dt / V  +  U0 )
// candidates; candidate k draws an ordered pair of distinct canonical ranks
// (i, j) and is accepted with probability g_ij / g_max (hard spheres; Maxwell
// molecules accept every candidate and use sigma*g = const in place of
// sigma*g_max; variable hard and soft spheres accept with probability
// (g / g_max)^(2 - 2 omega)).  An accepted pair scatters isotropically about
// its centre of mass (variable soft spheres: by the deflection law of the
// exponent alpha).  Candidates are sequential by definition -- candidate k sees the
// velocities left by candidates 0..k-1.
//
// Wave mapping: 64 consecutive candidates are drawn at once, one per lane
// (256 on a workgroup cell).  Lanes that will write velocities (accepted
// pairs) mark their two particles in an LDS owner array with an atomic min
// of their candidate index.  The first candidate whose particles were marked
// by an earlier one ends the batch: every candidate before it read exactly
// the state the sequential definition gives it, and the writers among them
// touch disjoint particles, so they commit in parallel.  The next batch
// starts at the first uncommitted candidate.  Importance weights, which
// every candidate updates, are applied afterwards in rounds of candidates
// that share no particle with an earlier pending one.  Results are
// bit-identical to the sequential loop.
#pragma once
#include "dsmc_kernels.h"

namespace dsmc {

template <typename R>
struct CollideArgs {
    Soa<R> s;                      // particles grouped by cell (or instance storage)
    const uint32_t *start;         // [ncell + 1] first particle of each cell
    const uint32_t *sched;         // block -> cell, or null for the identity
    // walled runs: s is written in the new sequence, gathered from src (the
    // streamed particles in the previous sequence): each cell's stays and
    // movers (the regrouping lists, reset once read)
    Soa<R> src;
    const uint32_t *src_start;     // [ncell + 1] cell ranges of src
    Regroup rg;
    const double *volume;          // per-cell volume, or null for Vuni
    double Vuni, dt, sigma, FN;
    double omega1;                 // VHS, VSS: 1 - omega
    double inv_alpha;              // VSS: 1 / alpha
    int molecule, cap, majorant;
    uint32_t k0, k1;
    double *sums;                  // [ncell][26] running FP64 sums
    unsigned long long *counters;  // [ncell][2] candidates, accepted
    DevState *st;
    uint32_t *big_list;            // cells too large for the LDS kernel
    unsigned int *bigc;            // their count (the step's slot for homogeneous runs)
    unsigned int *queue;           // persistent kernel: the step's work-unit queues
    uint32_t step_off;             // homogeneous runs: step within the recorded batch
    uint32_t *perm_g, *owner_g;    // [n] scratch of the global-memory kernel
    // learned majorant
    const float *mlp;              // [4673] FP32 weights or null
    const double *lattice;         // lattice values 2^(k/64), k in [-4096, 4096]
    double delta;
    uint32_t mlp_min_n;            // cells of fewer particles skip the network
    // importance weights: re-estimation every vr_reest steps (0: never) with
    // velocities scaled by vr_scale = 1 / sqrt(T0); majorant factor vr_kappa
    int vr_reest;
    double vr_scale, vr_kappa;
    uint32_t n_total, n_cells;     // particles and cells (index checks of the bounds-checking build)
};

constexpr int kNsum = 26;
// Transpose area of the moment reduction of a cell staged in LDS: 13 rows
// of kRedStride doubles (the cell's LDS area is at least this large).
constexpr int kRedStride = 64;
constexpr size_t kRedBytes = (size_t)13 * kRedStride * 8;
// Most NTC candidates one cell may take in one step (2^24); a larger count
// stops the step with DSMC_ECAPACITY, so that a run whose velocities have
// blown up ends with an error instead of keeping a wave busy for minutes.
constexpr double kMaxCandidates = 16777216.0;

// A cell is processed by T threads: one wave (T = 64), a workgroup of T / 64
// waves for large homogeneous instances, or one half of a wave (T = 32, two
// walled cells per wave).  Wave-level results of a workgroup are combined
// through a small LDS area after a barrier, every thread combining the waves
// in the same order.  In the one-wave workgroups of T = 64 and T = 32 a
// __syncthreads() orders the wave's LDS accesses and waits for no other
// wave, so the two halves of a wave may reach it on different paths.
constexpr int kWideThreads = 256;
struct GroupScratch {
    uint32_t u[kWideThreads / 64][8];
    double d[kWideThreads / 64][32];
};
template <int T>
__device__ __forceinline__ void grp_put(GroupScratch *gs, int slot, uint32_t v) {
    if constexpr (T > 64) {
        if (lane_id() == 0) gs->u[threadIdx.x >> 6][slot] = v;
    }
}
template <int T>
__device__ __forceinline__ void grp_putd(GroupScratch *gs, int slot, double v) {
    if constexpr (T > 64) {
        if (lane_id() == 0) gs->d[threadIdx.x >> 6][slot] = v;
    }
}
template <int T>
__device__ __forceinline__ uint32_t grp_min(const GroupScratch *gs, int slot, uint32_t v) {
    if constexpr (T > 64) {
        uint32_t r = gs->u[0][slot];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) r = r < gs->u[w][slot] ? r : gs->u[w][slot];
        return r;
    }
    return v;
}
template <int T>
__device__ __forceinline__ uint32_t grp_sum(const GroupScratch *gs, int slot, uint32_t v) {
    if constexpr (T > 64) {
        uint32_t r = gs->u[0][slot];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) r += gs->u[w][slot];
        return r;
    }
    return v;
}
// a barrier only between the waves of a workgroup (one wave needs none)
template <int T>
__device__ __forceinline__ void grp_sync() {
    if constexpr (T > 64) __syncthreads();
}

// ------------------------------------------------- lanes of one cell
// T = 32: a cell takes one half of a wave (lanes 0-31 or 32-63), so that a
// wave works on two cells at once; every cross-lane operation below stays
// inside the half, and a value that is uniform over the cell lives in a
// vector register.  T = 64: the whole wave (the results are wave-uniform).
// T > 64: the wave-level operation of the thread's own wave (combined over
// the workgroup by the grp_* helpers).
template <int T>
__device__ __forceinline__ uint32_t cell_tid() {
    if constexpr (T == 32) return (uint32_t)lane_id() & 31u;
    else return threadIdx.x;
}
template <int T>
__device__ __forceinline__ int cell_lane() {
    if constexpr (T == 32) return lane_id() & 31;
    else return lane_id();
}
// Ballot over the cell's lanes: bit l for cell lane l.
template <int T>
__device__ __forceinline__ unsigned long long cell_ballot(bool p) {
    const unsigned long long b = __ballot(p);
    if constexpr (T == 32) return (lane_id() & 32) ? (b >> 32) : (b & 0xFFFFFFFFull);
    else return b;
}
// Value of cell lane l (l in [0, T) for T <= 64).
template <int T, typename V>
__device__ __forceinline__ V cell_shfl(V x, int l) {
    if constexpr (T == 32) return __shfl(x, (lane_id() & 32) | l, 64);
    else return __shfl(x, l, 64);
}
// Combination of a value over each half-wave of 32 lanes, left in every lane:
// a butterfly of DPP moves inside each row of 16 (quad swaps of 1 and 2
// lanes, then the half-row and row mirrors, each pairing every lane with one
// of the other group), then v_permlane16_swap pairs each row with the other
// row of its half.  All sources lie in the lane's own half.
template <typename Op>
__device__ __forceinline__ uint32_t half_butterfly_u32(uint32_t v, Op op) {
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return op((uint32_t)sw[0], (uint32_t)sw[1]);
}
template <int T>
__device__ __forceinline__ uint32_t cell_min_u32(uint32_t v) {
    if constexpr (T == 32) {
        return half_butterfly_u32(v, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
    } else {
        return wave_min_u32(v);
    }
}
template <int T, typename V, typename Op>
__device__ __forceinline__ V cell_reduce_dpp(V v, V id, Op op) {
    if constexpr (T == 32) {
        v = op(v, dpp_any(id, v, 0x111));
        v = op(v, dpp_any(id, v, 0x112));
        v = op(v, dpp_any(id, v, 0x114));
        v = op(v, dpp_any(id, v, 0x118));
        v = op(v, dpp_any(id, v, 0x142));
        return __shfl(v, (lane_id() & 32) | 31, 64);
    } else {
        return wave_reduce_dpp(v, id, op);
    }
}
template <int T>
__device__ __forceinline__ uint32_t cell_sum_u32(uint32_t v) {
    if constexpr (T == 32) {
        return half_butterfly_u32(v, [](uint32_t a, uint32_t b) { return a + b; });
    } else {
        return wave_sum_u32(v);
    }
}
template <int T, typename V>
__device__ __forceinline__ V cell_max_t(V v) {
    if constexpr (T == 32) {
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        return v;
    } else {
        return wave_max_t(v);
    }
}
// Sum of K per-lane values over the cell's lanes by recursive halving: on
// return cell lane l holds the total of value index l / (T / K) (T <= 64).
template <int T, int K>
__device__ __forceinline__ double cell_sum_many(double (&v)[K]) {
    if constexpr (T == 32) {
        static_assert(K >= 1 && K <= 32 && (K & (K - 1)) == 0, "K must be a power of two <= 32");
        HalvingStep<K, K / 2, 16>::run(v, lane_id());
        double r = v[0];
#pragma unroll
        for (int o = 32 / (2 * K); o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
        return r;
    } else {
        return wave_sum_many<K>(v);
    }
}

// Rank check of a cell view in the bounds-checking build: a rank at or
// above the limit (the staged cell's capacity, or the size of a cell in
// global memory) is counted in the diagnostics and replaced by rank 0.  The
// release build keeps no state and returns the rank.
struct ViewCheck {
#ifdef DSMC_BOUNDS_CHECK
    uint32_t lim = 0xFFFFFFFFu;
    DevState *st = nullptr;
#endif
    __device__ __forceinline__ uint32_t operator()(uint32_t r) const {
#ifdef DSMC_BOUNDS_CHECK
        return st ? bounds_ck(r, lim, st) : r;
#else
        return r;
#endif
    }
};
__device__ __forceinline__ ViewCheck view_check(uint32_t lim, DevState *st) {
    ViewCheck v{};
#ifdef DSMC_BOUNDS_CHECK
    v.lim = lim;
    v.st = st;
#else
    (void)lim;
    (void)st;
#endif
    return v;
}

// One particle of a cell staged in LDS: velocity and weight side by side,
// so that a particle is read with one 16-byte access (two in double).
template <typename R>
struct alignas(16) Vel4 {
    R x, y, z, w;
};

// Cell staged in LDS (index = rank in the cell's collision order).  Without
// weights (PACKED) a particle's owner mark lives in the unused weight slot
// of its row (its first 32 bits), 16 instead of 20 bytes per particle in
// FP32, so more cells fit in LDS at once.
template <typename R, bool PACKED = false>
struct LdsView {
    static constexpr bool kInLds = true;
    Vel4<R> *p;
    uint32_t *owner;
    ViewCheck ck;
    __device__ __forceinline__ void get(uint32_t r, R &a, R &b, R &c) const {
        const Vel4<R> t = p[ck(r)];
        a = t.x; b = t.y; c = t.z;
    }
    __device__ __forceinline__ void put(uint32_t r, R a, R b, R c) const {
        r = ck(r);
        p[r].x = a; p[r].y = b; p[r].z = c;
    }
    __device__ __forceinline__ R getw(uint32_t r) const { return p[ck(r)].w; }
    __device__ __forceinline__ void putw(uint32_t r, R v) const { p[ck(r)].w = v; }
    __device__ __forceinline__ uint32_t *own(uint32_t r) const {
        r = ck(r);
        if constexpr (PACKED) return reinterpret_cast<uint32_t *>(&p[r].w);
        else return &owner[r];
    }
    __device__ __forceinline__ uint32_t read_own(uint32_t r) const { return *own(r); }
    __device__ __forceinline__ void clear_own(uint32_t r) const { *own(r) = 0xFFFFFFFFu; }
};

// Cell operated on in place in global memory, through a rank -> slot map.
template <typename R>
struct GlobalView {
    static constexpr bool kInLds = false;
    R *cx, *cy, *cz, *w;
    const uint32_t *perm;  // rank -> slot inside the cell, or null for the identity
    uint32_t *owner;
    ViewCheck ck;
    __device__ __forceinline__ uint32_t at(uint32_t r) const {
        r = ck(r);
        return perm ? ck(perm[r]) : r;
    }
    __device__ __forceinline__ void get(uint32_t r, R &a, R &b, R &c) const {
        const uint32_t q = at(r); a = cx[q]; b = cy[q]; c = cz[q];
    }
    __device__ __forceinline__ void put(uint32_t r, R a, R b, R c) const {
        const uint32_t q = at(r); cx[q] = a; cy[q] = b; cz[q] = c;
    }
    __device__ __forceinline__ R getw(uint32_t r) const { return w[at(r)]; }
    __device__ __forceinline__ void putw(uint32_t r, R v) const { w[at(r)] = v; }
    __device__ __forceinline__ uint32_t *own(uint32_t r) const { return &owner[ck(r)]; }
    // the marks are set by device-scope atomics; read and clear them at the
    // same scope so no stale L1 line is seen
    __device__ __forceinline__ uint32_t read_own(uint32_t r) const {
        return __hip_atomic_load(&owner[ck(r)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void clear_own(uint32_t r) const {
        __hip_atomic_store(&owner[ck(r)], 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Exact per-cell majorant: m = midpoint of the velocity bounding box,
// r_p = |c_p - m|, bound = (r_(1) + r_(2)) (1 + eps) >= |c_i - c_j| for every
// pair (triangle inequality); computed in double from max/min and top-two
// reductions, so the value does not depend on the order of the particles.
//
// In float the box extremes are reduced as unsigned keys that order like
// the values (sign-magnitude to offset binary: negative values inverted,
// positive ones with the top bit set; -0 sorts below +0, which changes no
// midpoint), so every reduction step is one DPP-fused integer min; maxima
// are minima of the inverted keys.  The top two r^2 (non-negative doubles,
// whose bit patterns order like their values) are found as the wave maximum
// of the high words, then of the low words among the lanes holding that
// high word; the second one the same way over every lane's largest value,
// except its second largest on the first lane holding the maximum.
__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ float from_order_key(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

// Maximum of non-negative doubles over the cell's lanes (exact, as 64-bit
// patterns).
template <int T>
__device__ __forceinline__ double cell_max_nonneg(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t hi = (uint32_t)(b >> 32), lo = (uint32_t)b;
    const uint32_t hmax = ~cell_min_u32<T>(~hi);
    const uint32_t lmax = ~cell_min_u32<T>(hi == hmax ? ~lo : 0xFFFFFFFFu);
    return __longlong_as_double((long long)(((uint64_t)hmax << 32) | lmax));
}

// Running minima of the velocity keys of one particle (box[0..2]: the keys,
// box[3..5]: the inverted keys), the first pass of the FP32 bound taken
// elsewhere (the gather of a walled cell has the velocities in registers).
// (a native vector type, so that it is passed in registers, not on the stack)
typedef uint32_t BoxKeys __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void box_keys_add(BoxKeys &box, float a, float b, float c) {
    const uint32_t ka = order_key(a), kb = order_key(b), kc = order_key(c);
    box[0] = min((uint32_t)box[0], ka); box[3] = min((uint32_t)box[3], ~ka);
    box[1] = min((uint32_t)box[1], kb); box[4] = min((uint32_t)box[4], ~kb);
    box[2] = min((uint32_t)box[2], kc); box[5] = min((uint32_t)box[5], ~kc);
}

// With SUMS the pass over r^2 also adds this thread's particles into the
// seven first and second moments sums[0..6] (sx, sy, sz, sxx, syy, szz, sxy),
// in the thread's particle order.
// (use_box: box holds this thread's key minima of the cell, already taken;
// FP32 only; the first pass over the cell is then skipped.)
template <typename R, typename View, int T = 64, bool SUMS = false>
__device__ double exact_bound(const View &v, uint32_t N, double &r_top, GroupScratch *gs = nullptr,
                              double *mid = nullptr, double *sums = nullptr, bool use_box = false,
                              BoxKeys box = BoxKeys{}) {
    const uint32_t tid = cell_tid<T>();
    double m0, m1, m2;
    if constexpr (sizeof(R) == 4) {
        uint32_t lo0 = ~0u, lo1 = ~0u, lo2 = ~0u, nh0 = ~0u, nh1 = ~0u, nh2 = ~0u;  // min keys, min inverted keys
        if (use_box) {
            lo0 = box[0]; lo1 = box[1]; lo2 = box[2];
            nh0 = box[3]; nh1 = box[4]; nh2 = box[5];
        } else {
            for (uint32_t r = tid; r < N; r += T) {
                R a, b, c;
                v.get(r, a, b, c);
                const uint32_t ka = order_key(a), kb = order_key(b), kc = order_key(c);
                lo0 = min(lo0, ka); nh0 = min(nh0, ~ka);
                lo1 = min(lo1, kb); nh1 = min(nh1, ~kb);
                lo2 = min(lo2, kc); nh2 = min(nh2, ~kc);
            }
        }
        lo0 = cell_min_u32<T>(lo0); lo1 = cell_min_u32<T>(lo1); lo2 = cell_min_u32<T>(lo2);
        nh0 = cell_min_u32<T>(nh0); nh1 = cell_min_u32<T>(nh1); nh2 = cell_min_u32<T>(nh2);
        grp_put<T>(gs, 0, lo0); grp_put<T>(gs, 1, lo1); grp_put<T>(gs, 2, lo2);
        grp_put<T>(gs, 3, nh0); grp_put<T>(gs, 4, nh1); grp_put<T>(gs, 5, nh2);
        grp_sync<T>();
        lo0 = grp_min<T>(gs, 0, lo0); lo1 = grp_min<T>(gs, 1, lo1); lo2 = grp_min<T>(gs, 2, lo2);
        nh0 = grp_min<T>(gs, 3, nh0); nh1 = grp_min<T>(gs, 4, nh1); nh2 = grp_min<T>(gs, 5, nh2);
        m0 = 0.5 * ((double)from_order_key(~nh0) + (double)from_order_key(lo0));
        m1 = 0.5 * ((double)from_order_key(~nh1) + (double)from_order_key(lo1));
        m2 = 0.5 * ((double)from_order_key(~nh2) + (double)from_order_key(lo2));
    } else {
        // box extremes: min and max are exact in the working precision
        R lo0 = (R)INFINITY, lo1 = (R)INFINITY, lo2 = (R)INFINITY;
        R hi0 = -(R)INFINITY, hi1 = -(R)INFINITY, hi2 = -(R)INFINITY;
        for (uint32_t r = tid; r < N; r += T) {
            R a, b, c;
            v.get(r, a, b, c);
            lo0 = fmin(lo0, a); hi0 = fmax(hi0, a);
            lo1 = fmin(lo1, b); hi1 = fmax(hi1, b);
            lo2 = fmin(lo2, c); hi2 = fmax(hi2, c);
        }
        const auto mn = [](R a, R b) { return fmin(a, b); };
        const auto mx = [](R a, R b) { return fmax(a, b); };
        const R inf = (R)INFINITY;
        lo0 = cell_reduce_dpp<T>(lo0, inf, mn); lo1 = cell_reduce_dpp<T>(lo1, inf, mn);
        lo2 = cell_reduce_dpp<T>(lo2, inf, mn);
        hi0 = cell_reduce_dpp<T>(hi0, -inf, mx); hi1 = cell_reduce_dpp<T>(hi1, -inf, mx);
        hi2 = cell_reduce_dpp<T>(hi2, -inf, mx);
        if constexpr (T > 64) {
            grp_putd<T>(gs, 0, (double)lo0); grp_putd<T>(gs, 1, (double)lo1); grp_putd<T>(gs, 2, (double)lo2);
            grp_putd<T>(gs, 3, (double)hi0); grp_putd<T>(gs, 4, (double)hi1); grp_putd<T>(gs, 5, (double)hi2);
            __syncthreads();
#pragma unroll
            for (int w = 0; w < T / 64; ++w) {
                lo0 = fmin(lo0, (R)gs->d[w][0]); lo1 = fmin(lo1, (R)gs->d[w][1]); lo2 = fmin(lo2, (R)gs->d[w][2]);
                hi0 = fmax(hi0, (R)gs->d[w][3]); hi1 = fmax(hi1, (R)gs->d[w][4]); hi2 = fmax(hi2, (R)gs->d[w][5]);
            }
        }
        m0 = 0.5 * ((double)hi0 + (double)lo0);
        m1 = 0.5 * ((double)hi1 + (double)lo1);
        m2 = 0.5 * ((double)hi2 + (double)lo2);
    }
    if (mid) {
        mid[0] = m0;
        mid[1] = m1;
        mid[2] = m2;
    }
    double a1 = 0.0, a2 = 0.0;  // largest, second largest r^2 of this lane
    for (uint32_t r = tid; r < N; r += T) {
        R a, b, c;
        v.get(r, a, b, c);
        const double dx = (double)a - m0, dy = (double)b - m1, dz = (double)c - m2;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        // the top two without branches: a1 = max, a2 = max(a2, the smaller
        // of a1 and r2); a NaN r2 leaves both unchanged
        const double lo = r2 > a1 ? a1 : r2;
        a2 = fmax(a2, lo);
        a1 = fmax(a1, r2);
        if constexpr (SUMS) {
            const double vx = (double)a, vy = (double)b, vz = (double)c;
            sums[0] += vx; sums[1] += vy; sums[2] += vz;
            sums[3] += vx * vx; sums[4] += vy * vy; sums[5] += vz * vz; sums[6] += vx * vy;
        }
    }
    double t1 = cell_max_nonneg<T>(a1);
    const unsigned long long at = cell_ballot<T>(a1 == t1);
    const bool first = cell_lane<T>() == __ffsll((long long)at) - 1;
    double t2 = cell_max_nonneg<T>(first ? a2 : a1);
    if constexpr (T > 64) {
        // top two of the waves' top twos
        grp_putd<T>(gs, 6, t1);
        grp_putd<T>(gs, 7, t2);
        __syncthreads();
        t1 = gs->d[0][6];
        int aw = 0;
#pragma unroll
        for (int w = 1; w < T / 64; ++w)
            if (gs->d[w][6] > t1) { t1 = gs->d[w][6]; aw = w; }
        t2 = 0.0;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) {
            if (w != aw) t2 = fmax(t2, gs->d[w][6]);
            t2 = fmax(t2, gs->d[w][7]);
        }
        __syncthreads();  // the scratch is reused
    }
    r_top = sqrt(t1);
    const double eps = sizeof(R) == 4 ? 0x1.0p-20 : 0x1.0p-50;
    return (sqrt(t1) + sqrt(t2)) * (1.0 + eps);
}

// The largest pair speed of the cell by brute force (lane r takes rows
// r, r + 64, ...), times the same rounding margin as the bound.
template <typename R, typename View, int T = 64>
__device__ double pair_diameter(const View &v, uint32_t N, GroupScratch *gs = nullptr) {
    double best = 0.0;
    for (uint32_t r = cell_tid<T>(); r < N; r += T) {
        R x, y, z;
        v.get(r, x, y, z);
        for (uint32_t t = r + 1; t < N; ++t) {
            R x2, y2, z2;
            v.get(t, x2, y2, z2);
            const double dx = (double)x - (double)x2, dy = (double)y - (double)y2, dz = (double)z - (double)z2;
            const double g2 = (dx * dx + dy * dy) + dz * dz;
            best = g2 > best ? g2 : best;
        }
    }
    best = cell_max_t<T>(best);
    if constexpr (T > 64) {
        grp_putd<T>(gs, 0, best);
        __syncthreads();
#pragma unroll
        for (int w = 0; w < T / 64; ++w) best = fmax(best, gs->d[w][0]);
        __syncthreads();  // the scratch is reused
    }
    const double eps = sizeof(R) == 4 ? 0x1.0p-20 : 0x1.0p-50;
    return sqrt(best) * (1.0 + eps);
}

// Uniform direction (Marsaglia 1972) from blocks 1, 2, ... of candidate k's
// PAIR stream; one attempt per block in double (u from words 0-1, v from
// words 2-3), two in float (words 0, 1, then words 2, 3).  The first
// successful attempt gives the direction; after 64 blocks without one it is
// (0, 0, 1).
template <typename R>
__device__ __forceinline__ bool marsaglia_block(const u32x4 &r, R &tx, R &ty, R &tz) {
#pragma unroll
    for (int a = 0; a < (sizeof(R) == 4 ? 2 : 1); ++a) {
        R u, v;
        if (sizeof(R) == 4) {
            u = (R)2 * (R)unif24(r.v[2 * a]) - (R)1;
            v = (R)2 * (R)unif24(r.v[2 * a + 1]) - (R)1;
        } else {
            u = (R)2 * (R)unif53(r.v[0], r.v[1]) - (R)1;
            v = (R)2 * (R)unif53(r.v[2], r.v[3]) - (R)1;
        }
        const R s = u * u + v * v;
        if (s < (R)1 && s > (R)0) {
            const R h = sqrt((R)1 - s);
            tx = ((R)2 * u) * h;
            ty = ((R)2 * v) * h;
            tz = (R)1 - (R)2 * s;
            return true;
        }
    }
    return false;
}

// Lanes with `pending` set try blocks first, first + 1, ... (first may differ
// between lanes; blocks before it are known to have failed) and receive the
// direction; the other lanes keep their values.
template <typename R>
__device__ __forceinline__ void direction(bool pending, uint32_t first, uint32_t k, uint32_t cell, uint32_t step,
                                          uint32_t k0, uint32_t k1, R &nx, R &ny, R &nz) {
    if (!__ballot(pending)) return;
    R tx = (R)0, ty = (R)0, tz = (R)1;
    bool want = pending;
    for (uint32_t it = 0; it < 64; ++it) {
        const uint32_t blk = first + it;
        if (want && blk > 64) want = false;  // no success in 64 blocks: (0, 0, 1)
        if (!__ballot(want)) break;
        if (want && marsaglia_block<R>(draw(k, kTagPair, blk, cell, step, k0, k1), tx, ty, tz)) want = false;
    }
    if (pending) {
        nx = tx;
        ny = ty;
        nz = tz;
    }
}

// Variable-soft-sphere collision of the pair (a, b) (Koura & Matsumoto 1991):
// the relative velocity g = a - b keeps its length and turns by the angle chi
// with cos chi = 2 B^(1/alpha) - 1 about g, at azimuth eps; the mean velocity
// is kept.  B and eps come from the pair's isotropic unit vector n:
// B = (1 + n_z) / 2, (cos eps, sin eps) = (n_x, n_y) / |(n_x, n_y)|.  The turn
// is taken in the frame of g spanned by the unit normals
// (h, -g_x g_y / h, -g_x g_z / h) / |g| and (0, g_z, -g_y) / h,
// h = |(g_y, g_z)| (Bird's component form), or the y and z axes when h = 0.
// Double throughout, in a fixed order; the new velocities are rounded to R.
template <typename R>
__device__ __forceinline__ void vss_pair(R ax, R ay, R az, R bx, R by, R bz, R nx, R ny, R nz, double inv_alpha,
                                         R &oax, R &oay, R &oaz, R &obx, R &oby, R &obz) {
    const double gx = (double)ax - (double)bx, gy = (double)ay - (double)by, gz = (double)az - (double)bz;
    const double g = sqrt((gx * gx + gy * gy) + gz * gz);
    const double cchi = 2.0 * vhs_pow(0.5 * (1.0 + (double)nz), inv_alpha) - 1.0;
    const double s2 = 1.0 - cchi * cchi;
    const double schi = s2 > 0.0 ? sqrt(s2) : 0.0;
    const double ex = (double)nx, ey = (double)ny;
    const double rho2 = ex * ex + ey * ey;
    double ce = 1.0, se = 0.0;
    if (rho2 > 0.0) {
        const double rho = sqrt(rho2);
        ce = ex / rho;
        se = ey / rho;
    }
    const double h2 = gy * gy + gz * gz;
    double px, py, pz;
    if (h2 > 0.0) {
        const double h = sqrt(h2);
        px = cchi * gx + (schi * se) * h;
        py = cchi * gy + schi * (((ce * g) * gz - (se * gx) * gy) / h);
        pz = cchi * gz - schi * (((ce * g) * gy + (se * gx) * gz) / h);
    } else {
        px = cchi * gx;
        py = (schi * ce) * g;
        pz = (schi * se) * g;
    }
    const double mx = 0.5 * ((double)ax + (double)bx), my = 0.5 * ((double)ay + (double)by),
                 mz = 0.5 * ((double)az + (double)bz);
    const double tx = 0.5 * px, ty = 0.5 * py, tz = 0.5 * pz;
    oax = (R)(mx + tx);
    oay = (R)(my + ty);
    oaz = (R)(mz + tz);
    obx = (R)(mx - tx);
    oby = (R)(my - ty);
    obz = (R)(mz - tz);
}

// Random draws of the fresh candidates (lanes with `fresh` set): the pair
// (i, j) and acceptance number U from block 0 of the candidate's PAIR
// stream, the scattering direction from blocks 1, 2, ...
//
// The fresh candidates of a window are consecutive, kf .. kf + m - 1, on a
// cyclic run of lanes (candidate k lives on lane k mod 64).  With m <= 32 the
// whole wave computes blocks for them at once: lane b m + t computes block b
// of candidate kf + t (and its direction attempts when b >= 1), so one pass
// yields block 0 and the first 64 / m - 1 direction blocks of every
// candidate; each candidate's lane then collects block 0 and the first
// successful direction block by lane shuffles.  Candidates whose computed
// blocks all fail continue one block at a time.  Same draws, same order of
// attempts: the result equals the per-candidate definition.
template <typename R>
__device__ __forceinline__ void draw_candidates(bool fresh, uint32_t k, uint32_t N, uint32_t cell, uint32_t step,
                                                uint32_t k0, uint32_t k1, uint32_t &i, uint32_t &j, R &U, R &nx,
                                                R &ny, R &nz) {
    const unsigned long long fm = __ballot(fresh);
    if (!fm) return;
    const uint32_t m = (uint32_t)__popcll(fm);
    // first lane of the run: fresh, with its predecessor not fresh
    const unsigned long long starts = fm & ~((fm << 1) | (fm >> 63));
    if (m > 32 || __popcll(starts) != 1) {
        if (fresh) {
            const u32x4 r = draw(k, kTagPair, 0, cell, step, k0, k1);
            i = scale_index(r.v[0], N);
            j = scale_index(r.v[1], N - 1);
            j += (j >= i) ? 1u : 0u;
            U = sizeof(R) == 4 ? (R)unif24(r.v[2]) : (R)unif53(r.v[2], r.v[3]);
        }
        direction<R>(fresh, 1u, k, cell, step, k0, k1, nx, ny, nz);
        return;
    }
    const uint32_t lane = (uint32_t)lane_id();
    const int l0 = __ffsll((long long)starts) - 1;
    const uint32_t kf = (uint32_t)__builtin_amdgcn_readlane((int)k, l0);
    // x / m as (x * ceil(2^16 / m)) >> 16, exact for x < 64 and m <= 64
    const uint32_t inv = (65536u + m - 1u) / m;
    const uint32_t b = (lane * inv) >> 16;
    const uint32_t t = lane - b * m;
    const u32x4 r = draw(kf + t, kTagPair, b, cell, step, k0, k1);
    R tx = (R)0, ty = (R)0, tz = (R)1;
    const bool ok = b >= 1u && marsaglia_block<R>(r, tx, ty, tz);
    const uint32_t own = fresh ? k - kf : 0u;  // this lane's candidate offset
    const uint32_t w0 = (uint32_t)__shfl((int)r.v[0], (int)own, 64);
    const uint32_t w1 = (uint32_t)__shfl((int)r.v[1], (int)own, 64);
    const uint32_t w2 = (uint32_t)__shfl((int)r.v[2], (int)own, 64);
    const uint32_t w3 = sizeof(R) == 8 ? (uint32_t)__shfl((int)r.v[3], (int)own, 64) : 0u;
    if (fresh) {
        i = scale_index(w0, N);
        j = scale_index(w1, N - 1);
        j += (j >= i) ? 1u : 0u;
        U = sizeof(R) == 4 ? (R)unif24(w2) : (R)unif53(w2, w3);
    }
    bool want = fresh;
    for (uint32_t blk = 1; blk < 64; ++blk) {
        const uint32_t src = blk * m + own;
        const bool avail = want && src < 64u;
        if (!__ballot(avail)) break;
        const int s = (int)(src & 63u);
        const int okb = __shfl((int)ok, s, 64);
        const R ax = __shfl(tx, s, 64), ay = __shfl(ty, s, 64), az = __shfl(tz, s, 64);
        if (avail && okb) {
            nx = ax;
            ny = ay;
            nz = az;
            want = false;
        }
    }
    // blocks 1 .. (63 - own) / m were computed for this candidate
    direction<R>(want, (((63u - own) * inv) >> 16) + 1u, k, cell, step, k0, k1, nx, ny, nz);
}

// The NTC candidate loop of one cell in conflict-free wave batches.
//
// The wave holds a window of up to 64 consecutive candidates, candidate k on
// lane k mod 64.  Velocities: only accepted candidates write them, so the
// window commits every candidate before the first one that reads a particle
// an earlier accepted candidate of the window has changed (marks: atomic min
// of the candidate index).  A candidate's random draws (pair, acceptance
// number, scattering direction) are functions of its index only and are
// computed once, however often it waits.
//
// Without weights, committed lanes take the candidate 64 later at once (the
// window rolls).  With importance weights every candidate writes the weights
// of its pair, and the weights never feed back into the velocity decisions:
// the window stays inside one generation of 64 candidates (64 g .. 64 g + 63)
// until all of them are committed, then the generation's weight updates are
// replayed in rounds: a round applies every pending candidate that no
// earlier pending candidate shares a particle with.  Both give exactly the
// sequential result.

// Velocity window over the live candidates (k in [kb, wend)); returns the
// first uncommitted candidate and sets `commit` and `accept` per lane.
template <typename R, typename View, int T>
__device__ __forceinline__ uint32_t velocity_window(const View &v, bool live, uint32_t k, uint32_t kb, uint32_t wend,
                                                    uint32_t i, uint32_t j, R U, R nx, R ny, R nz, R gm, R gm2,
                                                    double gmax2, double om1, double inv_alpha, int molecule,
                                                    bool &commit,
                                                    bool &accept, R &g2_out, double &pacc, uint32_t &acc,
                                                    uint32_t &over, GroupScratch *gs) {
    R ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0, g2 = 0;
    accept = false;
    pacc = 1.0;
    if (live) {
        v.get(i, ax, ay, az);
        v.get(j, bx, by, bz);
        const R dx = ax - bx, dy = ay - by, dz = az - bz;
        g2 = (dx * dx + dy * dy) + dz * dz;
        if (molecule == DSMC_MAXWELL) {
            accept = true;
        } else if (molecule == DSMC_VHS || molecule == DSMC_VSS) {
            // accept with probability (g / g_max)^(2 - 2 omega), in double
            pacc = vhs_pow((double)g2 / gmax2, om1);
            accept = (double)U < pacc;
        } else {
            const R a = U * gm;
            accept = (a * a) < g2;
        }
    }
    const bool writer = live && accept;
    if (writer) {
        atomicMin(v.own(i), k);
        atomicMin(v.own(j), k);
    }
    __syncthreads();
    const bool bad = live && (v.read_own(i) < k || v.read_own(j) < k);
    // first candidate that must wait; the window ends there (or at wend)
    uint32_t kend = cell_min_u32<T>(bad ? k : 0xFFFFFFFFu);
    grp_put<T>(gs, 0, kend);
    __syncthreads();
    kend = grp_min<T>(gs, 0, kend);
    kend = kend < wend ? kend : wend;
    commit = live && k < kend;
    if (writer) {
        v.clear_own(i);
        v.clear_own(j);
    }
    const bool coll = commit && accept;
    if (coll) {
        if (molecule == DSMC_VSS) {
            R oax, oay, oaz, obx, oby, obz;
            vss_pair<R>(ax, ay, az, bx, by, bz, nx, ny, nz, inv_alpha, oax, oay, oaz, obx, oby, obz);
            v.put(i, oax, oay, oaz);
            v.put(j, obx, oby, obz);
        } else {
            const R g = sqrt(g2);
            const R hg = (R)0.5 * g;
            const R mx = (R)0.5 * (ax + bx), my = (R)0.5 * (ay + by), mz = (R)0.5 * (az + bz);
            const R tx = hg * nx, ty = hg * ny, tz = hg * nz;
            v.put(i, mx + tx, my + ty, mz + tz);
            v.put(j, mx - tx, my - ty, mz - tz);
        }
    }
    if (molecule != DSMC_MAXWELL && commit && g2 > gm2) over++;
    acc += (uint32_t)__popcll(cell_ballot<T>(coll));
    g2_out = g2;
    __syncthreads();
    return kend;
}

template <typename R, bool VR, typename View, int T = 64>
__device__ void ntc_loop(const View &v, uint32_t N, double gmax, uint32_t M, uint32_t cell,
                         uint32_t step, uint32_t k0, uint32_t k1, int molecule, double om1, double inv_alpha,
                         uint32_t &n_acc,
                         uint32_t &n_over, GroupScratch *gs = nullptr) {
    constexpr uint32_t W = (uint32_t)T;  // candidates per window (one per thread)
    const R gm = (R)gmax;
    const R gm2 = gm * gm;
    const double gmax2 = gmax * gmax;
    uint32_t kb = 0, acc = 0, over = 0;
    uint32_t k = cell_tid<T>();  // candidate held by this thread; k in [kb, kb + W)
    bool fresh = true;   // its draws are still to be computed
    bool done = false;   // committed, waiting for the end of its generation (weights)
    bool acc_k = false;  // committed candidate's acceptance (weights)
    double p = 1.0;      // and its g / g_max (weights, rejected candidates)
    uint32_t i = 0, j = 0;
    R U = (R)0, nx = (R)0, ny = (R)0, nz = (R)1;
    uint32_t g0 = 0;     // first candidate of the current generation (weights)
    bool wpend = false;  // half-wave cell: generation complete, weights not yet replayed
    while (kb < M || wpend) {
        const bool act = k < M;
        const bool draw_now = act && fresh;
        if constexpr (T == 64) {
            draw_candidates<R>(draw_now, k, N, cell, step, k0, k1, i, j, U, nx, ny, nz);
        } else {
            if (draw_now) {
                const u32x4 r = draw(k, kTagPair, 0, cell, step, k0, k1);
                i = scale_index(r.v[0], N);
                j = scale_index(r.v[1], N - 1);
                j += (j >= i) ? 1u : 0u;
                U = sizeof(R) == 4 ? (R)unif24(r.v[2]) : (R)unif53(r.v[2], r.v[3]);
            }
            direction<R>(draw_now, 1u, k, cell, step, k0, k1, nx, ny, nz);
        }
        fresh = fresh && !act;
        const uint32_t gend = M - g0 > W ? g0 + W : M;
        const uint32_t wend = VR ? gend : (M - kb > W ? kb + W : M);
        bool commit, accept;
        R g2;
        double pacc;
        const uint32_t kend = velocity_window<R, View, T>(v, act && !done, k, kb, wend, i, j, U, nx, ny, nz, gm, gm2,
                                                          gmax2, om1, inv_alpha, molecule, commit, accept, g2, pacc,
                                                          acc, over, gs);
        kb = kend;
        if (!VR) {
            // committed threads move on to the candidate W later
            if (commit) {
                k += W;
                fresh = true;
            }
            continue;
        }
        if (commit) {
            done = true;
            acc_k = accept;
            p = (!accept && molecule != DSMC_MAXWELL)
                    ? ((molecule == DSMC_VHS || molecule == DSMC_VSS) ? pacc : sqrt((double)g2) / gmax)
                    : 1.0;
        }
        // (half-wave cells: a half whose generation is complete waits, its
        // lanes idle in the windows, until the other half's is complete too,
        // so that the wave replays both cells' weights in one set of rounds;
        // a half that has left the loop does not hold the other back)
        if constexpr (T == 32) {
            wpend = kb >= gend;
            if (__ballot(kb < gend) != 0ull) continue;
            wpend = false;
        } else {
            if (kb < gend) continue;
        }
        // generation complete: importance weights (Al-Mohssen & Hadjiconstantinou
        // 2010) of its candidates, in candidate order: accepted -> both W_i W_j;
        // rejected -> W_i (1 - p W_j) / (1 - p), p = g / g_max
        const bool mine = act && k < gend;  // this lane's candidate belongs to the generation
        bool pend = mine;
        for (;;) {
            bool any = cell_ballot<T>(pend) != 0ull;
            if constexpr (T > 64) {
                grp_put<T>(gs, 1, any ? 1u : 0u);
                __syncthreads();
                any = grp_sum<T>(gs, 1, 0u) != 0u;
            }
            if (!any) break;
            // a pending candidate is ready when no earlier pending candidate
            // touches its particles; ready candidates touch disjoint pairs and
            // every particle sees its updates in candidate order
            if (pend) {
                atomicMin(v.own(i), k);
                atomicMin(v.own(j), k);
            }
            __syncthreads();
            const bool ready = pend && v.read_own(i) == k && v.read_own(j) == k;
            __syncthreads();
            if (pend) {
                v.clear_own(i);
                v.clear_own(j);
            }
            if (ready) {
                const double wa = (double)v.getw(i), wb = (double)v.getw(j);
                if (acc_k) {
                    const double ab = wa * wb;
                    v.putw(i, (R)ab);
                    v.putw(j, (R)ab);
                } else {
                    const double q = 1.0 - p;
                    if (q > 0.0) {
                        v.putw(i, (R)((wa * (1.0 - p * wb)) / q));
                        v.putw(j, (R)((wb * (1.0 - p * wa)) / q));
                    }
                }
            }
            pend = pend && !ready;
            __syncthreads();
        }
        // next generation
        if (mine) {
            k += W;
            fresh = true;
            done = false;
        }
        g0 = gend;
    }
    // acc counts this wave's lanes; the workgroup adds its waves
    over = cell_sum_u32<T>(over);
    grp_put<T>(gs, 2, acc);
    grp_put<T>(gs, 3, over);
    grp_sync<T>();
    n_acc = grp_sum<T>(gs, 2, acc);
    n_over = grp_sum<T>(gs, 3, over);
    grp_sync<T>();
}

// ------------------------------------------------- weight re-estimation
// Importance-weight re-estimation of one cell (reconstruction step after
// Al-Mohssen & Hadjiconstantinou 2010, in this project's reading): the
// deviations d_i = W_i - 1 are replaced by their least-squares projection
// onto the 13 functions of v = c / sqrt(T0)
//   phi = (1, v_x, v_y, v_z, v_x^2, v_y^2, v_z^2, v_x v_y, v_x v_z, v_y v_z,
//          v_x |v|^2, v_y |v|^2, v_z |v|^2),
// whose raw-velocity counterparts are the functions the cell samples: every
// sampled weighted moment keeps its value, unit weights stay exactly 1.  The
// normal equations G a = b, G = sum phi phi^T, b = sum d phi, are solved by
// Gauss-Jordan elimination in double (in the elimination order the pivots
// are those of the Cholesky factorisation); a cell of fewer than 26
// particles, or one whose k-th pivot is not above 1e-12 G_kk, keeps its
// weights.
//
// G is assembled from 51 monomial sums: the monomials of degree 0-4 (index
// 0 for 1; 1-3 for v_x, v_y, v_z; 4-9 for xx yy zz xy xz yz; 10-19 and 20-34
// for degrees 3 and 4 in lexicographic order of the exponents), the degree-3
// monomials times |v|^2 (35-44) and xx yy zz xy xz yz times |v|^4 (45-50);
// b takes 13 more sums (51-63).  The sums are taken in four passes of 16
// over the cell's particles (0-15, 16-31, 32-47, 48-63), each reduced by
// recursive halving, so that few registers are live at a time.
constexpr int kReMin = 26;      // smallest cell that is re-estimated
constexpr int kReBasis = 13;

struct GramTable {
    uint8_t n[kReBasis][kReBasis];     // number of monomial sums of entry G_rc (1 or 3)
    uint8_t t[kReBasis][kReBasis][3];  // their indices
};

// exponents (x, y, z) and power of |v|^2 of the basis functions
constexpr int kReExp[kReBasis][4] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {2, 0, 0, 0},
                                     {0, 2, 0, 0}, {0, 0, 2, 0}, {1, 1, 0, 0}, {1, 0, 1, 0}, {0, 1, 1, 0},
                                     {1, 0, 0, 1}, {0, 1, 0, 1}, {0, 0, 1, 1}};

// rank of the exponents (i, j, n - i - j) among the monomials of degree n in
// lexicographic (descending) order
constexpr int lex_rank(int n, int i, int j) {
    int r = 0;
    for (int ii = i + 1; ii <= n; ++ii) r += n - ii + 1;
    return r + (n - i - j);
}
constexpr int deg2_slot(int i, int j, int k) {
    return i == 2 ? 0 : j == 2 ? 1 : k == 2 ? 2 : (i == 1 && j == 1) ? 3 : (i == 1 && k == 1) ? 4 : 5;
}
constexpr int mono_index(int i, int j, int k) {
    const int n = i + j + k;
    return n == 0 ? 0 : n == 1 ? (i ? 1 : j ? 2 : 3) : n == 2 ? 4 + deg2_slot(i, j, k)
         : n == 3 ? 10 + lex_rank(3, i, j) : 20 + lex_rank(4, i, j);
}
constexpr GramTable make_gram_table() {
    GramTable g{};
    for (int r = 0; r < kReBasis; ++r)
        for (int c = 0; c < kReBasis; ++c) {
            const int i = kReExp[r][0] + kReExp[c][0], j = kReExp[r][1] + kReExp[c][1],
                      k = kReExp[r][2] + kReExp[c][2], t = kReExp[r][3] + kReExp[c][3];
            if (t == 0) {
                g.n[r][c] = 1;
                g.t[r][c][0] = (uint8_t)mono_index(i, j, k);
            } else if (t == 2) {
                g.n[r][c] = 1;
                g.t[r][c][0] = (uint8_t)(45 + deg2_slot(i, j, k));
            } else if (i + j + k == 3) {
                g.n[r][c] = 1;
                g.t[r][c][0] = (uint8_t)(35 + lex_rank(3, i, j));
            } else {  // |v|^2 = v_x^2 + v_y^2 + v_z^2
                g.n[r][c] = 3;
                g.t[r][c][0] = (uint8_t)mono_index(i + 2, j, k);
                g.t[r][c][1] = (uint8_t)mono_index(i, j + 2, k);
                g.t[r][c][2] = (uint8_t)mono_index(i, j, k + 2);
            }
        }
    return g;
}
__constant__ const GramTable kGram = make_gram_table();

struct Reest {
    bool on;
    double sc;            // 1 / sqrt(T0)
    double a[kReBasis];   // coefficients of the new deviation
};

// Sum q[0..15] over the cell's threads: on return lane L of every wave holds
// the total of q[L >> 2] (the waves of a workgroup added in a fixed order);
// a half-wave cell (T = 32): cell lane l the total of q[l >> 1].
template <int T>
__device__ __forceinline__ double cell_sum16(double (&q)[16], GroupScratch *gs) {
    double t = cell_sum_many<T == 32 ? 32 : 64, 16>(q);
    if constexpr (T > 64) {
        const int lane = lane_id();
        if ((lane & 3) == 0) gs->d[threadIdx.x >> 6][lane >> 2] = t;
        __syncthreads();
        t = gs->d[0][lane >> 2];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) t += gs->d[w][lane >> 2];
        __syncthreads();  // the scratch is reused
    }
    return t;
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One pass of the Gram sums: PASS 0-3 accumulates sums 16 PASS .. 16 PASS + 15.
template <int PASS, typename R, typename View, int T>
__device__ __forceinline__ double gram_pass(const View &v, uint32_t N, double sc, GroupScratch *gs) {
    double q[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) q[u] = 0.0;
    for (uint32_t r = cell_tid<T>(); r < N; r += T) {
        R a, b, c;
        v.get(r, a, b, c);
        const double x = (double)a * sc, y = (double)b * sc, z = (double)c * sc;
        const double xx = x * x, yy = y * y, zz = z * z;
        if constexpr (PASS == 0) {  // 1, x y z, xx yy zz xy xz yz, xxx xxy xxz xyy xyz xzz
            const double xy = x * y;
            q[0] += 1.0; q[1] += x; q[2] += y; q[3] += z;
            q[4] += xx; q[5] += yy; q[6] += zz; q[7] += xy; q[8] = fma(x, z, q[8]); q[9] = fma(y, z, q[9]);
            q[10] = fma(xx, x, q[10]); q[11] = fma(xx, y, q[11]); q[12] = fma(xx, z, q[12]);
            q[13] = fma(xy, y, q[13]); q[14] = fma(xy, z, q[14]); q[15] = fma(x, zz, q[15]);
        } else if constexpr (PASS == 1) {  // yyy yyz yzz zzz, degree 4 (first 12)
            const double xxx = xx * x, xxy = xx * y, xxz = xx * z, xyy = x * yy, yyy = yy * y;
            q[0] += yyy; q[1] = fma(yy, z, q[1]); q[2] = fma(y, zz, q[2]); q[3] = fma(zz, z, q[3]);
            q[4] = fma(xxx, x, q[4]); q[5] = fma(xxx, y, q[5]); q[6] = fma(xxx, z, q[6]);
            q[7] = fma(xxy, y, q[7]); q[8] = fma(xxy, z, q[8]); q[9] = fma(xxz, z, q[9]);
            q[10] = fma(xyy, y, q[10]); q[11] = fma(xyy, z, q[11]); q[12] = fma(x * y, zz, q[12]);
            q[13] = fma(x * zz, z, q[13]); q[14] = fma(yyy, y, q[14]); q[15] = fma(yyy, z, q[15]);
        } else if constexpr (PASS == 2) {  // yyzz yzzz zzzz, degree 3 times s, xx yy zz times s^2
            const double s = (xx + yy) + zz;
            q[0] = fma(yy, zz, q[0]); q[1] = fma(y * z, zz, q[1]); q[2] = fma(zz, zz, q[2]);
            q[3] = fma(xx * x, s, q[3]); q[4] = fma(xx * y, s, q[4]); q[5] = fma(xx * z, s, q[5]);
            q[6] = fma(x * yy, s, q[6]); q[7] = fma((x * y) * z, s, q[7]); q[8] = fma(x * zz, s, q[8]);
            q[9] = fma(yy * y, s, q[9]); q[10] = fma(yy * z, s, q[10]); q[11] = fma(y * zz, s, q[11]);
            q[12] = fma(zz * z, s, q[12]);
            const double s2 = s * s;
            q[13] = fma(xx, s2, q[13]); q[14] = fma(yy, s2, q[14]); q[15] = fma(zz, s2, q[15]);
        } else {  // xy xz yz times s^2, then b: d phi_k
            const double s = (xx + yy) + zz, s2 = s * s;
            const double d = (double)v.getw(r) - 1.0;
            const double dx = d * x, dy = d * y, dz = d * z;
            q[0] = fma(x * y, s2, q[0]); q[1] = fma(x * z, s2, q[1]); q[2] = fma(y * z, s2, q[2]);
            q[3] += d; q[4] += dx; q[5] += dy; q[6] += dz;
            q[7] = fma(dx, x, q[7]); q[8] = fma(dy, y, q[8]); q[9] = fma(dz, z, q[9]);
            q[10] = fma(dx, y, q[10]); q[11] = fma(dx, z, q[11]); q[12] = fma(dy, z, q[12]);
            q[13] = fma(dx, s, q[13]); q[14] = fma(dy, s, q[14]); q[15] = fma(dz, s, q[15]);
        }
    }
    return cell_sum16<T>(q, gs);
}

// Normal equations of a half-wave cell (T = 32) from the four passes' sums
// (pass p's sum s on cell lanes 2 s and 2 s + 1): the same Gauss-Jordan
// elimination as the one-wave form, with two lanes per row: cell lane 2 r + q
// holds the entries (r, q + 2 j), j = 0..6 (column 13 is b).  The 64 sums
// are staged in lds[0..64) (the half's owner marks, free once the candidates
// are done), from which every lane assembles its entries; the solution goes
// to lds[0..13).  Returns false, writing no solution, if the cell keeps its
// weights.
__device__ __forceinline__ bool solve_half(double t0, double t1, double t2, double t3, double *lds) {
    const int cl = lane_id() & 31;
    const int row = cl >> 1, qc = cl & 1;
    // sum g = 16 p + s of pass p (p = qc and 2 + qc on cell lane 2 s + qc)
    lds[16 * qc + row] = qc ? t1 : t0;
    lds[16 * (2 + qc) + row] = qc ? t3 : t2;
    __syncthreads();
    const bool has_row = row < kReBasis;
    const int rr = has_row ? row : 0;
    double M[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int col = qc + 2 * j;
        double e = 0.0;
        if (has_row && col < kReBasis) {
            e = lds[kGram.t[rr][col][0]];
            if (kGram.n[rr][col] == 3) e = (e + lds[kGram.t[rr][col][1]]) + lds[kGram.t[rr][col][2]];
        } else if (has_row && col == kReBasis) {
            e = lds[51 + rr];
        }
        M[j] = e;
    }
    // this lane's original diagonal entry (row r: column r, slot r >> 1 on lane 2 r + (r & 1))
    double mdiag = M[0];
#pragma unroll
    for (int j = 1; j < 7; ++j) mdiag = (row >> 1) == j ? M[j] : mdiag;
    const double dg = (has_row && qc == (row & 1)) ? mdiag : 0.0;
    // Step k reads only columns k and up, so the row-k entries of columns
    // below k (eliminated) are neither broadcast nor updated; slot j holds
    // column qc + 2 j, needed by some lane when 2 j + 1 > k.  The pivot and
    // M[r][k] sit on lane 2 r + (k & 1) of each row's pair and reach its
    // partner by a DPP pair broadcast; the pivot test runs on the pivot's
    // own lane (the lane that holds the original G_kk).
    bool ok_lane = true;
#pragma unroll
    for (int k = 0; k < kReBasis; ++k) {
        double bk[7];
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (2 * j + 1 > k || j == (k >> 1)) bk[j] = cell_shfl<32>(M[j], 2 * k + qc);
        const double own = M[k >> 1], rowk = bk[k >> 1];
        const double piv = (k & 1) ? quad_perm_f64<0xF5>(rowk) : quad_perm_f64<0xA0>(rowk);
        const double mrk = (k & 1) ? quad_perm_f64<0xF5>(own) : quad_perm_f64<0xA0>(own);
        if (cl == 2 * k + (k & 1)) ok_lane = piv > 1e-12 * dg;
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        const double f = row == k ? 1.0 - inv : mrk * inv;
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (2 * j + 1 > k || j == (k >> 1)) M[j] = fma(-f, bk[j], M[j]);
    }
    // a pivot not above 1e-12 G_kk: the cell keeps its weights
    if (cell_ballot<32>(!ok_lane) != 0ull) return false;
    // solution: column 13 (cell lane 2 r + 1, slot 6); every lane has read
    // the sums it needed (the reads above precede these writes in the wave)
    __syncthreads();
    if (has_row && qc == 1) lds[row] = M[6];
    return true;
}

// Coefficients of the re-estimated deviations of the cell (identical on
// every thread), or re.on = false if the cell keeps its weights.
template <typename R, typename View, int T>
__device__ void reestimate_cell(const View &v, uint32_t N, double sc, Reest &re, GroupScratch *gs) {
    re.on = false;
    re.sc = sc;
    const double t0 = gram_pass<0, R, View, T>(v, N, sc, gs);
    const double t1 = gram_pass<1, R, View, T>(v, N, sc, gs);
    const double t2 = gram_pass<2, R, View, T>(v, N, sc, gs);
    const double t3 = gram_pass<3, R, View, T>(v, N, sc, gs);
    // sum g on lane 4 (g mod 16) + g / 16
    const int lane = lane_id();
    const int qb = lane & 3;
    const double sum = qb == 0 ? t0 : (qb == 1 ? t1 : (qb == 2 ? t2 : t3));
    const auto fetch = [&](int g) { return __shfl(sum, 4 * (g & 15) + (g >> 4), 64); };
    // augmented matrix [G | b], four lanes per row: lane 4 r + q holds the
    // entries (r, q + 4 j), j = 0..3 (column 13 is b)
    const int row = lane >> 2, qc = lane & 3;
    const bool has_row = row < kReBasis;
    const int rr = has_row ? row : 0;
    double M[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = qc + 4 * j;
        const int cc = col < kReBasis ? col : 0;
        // every lane takes part in the shuffles; values of lanes without the
        // entry are discarded
        const int nt = kGram.n[rr][cc];
        const double e0 = fetch(col == kReBasis ? 51 + rr : kGram.t[rr][cc][0]);
        const double e1 = fetch(nt == 3 ? kGram.t[rr][cc][1] : 0);
        const double e2 = fetch(nt == 3 ? kGram.t[rr][cc][2] : 0);
        M[j] = (!has_row || col > kReBasis) ? 0.0 : ((col < kReBasis && nt == 3) ? (e0 + e1) + e2 : e0);
    }
    // this lane's original diagonal entry (for the pivot test)
    const int sl = row >> 2;
    const double mdiag = sl == 0 ? M[0] : (sl == 1 ? M[1] : (sl == 2 ? M[2] : M[3]));
    const double dg = (has_row && qc == (row & 3)) ? mdiag : 0.0;
    // Gauss-Jordan: row k is divided by the pivot, every other row r loses
    // M[r][k] / pivot times row k; for row k itself that is the same update
    // with the factor 1 - 1 / pivot.  The reciprocal is the hardware
    // estimate refined by one Newton step.  Step k reads only columns k and
    // up: slot j (column qc + 4 j) is broadcast and updated only when
    // 4 j + 3 > k.  M[r][k] sits on lane 4 r + (k & 3) of the row's quad and
    // reaches the other three by a DPP quad broadcast.
    bool ok = true;
#pragma unroll
    for (int k = 0; k < kReBasis; ++k) {
        const int kl = 4 * k + (k & 3);
        const double piv = readlane_f64(M[k >> 2], kl);
        ok = ok && piv > 1e-12 * readlane_f64(dg, kl);
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        const double own = M[k >> 2];
        const double mrk = (k & 3) == 0 ? quad_perm_f64<0x00>(own)
                         : (k & 3) == 1 ? quad_perm_f64<0x55>(own)
                         : (k & 3) == 2 ? quad_perm_f64<0xAA>(own) : quad_perm_f64<0xFF>(own);
        const double f = row == k ? 1.0 - inv : mrk * inv;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (4 * j + 3 > k) M[j] = fma(-f, __shfl(M[j], 4 * k + qc, 64), M[j]);
    }
    if (!ok) return;  // a pivot not above 1e-12 G_kk: the cell keeps its weights
    // solution: column 13 (lane 4 r + 1, slot 3)
#pragma unroll
    for (int r = 0; r < kReBasis; ++r) re.a[r] = readlane_f64(M[3], 4 * r + 1);
    re.on = true;
}

// New weight of a particle from the re-estimated deviation (k: the thirteen
// coefficients, in registers or in LDS).
template <typename R, typename Coef>
__device__ __forceinline__ R reestimated_weight(const Coef &k, double sc, R a, R b, R c) {
    const double x = (double)a * sc, y = (double)b * sc, z = (double)c * sc;
    const double s = (x * x + y * y) + z * z;
    double d = k[0];
    d = fma(k[1], x, d); d = fma(k[2], y, d); d = fma(k[3], z, d);
    d = fma(k[4], x * x, d); d = fma(k[5], y * y, d); d = fma(k[6], z * z, d);
    d = fma(k[7], x * y, d); d = fma(k[8], x * z, d); d = fma(k[9], y * z, d);
    d = fma((k[10] * x + k[11] * y) + k[12] * z, s, d);
    return (R)(1.0 + d);
}

// Re-estimate the weights of the cell held by the view (in place), if due.
template <typename R, typename View, int T>
__device__ __forceinline__ void reestimate_weights(const View &v, uint32_t N, double sc, GroupScratch *gs) {
    if constexpr (T == 32) {
        // half-wave cell: the sums and the coefficients in the owner array
        // of its LDS area (the candidates, which use the marks, are done;
        // the two-cell launch gives a cell at least 128 + 4 marks, room for
        // 64 doubles)
        static_assert(View::kInLds, "half-wave cells are staged in LDS");
        double *coef = reinterpret_cast<double *>(v.owner);
        const double t0 = gram_pass<0, R, View, T>(v, N, sc, gs);
        const double t1 = gram_pass<1, R, View, T>(v, N, sc, gs);
        const double t2 = gram_pass<2, R, View, T>(v, N, sc, gs);
        const double t3 = gram_pass<3, R, View, T>(v, N, sc, gs);
        if (!solve_half(t0, t1, t2, t3, coef)) return;
        __syncthreads();
        const double *k = coef;
        for (uint32_t r = cell_tid<T>(); r < N; r += T) {
            R a, b, c;
            v.get(r, a, b, c);
            v.putw(r, reestimated_weight<R>(k, sc, a, b, c));
        }
        __syncthreads();
        return;
    }
    Reest re;
    reestimate_cell<R, View, T>(v, N, sc, re, gs);
    if (!re.on) return;
    for (uint32_t r = cell_tid<T>(); r < N; r += T) {
        R a, b, c;
        v.get(r, a, b, c);
        v.putw(r, reestimated_weight<R>(re.a, re.sc, a, b, c));
    }
    grp_sync<T>();
}

// The running sum a lane owns in the moment reduction, or -1.  Cells in
// global memory: lane L owns sum L.  Cells staged in LDS: the four lanes of
// quad r add up row r (moment r) together, and lane 4 r + h keeps the total
// of set h (h = 0 plain, 1 weighted): sum 13 h + r.  Half-wave cells (T =
// 32, staged in LDS): cell lanes 2 r and 2 r + 1 add up row r, and cell lane
// 2 r + h keeps sum 13 h + r.
template <bool IN_LDS, bool VR, int T = 64>
__device__ __forceinline__ int owned_sum(int lane) {
    if (!IN_LDS) return lane < (VR ? kNsum : 13) ? lane : -1;
    if constexpr (T == 32) {
        const int r = lane >> 1, h = lane & 1;
        return (r < 13 && h < (VR ? 2 : 1)) ? 13 * h + r : -1;
    }
    const int r = lane >> 2, h = lane & 3;
    return (r < 13 && h < (VR ? 2 : 1)) ? 13 * h + r : -1;
}

// The cell's running sums and counters.  Without weights they are read at
// the start of the cell's work, so that the final read-modify-write does not
// wait on memory (each lane the sum it owns, lane 0 the counters).  With
// weights they are read at the end: held through the whole cell they would
// take the six registers that let the one-wave kernel run six waves per SIMD.
template <bool ON>
struct CellPrefetch {};
template <>
struct CellPrefetch<true> {
    double sum;
    unsigned long long cand, acc;
};

template <typename R, bool VR, bool IN_LDS, int T = 64>
__device__ __forceinline__ CellPrefetch<!VR> prefetch_cell(const CollideArgs<R> &a, uint32_t cell) {
    CellPrefetch<!VR> pf{};
    if constexpr (!VR) {
        const int lane = cell_lane<T>();
        const int idx = owned_sum<IN_LDS, VR, T>(lane);
        pf.sum = idx >= 0 ? a.sums[(size_t)cell * kNsum + idx] : 0.0;
        pf.cand = 0ull;
        pf.acc = 0ull;
        if (lane == 0) {
            pf.cand = a.counters[2 * (size_t)cell];
            pf.acc = a.counters[2 * (size_t)cell + 1];
        }
    } else {
        (void)a;
        (void)cell;
    }
    return pf;
}

// FP64 moment sums of the post-collision state of one cell, added to the
// running sums; per-cell counters and diagnostics.  Each lane accumulates
// the moments of its particles; the 13 (26 with weights) sums are then
// reduced over the wave.  A cell in global memory reduces by shuffles
// (recursive halving).  A cell staged in LDS writes its velocities and
// weights back to the particle arrays at wb_base during the accumulation,
// and then uses its LDS area (`red`, at least kRedBytes) for a transpose,
// once per set of 13 sums: every lane stores its partial sums as a column,
// the four lanes of quad r add up a quarter of row r each (interleaved
// 16-byte columns, starting at column block r mod 8 so that the rows read
// different banks) and the quad combines its four parts.
template <typename R, bool VR, typename View, int T = 64>
__device__ void sample_cell(const CollideArgs<R> &a, const View &v, uint32_t cell, uint32_t N, uint32_t M,
                            uint32_t acc, uint32_t over, const CellPrefetch<!VR> &pf, double *red,
                            uint32_t wb_base, GroupScratch *gs = nullptr) {
    const int lane = cell_lane<T>();
    const uint32_t tid = cell_tid<T>();
    constexpr int K = VR ? 32 : 16;  // 26 or 13 sums, padded to a power of two
    const int owned = owned_sum<View::kInLds && T <= 64, VR, T>((int)tid);
    const uint32_t idx = (uint32_t)owned;
    const bool writer = owned >= 0;
    const uint32_t ce = bounds_ck(cell, a.n_cells, a.st);
    double *sum_at = a.sums + (size_t)ce * kNsum + idx;
    unsigned long long *cnt_at = a.counters + 2 * (size_t)ce;
    // half-wave cells with weights read their running sums here, so that
    // the latency overlaps the accumulation below (the one-wave kernel at six
    // waves per SIMD has no registers to spare and reads them at the end)
    constexpr bool kEarly = VR && T == 32;
    double old_sum = 0.0;
    if constexpr (kEarly) {
        if (writer) old_sum = *sum_at;
    }
    double q[K];
#pragma unroll
    for (int t = VR ? 26 : 13; t < K; ++t) q[t] = 0.0;  // padding
    // the lane's first particle sets the sums (a lane without one sets
    // zeros), the others are added; products are added with fused
    // multiply-adds (the sums are compared with a tolerance; the particle
    // state is what must match exactly)
    for (uint32_t r = tid; r < N || r == tid; r += T) {
        const bool has = r < N;
        R x = (R)0, y = (R)0, z = (R)0, w = (R)1;
        if (has) {
            v.get(r, x, y, z);
            if (VR) w = v.getw(r);
            if (View::kInLds) {
                a.s.cx[wb_base + r] = x; a.s.cy[wb_base + r] = y; a.s.cz[wb_base + r] = z;
                if (VR) a.s.w[wb_base + r] = w;
            }
        }
        const double vx = (double)x, vy = (double)y, vz = (double)z;
        const double xx = vx * vx, yy = vy * vy, zz = vz * vz;
        const double c2 = (xx + yy) + zz;
        if (r == tid) {
            q[0] = has ? 1.0 : 0.0; q[1] = vx; q[2] = vy; q[3] = vz;
            q[4] = xx; q[5] = yy; q[6] = zz;
            q[7] = vx * vy; q[8] = vx * vz; q[9] = vy * vz;
            q[10] = vx * c2; q[11] = vy * c2; q[12] = vz * c2;
        } else {
            q[0] += 1.0; q[1] += vx; q[2] += vy; q[3] += vz;
            q[4] += xx; q[5] += yy; q[6] += zz;
            q[7] = fma(vx, vy, q[7]); q[8] = fma(vx, vz, q[8]); q[9] = fma(vy, vz, q[9]);
            q[10] = fma(vx, c2, q[10]); q[11] = fma(vy, c2, q[11]); q[12] = fma(vz, c2, q[12]);
        }
        if (VR) {
            const double f = 1.0 - (double)w;
            const double fx = f * vx, fy = f * vy, fz = f * vz;
            if (r == tid) {
                q[13] = f; q[14] = fx; q[15] = fy; q[16] = fz;
                q[17] = fx * vx; q[18] = fy * vy; q[19] = fz * vz;
                q[20] = fx * vy; q[21] = fx * vz; q[22] = fy * vz;
                q[23] = fx * c2; q[24] = fy * c2; q[25] = fz * c2;
            } else {
                q[13] += f; q[14] += fx; q[15] += fy; q[16] += fz;
                q[17] = fma(fx, vx, q[17]); q[18] = fma(fy, vy, q[18]); q[19] = fma(fz, vz, q[19]);
                q[20] = fma(fx, vy, q[20]); q[21] = fma(fx, vz, q[21]); q[22] = fma(fy, vz, q[22]);
                q[23] = fma(fx, c2, q[23]); q[24] = fma(fy, c2, q[24]); q[25] = fma(fz, c2, q[25]);
            }
        }
    }
    // each lane ends up with the total of the sum it owns
    double tot = 0.0;
    if constexpr (T > 64) {
        // per wave by recursive halving, then the waves in a fixed order:
        // thread t < 26 (13) owns sum t
        (void)red;
        const double t = wave_sum_many<K>(q);  // lane L: total of index L >> (VR ? 1 : 2)
        if ((lane & (VR ? 1 : 3)) == 0) gs->d[tid >> 6][lane >> (VR ? 1 : 2)] = t;
        __syncthreads();
        if (tid < (uint32_t)(VR ? kNsum : 13)) {
#pragma unroll
            for (int w = 0; w < T / 64; ++w) tot += gs->d[w][tid];
        }
    } else if constexpr (T == 32) {
        // the transpose in the half's own area: 13 rows of 32 doubles, two
        // lanes per row, each adding 16 of its doubles (8 interleaved
        // 16-byte columns, starting at column block r mod 8)
        static_assert(View::kInLds, "half-wave cells are staged in LDS");
        constexpr int RS = 32;
        const int row = lane >> 1, part = lane & 1;
        __syncthreads();
#pragma unroll
        for (int h = 0; h < (VR ? 2 : 1); ++h) {
#pragma unroll
            for (int u = 0; u < 13; ++u) red[u * RS + lane] = q[13 * h + u];
            __syncthreads();
            double t = 0.0;
            if (row < 13) {
                const double2 *rp = (const double2 *)(red + row * RS);
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const double2 e = rp[2 * ((c + row) & 7) + part];
                    s0 += e.x;
                    s1 += e.y;
                }
                t = s0 + s1;
            }
            t = t + quad_perm_f64<0xB1>(t);
            if (part == h) tot = t;
            __syncthreads();
        }
    } else if constexpr (View::kInLds) {
        constexpr int RS = kRedStride;
        const int row = lane >> 2, part = lane & 3;
        __syncthreads();
#pragma unroll
        for (int h = 0; h < (VR ? 2 : 1); ++h) {
#pragma unroll
            for (int u = 0; u < 13; ++u) red[u * RS + lane] = q[13 * h + u];
            __syncthreads();
            double t = 0.0;
            if (row < 13) {
                const double2 *rp = (const double2 *)(red + row * RS);
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const double2 e = rp[4 * ((c + row) & 7) + part];
                    s0 += e.x;
                    s1 += e.y;
                }
                t = s0 + s1;
            }
            t = quad_sum_f64(t);
            if (part == h) tot = t;
            __syncthreads();
        }
    } else {
        (void)red;
        const double t = wave_sum_many<K>(q);  // lane L: total of index L >> (VR ? 1 : 2)
        tot = __shfl(t, (lane << (VR ? 1 : 2)) & 63, 64);
    }
    const bool nonfinite = writer && !isfinite(tot);
    const bool bad_plain = cell_ballot<T>(nonfinite && idx < 13) != 0ull;
    const bool bad_vr = cell_ballot<T>(nonfinite && idx >= 13) != 0ull;
    if constexpr (!VR) {
        if (writer) *sum_at = pf.sum + tot;
    } else if constexpr (kEarly) {
        if (writer) *sum_at = old_sum + tot;
    } else {
        if (writer) *sum_at = *sum_at + tot;
    }
    if (tid == 0) {
        if constexpr (!VR) {
            cnt_at[0] = pf.cand + M;
            cnt_at[1] = pf.acc + acc;
        } else {
            cnt_at[0] = cnt_at[0] + M;
            cnt_at[1] = cnt_at[1] + acc;
        }
        if (over) diag_add(a.st, kDiagOvershoot, (unsigned long long)over);
        if (bad_plain) set_error(a.st, DSMC_ENONFINITE);
        if (bad_vr) diag_add(a.st, kDiagVrNonfinite, 1ull);
    }
}

// Real-valued NTC candidate count 1/2 N (N-1) F_N (sigma g)_max dt / V, in
// this left-to-right order: (sigma g)_max = sigma g_max (hard spheres),
// sigma (Maxwell molecules, sigma g constant) or sigma g_max^(2 - 2 omega)
// (variable hard and soft spheres).
template <typename R>
__device__ __forceinline__ double candidates_real(const CollideArgs<R> &a, double Nd, double gmax, double V) {
    if (a.molecule == DSMC_MAXWELL) return (((((0.5 * Nd) * (Nd - 1.0)) * a.FN) * a.sigma) * a.dt) / V;
    if (a.molecule == DSMC_VHS || a.molecule == DSMC_VSS)
        return ((((((0.5 * Nd) * (Nd - 1.0)) * a.FN) * a.sigma) * vhs_pow(gmax * gmax, a.omega1)) * a.dt) / V;
    return ((((((0.5 * Nd) * (Nd - 1.0)) * a.FN) * a.sigma) * gmax) * a.dt) / V;
}

// Whether the weights of a cell of N particles are re-estimated in this step.
template <typename R>
__device__ __forceinline__ bool reestimate_now(const CollideArgs<R> &a, uint32_t N, uint32_t step) {
    return a.vr_reest > 0 && N >= (uint32_t)kReMin && step % (uint32_t)a.vr_reest == 0u;
}

// Majorant, candidate count, NTC loop and sampling of one cell; the view
// already holds the cell in canonical order.
template <typename R, bool VR, typename View, int T = 64>
__device__ void process_cell(const CollideArgs<R> &a, const View &v, uint32_t cell, uint32_t N,
                             uint32_t step, const CellPrefetch<!VR> &pf, double *red = nullptr, uint32_t wb_base = 0,
                             GroupScratch *gs = nullptr, bool use_box = false, BoxKeys box = BoxKeys{}) {
    uint32_t M = 0, acc = 0, over = 0;
    if (N >= 2) {
        double rt;
        double gmax = 1.0;
        if (a.molecule != DSMC_MAXWELL) {
            gmax = a.majorant == DSMC_MAJORANT_DIAMETER ? pair_diameter<R, View, T>(v, N, gs)
                                                        : exact_bound<R, View, T>(v, N, rt, gs, nullptr, nullptr, use_box, box);
            if (VR && a.vr_kappa > 1.0) gmax = gmax * a.vr_kappa;
        }
        const double V = a.volume ? a.volume[cell] : a.Vuni;
        const double Nd = (double)N;
        const double Mreal = candidates_real<R>(a, Nd, gmax, V);
        const u32x4 r = draw(0, kTagNcand, 0, cell, step, a.k0, a.k1);
        double Mf = floor(Mreal + unif53(r.v[0], r.v[1]));
        if (!(Mf >= 0.0)) Mf = 0.0;
        if (Mf > kMaxCandidates) {
            if (cell_tid<T>() == 0) set_error(a.st, DSMC_ECAPACITY);
            Mf = 0.0;
        }
        M = (uint32_t)Mf;
        ntc_loop<R, VR, View, T>(v, N, gmax, M, cell, step, a.k0, a.k1, a.molecule, a.omega1, a.inv_alpha, acc,
                                 over, gs);
    }
    if (VR && reestimate_now(a, N, step)) reestimate_weights<R, View, T>(v, N, a.vr_scale, gs);
    sample_cell<R, VR, View, T>(a, v, cell, N, M, acc, over, pf, red, wb_base, gs);
}

}  // namespace dsmc
