// dsmc_learned.h -- learned collision majorant with exact verification.
//
// A small network (6 -> 64 -> 64 -> 1, ReLU, BF16 weights held as FP32,
// FP32 arithmetic) predicts log2 of the largest relative speed in a cell from
// six moments of its pre-collision state.  The proposal is rounded up to the
// lattice 2^(k/64) and used only if (a) it is below the exact bound and
// (b) the kernel proves that it bounds every pair: with g_v = g_pred (1 - eps)
// (eps the exact bound's rounding margin), a pair faster than g_v has both
// members in S = {p : r_p + r_(1) > g_v} (r_p = distance to the bounding-box
// midpoint), so if |S| <= 64 all pairs of S are compared with g_v in double;
// otherwise, or if a pair exceeds it, the exact bound is used.  The decision
// depends only on the pre-collision state, so the collision law is that of
// the exact method (both majorants bound the pre-collision pairs; a pair made
// faster than the majorant by an earlier collision of the same step has its
// acceptance truncated at 1 under either, and is counted as an overshoot).
//
// One wave per cell; hidden unit h of both layers lives on lane h, the
// output is reduced by the butterfly with strides 32..1 (a fixed order, so
// the lattice index is reproducible).  Device weight layout: W1[64][6],
// b1[64], W2 transposed [64 in][64 out], b2[64], w3[64], b3.
#pragma once
#include "dsmc_collide.h"

namespace dsmc {

constexpr int kLatticeHalf = 4096;
constexpr int kLatticeSize = 2 * kLatticeHalf + 1;
constexpr int kMlpIn = 6, kMlpH = 64;

struct Features { float f[kMlpIn]; };

// Features from the seven moment sums of a cell, sum k on lane k (k < 7),
// identical on every lane:
//   log2(number density), u_x / sqrt(T), u_y / sqrt(T), log2(T),
//   P_xx / p - 1, P_xy / p      (FP64, each rounded once to float)
// The independent divisions (and the two logarithms) of each stage run side
// by side on different lanes; every value is the same IEEE operation on the
// same operands as in the written-out formulas.
__device__ __forceinline__ Features features_from_lane_sums(double S, uint32_t N, double FNum, double V) {
    const int lane = lane_id();
    const auto rl = [](double x, int l) {
        const uint64_t b = (uint64_t)__double_as_longlong(x);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    };
    const double Nd = (double)N;
    const double s3 = rl(S, 3), s4 = rl(S, 4), s5 = rl(S, 5);
    // stage 1: u_x, u_y, u_z, <c^2>, <c_x^2>, <c_x c_y>, density
    double num = S, den = Nd;
    if (lane == 3) num = (s3 + s4) + s5;
    if (lane == 4) num = s3;
    if (lane == 5) num = rl(S, 6);
    if (lane == 6) { num = Nd * FNum; den = V; }
    const double q = num / den;
    const double ux = rl(q, 0), uy = rl(q, 1), uz = rl(q, 2), ec2 = rl(q, 3), exx = rl(q, 4), exy = rl(q, 5),
                 dens = rl(q, 6);
    // stage 2: temperature, pressures
    double Tk = (ec2 - ((ux * ux + uy * uy) + uz * uz)) / 3.0;
    if (!(Tk > 1e-300)) Tk = 1e-300;
    const double Pxx = dens * (exx - ux * ux);
    const double Pxy = dens * (exy - ux * uy);
    const double pr = dens * Tk;
    const double sT = sqrt(Tk);
    // stage 3: feature k on lane k
    double n3 = 1.0, d3 = 1.0, lg = 1.0;
    if (lane == 1) { n3 = ux; d3 = sT; }
    if (lane == 2) { n3 = uy; d3 = sT; }
    if (lane == 4) { n3 = Pxx; d3 = pr; }
    if (lane == 5) { n3 = Pxy; d3 = pr; }
    if (lane == 0) lg = dens;
    if (lane == 3) lg = Tk;
    const double dq = n3 / d3;
    const double lq = log2(lg);
    const float f = (float)(lane == 0 || lane == 3 ? lq : (lane == 4 ? dq - 1.0 : dq));
    Features F;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) F.f[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), k));
    return F;
}

// Moment sums of this lane (7 values) reduced over the wave, sum k to lane k.
__device__ __forceinline__ double wave_sums_to_lanes(double (&q)[8]) {
    const double t = wave_sum_many<8>(q);  // lane L: total of sum L >> 3
    return __shfl(t, (lane_id() & 7) << 3, 64);
}

// Features of the cell held by the view (one wave), for the training data.
template <typename R, typename View>
__device__ Features cell_features(const View &v, uint32_t N, double FNum, double V) {
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // sx, sy, sz, sxx, syy, szz, sxy, (pad)
    for (uint32_t r = lane_id(); r < N; r += 64) {
        R a, b, c;
        v.get(r, a, b, c);
        const double vx = (double)a, vy = (double)b, vz = (double)c;
        q[0] += vx; q[1] += vy; q[2] += vz;
        q[3] += vx * vx; q[4] += vy * vy; q[5] += vz * vz; q[6] += vx * vy;
    }
    return features_from_lane_sums(wave_sums_to_lanes(q), N, FNum, V);
}

// Network output (log2 units), identical on every lane.
__device__ __forceinline__ float mlp_forward_wave(const float *P, const Features &F) {
    const int h = lane_id();
    const float *W1 = P, *b1 = W1 + kMlpH * kMlpIn, *W2T = b1 + kMlpH, *b2 = W2T + kMlpH * kMlpH,
                *w3 = b2 + kMlpH, *b3 = w3 + kMlpH;
    float acc = b1[h];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) acc = fmaf(W1[h * kMlpIn + i], F.f[i], acc);
    const float a1 = acc > 0.0f ? acc : 0.0f;
    acc = b2[h];
    // hidden value i read from lane i as a scalar (no LDS permute)
#pragma unroll
    for (int i = 0; i < kMlpH; ++i)
        acc = fmaf(W2T[i * kMlpH + h], __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a1), i)), acc);
    const float a2 = acc > 0.0f ? acc : 0.0f;
    float s = w3[h] * a2;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s = s + __shfl_xor(s, off, 64);
    return s + b3[0];
}

// Verified learned majorant; returns the majorant and sets used to
// 1 (learned), 0 (proposal not below the exact bound), -1 (fallback).  Run by
// all T threads of the cell (every wave evaluates the network; the results
// are identical); the particle passes are spread over the threads.  Only the
// size of S and whether some pair of S exceeds the proposal decide, so the
// order in which members are found does not matter.
template <typename R, typename View, int T = 64>
__device__ double learned_majorant(const CollideArgs<R> &a, const View &v, uint32_t N, double V, int &used,
                                   GroupScratch *gs = nullptr) {
    const int lane = lane_id();
    double r1, mid[3];
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // moment sums of this thread's particles
    const double gb = exact_bound<R, View, T, true>(v, N, r1, gs, mid, q);
    // size gate: cells too small to repay the network and the verification
    // take the exact bound directly
    if (N < a.mlp_min_n) { used = 0; return gb; }
    // the proposal: on the first wave only (shared through LDS in a workgroup)
    double S = wave_sums_to_lanes(q);
    if constexpr (T > 64) {
        if (lane < 7) gs->d[threadIdx.x >> 6][8 + lane] = S;
        __syncthreads();
    }
    double gp = 0.0;
    if (threadIdx.x < 64) {
        if constexpr (T > 64) {
            // the waves' sums in a fixed order
            if (lane < 7) {
                S = gs->d[0][8 + lane];
#pragma unroll
                for (int w = 1; w < T / 64; ++w) S += gs->d[w][8 + lane];
            }
        }
        const Features F = features_from_lane_sums(S, N, a.FN, V);
        const float y = mlp_forward_wave(a.mlp, F);
        double kk = ceil(64.0 * ((double)y + a.delta));
        if (!(kk > -(double)kLatticeHalf)) kk = -(double)kLatticeHalf;
        if (kk > (double)kLatticeHalf) kk = (double)kLatticeHalf;
        gp = a.lattice[(int)kk + kLatticeHalf];
    }
    if constexpr (T > 64) {
        if (threadIdx.x == 0) gs->d[0][16] = gp;
        __syncthreads();
        gp = gs->d[0][16];
        __syncthreads();  // the scratch is reused
    }
    if (!(gp < gb)) { used = 0; return gb; }
    // verified against gp (1 - eps), eps the exact bound's rounding margin:
    // a pair that passes then stays below the proposal also after the
    // proposal and the pair's squared speed are rounded to the working
    // precision of the acceptance test
    const double gv = gp * (1.0 - (sizeof(R) == 4 ? 0x1.0p-20 : 0x1.0p-50));
    const double m0 = mid[0], m1 = mid[1], m2 = mid[2];
    const auto in_s = [&](uint32_t r) {
        R x, yv, z;
        v.get(r, x, yv, z);
        const double dx = (double)x - m0, dy = (double)yv - m1, dz = (double)z - m2;
        return sqrt((dx * dx + dy * dy) + dz * dz) + r1 > gv;
    };
    uint32_t mine = 0xFFFFFFFFu;  // rank of the member held by this lane
    uint32_t ns = 0;
    bool overflow = false;
    if constexpr (T > 64) {
        // members listed in LDS in the order they are found (slot from an
        // LDS counter); the list overlays the double scratch, free here
        uint32_t *list = (uint32_t *)&gs->d[0][0];
        uint32_t *count = &gs->u[0][7];
        if (threadIdx.x == 0) *count = 0u;
        __syncthreads();
        for (uint32_t r = threadIdx.x; r < N; r += T) {
            if (in_s(r)) {
                const uint32_t slot = atomicAdd(count, 1u);
                if (slot < 64u) list[slot] = r;
            }
        }
        __syncthreads();
        ns = *count;
        overflow = ns > 64u;
        if (!overflow && (uint32_t)lane < ns) mine = list[lane];
        __syncthreads();  // the scratch is reused
    } else {
        for (uint32_t r0 = 0; r0 < N && !overflow; r0 += 64) {
            const uint32_t r = r0 + (uint32_t)lane;
            const bool in = r < N && in_s(r);
            const unsigned long long m = __ballot(in);
            const uint32_t cnt = (uint32_t)__popcll(m);
            if (ns + cnt > 64) { overflow = true; break; }
            // the q-th member (in lane order) moves to lane ns + q
            const int qq = lane - (int)ns;
            int src = 0;
            if (qq >= 0 && qq < (int)cnt) {
                unsigned long long mm = m;
                for (int t = 0; t < qq; ++t) mm &= mm - 1ull;
                src = __ffsll((long long)mm) - 1;
            }
            const uint32_t val = __shfl(r, src, 64);
            if (qq >= 0 && qq < (int)cnt) mine = val;
            ns += cnt;
        }
    }
    bool ok = !overflow;
    if (ok && ns >= 2) {
        // every wave holds all members (lane s: member s)
        R x = 0, yv = 0, z = 0;
        if ((uint32_t)lane < ns) v.get(mine, x, yv, z);
        const double gv2 = gv * gv;
        bool bad = false;
        // lane l compares its member with member (l + d) mod ns for
        // d = 1 .. ns/2, which covers every pair in half the rounds of the
        // triangle; wave w takes d = 1 + w, 1 + w + T/64, ...
        for (uint32_t d = 1 + (threadIdx.x >> 6); d <= ns / 2; d += T / 64) {
            uint32_t q = (uint32_t)lane + d;
            q = q >= ns ? q - ns : q;
            const R bx = __shfl(x, (int)q, 64), by = __shfl(yv, (int)q, 64), bz = __shfl(z, (int)q, 64);
            if ((uint32_t)lane < ns) {
                const double dx = (double)x - (double)bx, dy = (double)yv - (double)by, dz = (double)z - (double)bz;
                const double g2 = (dx * dx + dy * dy) + dz * dz;
                if (g2 > gv2) bad = true;
            }
        }
        uint32_t nbad = __ballot(bad) != 0ull ? 1u : 0u;
        grp_put<T>(gs, 6, nbad);
        grp_sync<T>();
        nbad = grp_sum<T>(gs, 6, nbad);
        grp_sync<T>();  // the scratch is reused
        ok = nbad == 0u;
    }
    if (!ok) { used = -1; return gb; }
    used = 1;
    return gp;
}

// Same as process_cell, with the learned majorant.
template <typename R, bool VR, typename View, int T = 64>
__device__ void process_cell_learned(const CollideArgs<R> &a, const View &v, uint32_t cell, uint32_t N,
                                     uint32_t step, const CellPrefetch<!VR> &pf, double *red = nullptr,
                                     uint32_t wb_base = 0, GroupScratch *gs = nullptr) {
    uint32_t M = 0, acc = 0, over = 0;
    if (N >= 2) {
        const double V = a.volume ? a.volume[cell] : a.Vuni;
        int used = 0;
        double gmax = learned_majorant<R, View, T>(a, v, N, V, used, gs);
        if (VR && a.vr_kappa > 1.0 && a.molecule != DSMC_MAXWELL) gmax = gmax * a.vr_kappa;
        if (threadIdx.x == 0) {
            const int slot = used == 1 ? kDiagLearned : (used == -1 ? kDiagFallback : kDiagSkip);
            diag_add(a.st, slot, 1ull);
        }
        const double Nd = (double)N;
        const double Mreal = candidates_real<R>(a, Nd, gmax, V);
        const u32x4 r = draw(0, kTagNcand, 0, cell, step, a.k0, a.k1);
        double Mf = floor(Mreal + unif53(r.v[0], r.v[1]));
        if (!(Mf >= 0.0)) Mf = 0.0;
        if (Mf > kMaxCandidates) {
            if (threadIdx.x == 0) set_error(a.st, DSMC_ECAPACITY);
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
