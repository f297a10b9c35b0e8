// dsmc_learned.h -- learned collision majorant with exact verification.
//
// A small network (6 -> 64 -> 64 -> 1, ReLU, BF16 weights held as FP32,
// FP32 arithmetic) predicts log2 of the largest relative speed in a cell from
// six moments of its pre-collision state.  The proposal is rounded up to the
// lattice 2^(k/64) and used only if (a) it is below the exact bound and
// (b) the kernel proves that it bounds every pair: a pair faster than g_pred
// has both members in S = {p : r_p + r_(1) > g_pred} (r_p = distance to the
// bounding-box midpoint), so if |S| <= 64 all pairs of S are compared with
// g_pred in double; otherwise, or if a pair exceeds it, the exact bound is
// used.  The decision depends only on the pre-collision state, so the
// collision law is that of the exact method.
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

// Features of the cell held by the view: FP64 moments, rounded once to float.
//   log2(number density), u_x / sqrt(T), u_y / sqrt(T), log2(T),
//   P_xx / p - 1, P_xy / p
template <typename R, typename View>
__device__ Features cell_features(const View &v, uint32_t N, double FNum, double V) {
    const int lane = lane_id();
    double s0 = 0, s1 = 0, s2 = 0, sxx = 0, syy = 0, szz = 0, sxy = 0;
    for (uint32_t r = lane; r < N; r += 64) {
        R a, b, c;
        v.get(r, a, b, c);
        const double vx = (double)a, vy = (double)b, vz = (double)c;
        s0 += vx; s1 += vy; s2 += vz;
        sxx += vx * vx; syy += vy * vy; szz += vz * vz; sxy += vx * vy;
    }
    s0 = wave_sum(s0); s1 = wave_sum(s1); s2 = wave_sum(s2);
    sxx = wave_sum(sxx); syy = wave_sum(syy); szz = wave_sum(szz); sxy = wave_sum(sxy);
    const double Nd = (double)N;
    const double ux = s0 / Nd, uy = s1 / Nd, uz = s2 / Nd;
    double T = (((sxx + syy) + szz) / Nd - ((ux * ux + uy * uy) + uz * uz)) / 3.0;
    if (!(T > 1e-300)) T = 1e-300;
    const double dens = (Nd * FNum) / V;
    const double Pxx = dens * (sxx / Nd - ux * ux);
    const double Pxy = dens * (sxy / Nd - ux * uy);
    const double pr = dens * T;
    const double sT = sqrt(T);
    Features F;
    F.f[0] = (float)log2(dens);
    F.f[1] = (float)(ux / sT);
    F.f[2] = (float)(uy / sT);
    F.f[3] = (float)log2(T);
    F.f[4] = (float)(Pxx / pr - 1.0);
    F.f[5] = (float)(Pxy / pr);
    return F;
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
#pragma unroll 16
    for (int i = 0; i < kMlpH; ++i) acc = fmaf(W2T[i * kMlpH + h], __shfl(a1, i, 64), acc);
    const float a2 = acc > 0.0f ? acc : 0.0f;
    float s = w3[h] * a2;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s = s + __shfl_xor(s, off, 64);
    return s + b3[0];
}

// Verified learned majorant; returns the majorant and sets used to
// 1 (learned), 0 (proposal not below the exact bound), -1 (fallback).
template <typename R, typename View>
__device__ double learned_majorant(const CollideArgs<R> &a, const View &v, uint32_t cell, uint32_t N,
                                   double V, int &used) {
    const int lane = lane_id();
    double r1;
    const double gb = exact_bound<R>(v, N, r1);
    const Features F = cell_features<R>(v, N, a.FN, V);
    const float y = mlp_forward_wave(a.mlp, F);
    double kk = ceil(64.0 * ((double)y + a.delta));
    if (!(kk > -(double)kLatticeHalf)) kk = -(double)kLatticeHalf;
    if (kk > (double)kLatticeHalf) kk = (double)kLatticeHalf;
    const double gp = a.lattice[(int)kk + kLatticeHalf];
    if (!(gp < gb)) { used = 0; return gb; }
    // bounding-box midpoint (same reductions as the exact bound)
    double lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    for (uint32_t r = lane; r < N; r += 64) {
        R x, yv, z;
        v.get(r, x, yv, z);
        lo0 = fmin(lo0, (double)x); hi0 = fmax(hi0, (double)x);
        lo1 = fmin(lo1, (double)yv); hi1 = fmax(hi1, (double)yv);
        lo2 = fmin(lo2, (double)z); hi2 = fmax(hi2, (double)z);
    }
    lo0 = wave_min(lo0); lo1 = wave_min(lo1); lo2 = wave_min(lo2);
    hi0 = wave_max(hi0); hi1 = wave_max(hi1); hi2 = wave_max(hi2);
    const double m0 = 0.5 * (hi0 + lo0), m1 = 0.5 * (hi1 + lo1), m2 = 0.5 * (hi2 + lo2);
    // collect S (at most 64 members, one per lane)
    uint32_t mine = 0xFFFFFFFFu;
    uint32_t ns = 0;
    bool overflow = false;
    for (uint32_t r0 = 0; r0 < N && !overflow; r0 += 64) {
        const uint32_t r = r0 + (uint32_t)lane;
        bool in = false;
        if (r < N) {
            R x, yv, z;
            v.get(r, x, yv, z);
            const double dx = (double)x - m0, dy = (double)yv - m1, dz = (double)z - m2;
            in = sqrt((dx * dx + dy * dy) + dz * dz) + r1 > gp;
        }
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
    bool ok = !overflow;
    if (ok && ns >= 2) {
        R x = 0, yv = 0, z = 0;
        if ((uint32_t)lane < ns) v.get(mine, x, yv, z);
        const double gp2 = gp * gp;
        bool bad = false;
        for (uint32_t b = 0; b < ns; ++b) {
            const R bx = __shfl(x, b, 64), by = __shfl(yv, b, 64), bz = __shfl(z, b, 64);
            if ((uint32_t)lane < ns && b > (uint32_t)lane) {
                const double dx = (double)x - (double)bx, dy = (double)yv - (double)by, dz = (double)z - (double)bz;
                const double g2 = (dx * dx + dy * dy) + dz * dz;
                if (g2 > gp2) bad = true;
            }
        }
        ok = __ballot(bad) == 0ull;
    }
    if (!ok) { used = -1; return gb; }
    used = 1;
    return gp;
}

// Same as process_cell, with the learned majorant.  A workgroup cell
// (T > 64) computes the majorant on its first wave and shares it through LDS.
template <typename R, bool VR, typename View, int T = 64>
__device__ void process_cell_learned(const CollideArgs<R> &a, const View &v, uint32_t cell, uint32_t N,
                                     uint32_t step, const CellPrefetch &pf, double *red = nullptr,
                                     uint32_t wb_base = 0, GroupScratch *gs = nullptr) {
    uint32_t M = 0, acc = 0, over = 0;
    if (N >= 2) {
        const double V = a.volume ? a.volume[cell] : a.Vuni;
        double gmax = 0.0;
        if (threadIdx.x < 64) {
            int used = 0;
            gmax = learned_majorant<R>(a, v, cell, N, V, used);
            if (threadIdx.x == 0) {
                const int slot = used == 1 ? kDiagLearned : (used == -1 ? kDiagFallback : kDiagSkip);
                diag_add(a.st, slot, 1ull);
            }
        }
        if constexpr (T > 64) {
            if (threadIdx.x == 0) gs->d[0][8] = gmax;
            __syncthreads();
            gmax = gs->d[0][8];
            __syncthreads();  // the scratch is reused
        }
        const double Nd = (double)N;
        const double Mreal = candidates_real<R>(a, Nd, gmax, V);
        const u32x4 r = draw(0, kTagNcand, 0, cell, step, a.k0, a.k1);
        double Mf = floor(Mreal + unif53(r.v[0], r.v[1]));
        if (!(Mf >= 0.0)) Mf = 0.0;
        if (Mf > 2147483647.0) {
            if (threadIdx.x == 0) set_error(a.st, DSMC_ECAPACITY);
            Mf = 0.0;
        }
        M = (uint32_t)Mf;
        ntc_loop<R, VR, View, T>(v, N, gmax, M, cell, step, a.k0, a.k1, a.molecule, a.omega1, a.inv_alpha, acc,
                                 over, gs);
    }
    sample_cell<R, VR, View, T>(a, v, cell, N, M, acc, over, pf, red, wb_base, gs);
}

}  // namespace dsmc
