// dsmc_collide_kernels.h -- the collision kernels: cells staged in LDS (one
// wave per cell) and, for cells above the LDS capacity, a global-memory
// variant; each with the exact or the learned majorant.
#pragma once
#include "dsmc_collide.h"
#include "dsmc_learned.h"

namespace dsmc {

// One pass of the id ranking: J slots per lane (slots s0 + 64 j + lane),
// each counted against every id of the cell with 16-byte broadcast reads;
// the slot's particle is placed at its rank in the LDS arrays.
template <typename R, bool VR, int J>
__device__ __forceinline__ void rank_pass(const CollideArgs<R> &a, uint32_t base, uint32_t s0, uint32_t N,
                                          uint32_t n4, const uint32_t *ids, const uint4 *ids4, R *vx, R *vy,
                                          R *vz, R *w, uint16_t *rank_of_slot) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t me[J], rk[J];
    R x[J], y[J], z[J], ww[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t s = s0 + (uint32_t)j * 64 + lane;
        me[j] = 0u;
        rk[j] = 0u;
        if (s < N) {
            me[j] = ids[s];
            x[j] = a.s.cx[base + s]; y[j] = a.s.cy[base + s]; z[j] = a.s.cz[base + s];
            if (VR) ww[j] = a.s.w[base + s];
        }
    }
    for (uint32_t t4 = 0; t4 < n4; ++t4) {
        const uint4 q = ids4[t4];
#pragma unroll
        for (int j = 0; j < J; ++j)
            rk[j] += (uint32_t)(q.x < me[j]) + (uint32_t)(q.y < me[j]) + (uint32_t)(q.z < me[j]) +
                     (uint32_t)(q.w < me[j]);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t s = s0 + (uint32_t)j * 64 + lane;
        if (s < N) {
            rank_of_slot[s] = (uint16_t)rk[j];
            vx[rk[j]] = x[j]; vy[rk[j]] = y[j]; vz[rk[j]] = z[j];
            if (VR) w[rk[j]] = ww[j];
        }
    }
}

// Cells of at most 256 particles: J slots per lane, ids and velocities loaded
// in one round trip, ids shared through LDS, then ranked and placed.
template <typename R, bool VR, int J>
__device__ __forceinline__ void rank_single(const CollideArgs<R> &a, uint32_t base, uint32_t N, uint32_t n4,
                                            uint32_t *ids, const uint4 *ids4, R *vx, R *vy, R *vz, R *w,
                                            uint16_t *rank_of_slot) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t me[J], rk[J];
    R x[J], y[J], z[J], ww[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        me[j] = 0u;
        rk[j] = 0u;
        if (s < N) {
            me[j] = a.s.id[base + s];
            x[j] = a.s.cx[base + s]; y[j] = a.s.cy[base + s]; z[j] = a.s.cz[base + s];
            if (VR) ww[j] = a.s.w[base + s];
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        if (s < N) ids[s] = me[j];
    }
    if (lane < 4) ids[N + lane] = 0xFFFFFFFFu;  // padding never ranks below a real id
    __syncthreads();
    for (uint32_t t4 = 0; t4 < n4; ++t4) {
        const uint4 q = ids4[t4];
#pragma unroll
        for (int j = 0; j < J; ++j)
            rk[j] += (uint32_t)(q.x < me[j]) + (uint32_t)(q.y < me[j]) + (uint32_t)(q.z < me[j]) +
                     (uint32_t)(q.w < me[j]);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        if (s < N) {
            rank_of_slot[s] = (uint16_t)rk[j];
            vx[rk[j]] = x[j]; vy[rk[j]] = y[j]; vz[rk[j]] = z[j];
            if (VR) w[rk[j]] = ww[j];
        }
    }
}

// LDS kernel: one wave per cell.  BYID: the cell arrives in arbitrary order
// from the counting sort and is ranked by particle id in LDS (canonical
// order); otherwise (homogeneous instances) storage order is canonical.
// D is the run's dimension (0 for homogeneous instances); walled runs rank
// by particle id.
template <typename R, bool VR, int D, bool LEARNED>
__device__ __forceinline__ void collide_lds_body(const CollideArgs<R> &a, unsigned char *smem, uint32_t cell) {
    constexpr bool BYID = D > 0;
    const int lane = lane_id();
    const uint32_t base = a.start[cell];
    const uint32_t N = a.start[cell + 1] - base;
    if (N > (uint32_t)a.cap) {
        if (lane == 0) {
            const uint32_t q = atomicAdd(&a.st->big_count, 1u);
            a.big_list[q] = cell;
        }
        return;
    }
    const uint32_t step = (uint32_t)a.st->step_cur;
    const CellPrefetch pf = prefetch_cell<R, VR>(a, cell);
    const int cap = a.cap;
    R *vx = (R *)smem, *vy = vx + cap, *vz = vy + cap;
    R *w = VR ? vz + cap : nullptr;
    uint32_t *owner = (uint32_t *)(VR ? w + cap : vz + cap);  // cap + 4 entries
    uint16_t *rank_of_slot = (uint16_t *)(owner + cap + 4);
    if (BYID) {
        // canonical order: rank of each slot by particle id, counted against
        // the whole cell with 16-byte broadcast reads; up to four slots per
        // lane per pass (cells of up to 256 particles take one pass)
        uint32_t *ids = owner;  // the owner array is free until the ranks are known
        const uint4 *ids4 = (const uint4 *)ids;
        const uint32_t n4 = (N + 3) / 4;
        if (N <= 256) {
            // one pass: ids and velocities are fetched together before the
            // ids are shared through LDS
            if (N > 192) rank_single<R, VR, 4>(a, base, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
            else if (N > 128) rank_single<R, VR, 3>(a, base, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
            else if (N > 64) rank_single<R, VR, 2>(a, base, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
            else rank_single<R, VR, 1>(a, base, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
        } else {
            for (uint32_t s = lane; s < N; s += 64) ids[s] = a.s.id[base + s];
            if (lane < 4) ids[N + lane] = 0xFFFFFFFFu;  // padding never ranks below a real id
            __syncthreads();
            for (uint32_t s0 = 0; s0 < N; s0 += 256) {
                const uint32_t left = N - s0;
                if (left > 192) rank_pass<R, VR, 4>(a, base, s0, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
                else if (left > 128) rank_pass<R, VR, 3>(a, base, s0, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
                else if (left > 64) rank_pass<R, VR, 2>(a, base, s0, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
                else rank_pass<R, VR, 1>(a, base, s0, N, n4, ids, ids4, vx, vy, vz, w, rank_of_slot);
            }
        }
        __syncthreads();
    } else {
        for (uint32_t s = lane; s < N; s += 64) {
            vx[s] = a.s.cx[base + s]; vy[s] = a.s.cy[base + s]; vz[s] = a.s.cz[base + s];
            if (VR) w[s] = a.s.w[base + s];
        }
    }
    for (uint32_t r = lane; r < N; r += 64) owner[r] = 0xFFFFFFFFu;
    __syncthreads();
    const LdsView<R> view{vx, vy, vz, w, owner};
    if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf);
    else process_cell<R, VR>(a, view, cell, N, step, pf);
    __syncthreads();
    for (uint32_t s = lane; s < N; s += 64) {
        const uint32_t r = BYID ? (uint32_t)rank_of_slot[s] : s;
        a.s.cx[base + s] = vx[r]; a.s.cy[base + s] = vy[r]; a.s.cz[base + s] = vz[r];
        if (VR) a.s.w[base + s] = w[r];
    }
}

// Global-memory kernel for cells larger than the LDS capacity: works in
// place through a rank -> slot permutation and a global owner array.
template <typename R, bool VR, int D, bool LEARNED>
__device__ __forceinline__ void collide_big_body(const CollideArgs<R> &a) {
    constexpr bool BYID = D > 0;
    const int lane = lane_id();
    const uint32_t step = (uint32_t)a.st->step_cur;
    const uint32_t nbig = a.st->big_count;
    for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const uint32_t cell = a.big_list[q];
        const uint32_t base = a.start[cell];
        const uint32_t N = a.start[cell + 1] - base;
        uint32_t *perm = BYID ? a.perm_g + base : nullptr;
        if (BYID) {
            for (uint32_t s = lane; s < N; s += 64) {
                const uint32_t me = a.s.id[base + s];
                uint32_t rank = 0;
                for (uint32_t t = 0; t < N; ++t) rank += a.s.id[base + t] < me ? 1u : 0u;
                perm[rank] = s;
            }
        }
        const GlobalView<R> view{a.s.cx + base, a.s.cy + base, a.s.cz + base,
                                 VR ? a.s.w + base : nullptr, perm, a.owner_g + base};
        for (uint32_t r = lane; r < N; r += 64) view.clear_own(r);
        __syncthreads();
        const CellPrefetch pf = prefetch_cell<R, VR>(a, cell);
        if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf);
        else process_cell<R, VR>(a, view, cell, N, step, pf);
        if (lane == 0) diag_add(a.st, kDiagBig, 1ull);
        __syncthreads();
    }
}

template <typename R, bool VR, int D>
__global__ __launch_bounds__(64) void k_collide(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_lds_body<R, VR, D, false>(a, smem, a.sched ? a.sched[blockIdx.x] : blockIdx.x);
}

template <typename R, bool VR, int D>
__global__ __launch_bounds__(64) void k_collide_big(CollideArgs<R> a) {
    collide_big_body<R, VR, D, false>(a);
}

template <typename R, bool VR, int D>
__global__ __launch_bounds__(64) void k_collide_learned(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_lds_body<R, VR, D, true>(a, smem, a.sched ? a.sched[blockIdx.x] : blockIdx.x);
}

template <typename R, bool VR, int D>
__global__ __launch_bounds__(64) void k_collide_big_learned(CollideArgs<R> a) {
    collide_big_body<R, VR, D, true>(a);
}

// Persistent collision kernel for homogeneous instances: a fixed grid of
// waves takes work units from eight device queues (reset by the step
// bookkeeping kernel).  A unit is a run of consecutive entries of the
// longest-first schedule: one large instance, or several small ones; unit u
// belongs to queue u mod 8.  A wave starts on the queue of its XCD and, once
// that queue is exhausted, moves on to the next ones, so every unit is taken
// exactly once and the grid drains each step.  The claim of the next unit is
// issued before the current unit is processed, so its latency overlaps the
// current unit's loads.
template <typename R, bool VR, bool LEARNED>
__global__ __launch_bounds__(64) void k_collide_persistent(CollideArgs<R> a, const uint2 *units, uint32_t n_units) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t q = blockIdx.x % kQueues;
    uint32_t left = kQueues;  // queues not yet found exhausted
    uint32_t u = n_units;
    // blocking claim: the next unit of queue q, moving on when q is exhausted
    while (left > 0) {
        uint32_t k = 0;
        if (lane_id() == 0) k = atomicAdd(&a.st->queue[q * kQueueStride], 1u);
        k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
        u = q + k * kQueues;
        if (u < n_units) break;
        q = (q + 1) % kQueues;
        --left;
        u = n_units;
    }
    while (u < n_units) {
        const uint2 w = units[u];
        uint32_t pending = 0;
        if (lane_id() == 0) pending = atomicAdd(&a.st->queue[q * kQueueStride], 1u);
        for (uint32_t k = 0; k < w.y; ++k) {
            collide_lds_body<R, VR, 0, LEARNED>(a, smem, a.sched[w.x + k]);
            __syncthreads();
        }
        u = q + (uint32_t)__builtin_amdgcn_readfirstlane((int)pending) * kQueues;
        if (u < n_units) continue;
        q = (q + 1) % kQueues;
        --left;
        u = n_units;
        while (left > 0) {
            uint32_t k = 0;
            if (lane_id() == 0) k = atomicAdd(&a.st->queue[q * kQueueStride], 1u);
            k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
            u = q + k * kQueues;
            if (u < n_units) break;
            q = (q + 1) % kQueues;
            --left;
            u = n_units;
        }
    }
}

// Training data for the learned majorant: per cell, the six input features
// and log2 of the exact largest pairwise relative speed (brute force over all
// pairs, in double); -inf for cells with fewer than two particles.
template <typename R>
__global__ __launch_bounds__(64) void k_collect_features(CollideArgs<R> a, int ncell, float *feat, float *label,
                                                         float *bound) {
    const int lane = lane_id();
    const uint32_t cell = blockIdx.x;
    if ((int)cell >= ncell) return;
    const uint32_t base = a.start[cell];
    const uint32_t N = a.start[cell + 1] - base;
    const GlobalView<R> v{a.s.cx + base, a.s.cy + base, a.s.cz + base, nullptr, nullptr, nullptr};
    if (N < 2) {
        if (lane < 6) feat[(size_t)cell * 6 + lane] = 0.0f;
        if (lane == 0) label[cell] = -INFINITY;
        if (lane == 0 && bound) bound[cell] = -INFINITY;
        return;
    }
    const double V = a.volume ? a.volume[cell] : a.Vuni;
    const Features F = cell_features<R>(v, N, a.FN, V);
    double best = 0.0;
    for (uint32_t r = lane; r < N; r += 64) {
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
    best = wave_max_t(best);
    if (lane < 6) feat[(size_t)cell * 6 + lane] = F.f[lane == 0 ? 0 : lane == 1 ? 1 : lane == 2 ? 2 : lane == 3 ? 3 : lane == 4 ? 4 : 5];
    if (lane == 0) label[cell] = (float)log2(sqrt(best));
    if (bound) {
        double rt;
        const double gb = exact_bound<R>(v, N, rt);
        if (lane == 0) bound[cell] = (float)log2(gb);
    }
}

}  // namespace dsmc
