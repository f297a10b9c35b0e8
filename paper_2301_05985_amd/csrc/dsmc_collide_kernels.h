// dsmc_collide_kernels.h -- the collision kernels: cells staged in LDS (one
// wave per cell) and, for cells above the LDS capacity, a global-memory
// variant; each with the exact or the learned majorant.
#pragma once
#include "dsmc_collide.h"
#include "dsmc_learned.h"

namespace dsmc {

// LDS kernel: one wave per cell.  BYID: the cell arrives in arbitrary order
// from the counting sort and is ranked by particle id in LDS (canonical
// order); otherwise (homogeneous instances) storage order is canonical.
template <typename R, bool VR, bool BYID, bool LEARNED>
__device__ __forceinline__ void collide_lds_body(const CollideArgs<R> &a, unsigned char *smem) {
    const int lane = lane_id();
    const uint32_t cell = a.sched ? a.sched[blockIdx.x] : blockIdx.x;
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
    const int cap = a.cap;
    R *vx = (R *)smem, *vy = vx + cap, *vz = vy + cap;
    R *w = VR ? vz + cap : nullptr;
    uint32_t *owner = (uint32_t *)(VR ? w + cap : vz + cap);
    uint16_t *rank_of_slot = (uint16_t *)(owner + cap);
    if (BYID) {
        uint32_t *ids = owner;  // the owner array is free until the ranks are known
        for (uint32_t s = lane; s < N; s += 64) ids[s] = a.s.id[base + s];
        __syncthreads();
        for (uint32_t s0 = 0; s0 < N; s0 += 64) {
            const uint32_t s = s0 + lane;
            if (s < N) {
                const R x = a.s.cx[base + s], y = a.s.cy[base + s], z = a.s.cz[base + s];
                R ww = (R)0;
                if (VR) ww = a.s.w[base + s];
                const uint32_t me = ids[s];
                uint32_t rank = 0;
                for (uint32_t t = 0; t < N; ++t) rank += ids[t] < me ? 1u : 0u;
                rank_of_slot[s] = (uint16_t)rank;
                vx[rank] = x; vy[rank] = y; vz[rank] = z;
                if (VR) w[rank] = ww;
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
    if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step);
    else process_cell<R, VR>(a, view, cell, N, step);
    __syncthreads();
    for (uint32_t s = lane; s < N; s += 64) {
        const uint32_t r = BYID ? (uint32_t)rank_of_slot[s] : s;
        a.s.cx[base + s] = vx[r]; a.s.cy[base + s] = vy[r]; a.s.cz[base + s] = vz[r];
        if (VR) a.s.w[base + s] = w[r];
    }
}

// Global-memory kernel for cells larger than the LDS capacity: works in
// place through a rank -> slot permutation and a global owner array.
template <typename R, bool VR, bool BYID, bool LEARNED>
__device__ __forceinline__ void collide_big_body(const CollideArgs<R> &a) {
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
        if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step);
        else process_cell<R, VR>(a, view, cell, N, step);
        if (lane == 0) atomicAdd(&a.st->diag[kDiagBig], 1ull);
        __syncthreads();
    }
}

template <typename R, bool VR, bool BYID>
__global__ __launch_bounds__(64) void k_collide(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_lds_body<R, VR, BYID, false>(a, smem);
}

template <typename R, bool VR, bool BYID>
__global__ __launch_bounds__(64) void k_collide_big(CollideArgs<R> a) {
    collide_big_body<R, VR, BYID, false>(a);
}

template <typename R, bool VR, bool BYID>
__global__ __launch_bounds__(64) void k_collide_learned(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_lds_body<R, VR, BYID, true>(a, smem);
}

template <typename R, bool VR, bool BYID>
__global__ __launch_bounds__(64) void k_collide_big_learned(CollideArgs<R> a) {
    collide_big_body<R, VR, BYID, true>(a);
}

}  // namespace dsmc
