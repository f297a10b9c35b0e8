// dsmc_collide_kernels.h -- the collision kernels: cells staged in LDS (one
// wave per cell) and, for cells above the LDS capacity, a global-memory
// variant; each with the exact or the learned majorant.
#pragma once
#include "dsmc_collide.h"
#include "dsmc_learned.h"

namespace dsmc {

// ------------------------------------------------ gather of a walled cell
// Cell t of the new sequence holds, in order, the particles of the previous
// sequence whose new cell is t (a stable counting sort).  They come from the
// cells around t: along each axis t - 1, t and t + 1 (wrapped when periodic,
// dropped outside the grid), visited in ascending cell index, so that taking
// in each source cell the particles whose move code leads to t, in position
// order, yields them in ascending position.  Far movers (from farther away)
// are taken from the cell's list and merged by position.

// Distinct source coordinates of destination coordinate t along one axis,
// ascending, with the move code step from each to t.
struct AxisSources {
    int n;
    int c[3], d[3];
};

__device__ __forceinline__ AxisSources axis_sources(int t, int n, bool periodic) {
    constexpr int kNone = 0x7FFFFFFF;
    int a = t - 1, b = t + 1;
    if (periodic) {
        a = a < 0 ? a + n : a;
        b = b >= n ? b - n : b;
    } else {
        a = a < 0 ? kNone : a;
        b = b >= n ? kNone : b;
    }
    int v0 = a, v1 = t, v2 = b, tmp;
    if (v0 > v1) { tmp = v0; v0 = v1; v1 = tmp; }
    if (v1 > v2) { tmp = v1; v1 = v2; v2 = tmp; }
    if (v0 > v1) { tmp = v0; v0 = v1; v1 = tmp; }
    AxisSources r;
    const int w1 = v1 > v0 ? v1 : v2;  // the next distinct value, if any
    const bool h1 = w1 > v0 && w1 != kNone;
    const bool h2 = h1 && v1 > v0 && v2 > v1 && v2 != kNone;
    r.n = 1 + (h1 ? 1 : 0) + (h2 ? 1 : 0);
    r.c[0] = v0;
    r.c[1] = w1;
    r.c[2] = v2;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.d[k] = axis_move(r.c[k] == kNone ? t : r.c[k], t, n, periodic);
    return r;
}

// Near movers of `cell`: source positions written to sel[0..) in ascending
// order (at most N are written); returns how many were found.  The first
// PRE x 64 codes of every source cell are loaded before any is consumed.
template <typename R, int D>
__device__ __forceinline__ uint32_t select_near(const CollideArgs<R> &a, uint32_t cell, uint32_t N, uint32_t *sel) {
    constexpr int PRE = D == 1 ? 4 : 2;
    constexpr int NS = D == 1 ? 3 : 9;
    const int lane = lane_id();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int tx = (int)(cell % (uint32_t)a.nx), ty = (int)(cell / (uint32_t)a.nx);
    const AxisSources xs = axis_sources(tx, a.nx, a.periodic_x != 0);
    AxisSources ys;
    if (D == 2) {
        ys = axis_sources(ty, a.ny, a.periodic_y != 0);
    } else {
        ys.n = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) { ys.c[k] = 0; ys.d[k] = 0; }
    }
    if (N == 0) return 0;  // nothing lands here (and the sequence may be empty)
    uint32_t b[NS], e[NS];
    uint32_t req[NS];
    uint32_t cd[NS][PRE];
    // every load below is issued unconditionally from an in-bounds address
    // (positions past a source range are clamped to the last particle) and
    // masked afterwards: no branches around the loads
    const uint32_t last = a.src_start[(uint32_t)a.nx * (uint32_t)(D == 2 ? a.ny : 1)] - 1u;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int iy = k / 3, ix = k % 3;
        const bool ok = ix < xs.n && iy < ys.n;
        const uint32_t src = ok ? (uint32_t)ys.c[iy] * (uint32_t)a.nx + (uint32_t)xs.c[ix] : 0u;
        const uint32_t lb = a.src_start[src], le = a.src_start[src + 1];
        b[k] = ok ? lb : 0u;
        e[k] = ok ? le : 0u;
        req[k] = (uint32_t)((xs.d[ix] + 1) + 3 * (ys.d[iy] + 1));
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const uint32_t i = b[k] + (uint32_t)(64 * j + lane);
            const uint32_t v = (uint32_t)a.code[i < e[k] ? i : last];
            cd[k][j] = i < e[k] ? v : (uint32_t)kFarMove;
        }
    uint32_t nsel = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const bool m = cd[k][j] == req[k];
            const unsigned long long bal = __ballot(m);
            if (m) {
                const uint32_t pos = nsel + (uint32_t)__popcll(bal & lt);
                if (pos < N) sel[pos] = b[k] + (uint32_t)(64 * j + lane);
            }
            nsel += (uint32_t)__popcll(bal);
        }
        // source cells longer than the preloaded part
        for (uint32_t i0 = b[k] + 64 * PRE; i0 < e[k]; i0 += 64) {
            const uint32_t i = i0 + (uint32_t)lane;
            const bool m = i < e[k] && (uint32_t)a.code[i] == req[k];
            const unsigned long long bal = __ballot(m);
            if (m) {
                const uint32_t pos = nsel + (uint32_t)__popcll(bal & lt);
                if (pos < N) sel[pos] = i;
            }
            nsel += (uint32_t)__popcll(bal);
        }
    }
    return nsel;
}

// Far movers of `cell`: walked by lane 0 from the cell's list into
// sel[n_near..N); the list head is reset for the next step.  Any mismatch
// with the cell's count is reported, and sel is filled with valid positions.
template <typename R>
__device__ __forceinline__ void select_far(const CollideArgs<R> &a, uint32_t cell, uint32_t n_near, uint32_t N,
                                           uint32_t *sel) {
    if (lane_id() == 0) {
        uint32_t k = a.far_head[cell], m = n_near;
        while (k != kEmpty && m < N) {
            sel[m++] = a.far_src[k];
            k = a.far_next[k];
        }
        if (k != kEmpty || m != N) set_error(a.st, DSMC_ECAPACITY);
        while (m < N) sel[m++] = 0u;
        a.far_head[cell] = kEmpty;
    }
}

// Position of source position q in the merged order: the number of smaller
// entries of sel[0..N) (only cells with far movers need it).
__device__ __forceinline__ uint32_t merged_rank(const uint32_t *sel, uint32_t N, uint32_t q) {
    uint32_t r = 0;
    for (uint32_t t = 0; t < N; ++t) r += sel[t] < q ? 1u : 0u;
    return r;
}

// J elements per lane (e0 + 64 j + lane): every load issued before the first
// store.  Positions, ids go straight to the new sequence; velocities and
// weights to LDS at the element's rank.
template <typename R, bool VR, int D, int J>
__device__ __forceinline__ void gather_j(const CollideArgs<R> &a, uint32_t base, uint32_t e0, uint32_t N,
                                         const uint32_t *sel, bool merge, R *vx, R *vy, R *vz, R *w) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t q[J], r[J], id[J];
    R x[J], y[J], c0[J], c1[J], c2[J], ww[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t el = e0 + 64u * (uint32_t)j + lane;
        q[j] = el < N ? sel[el] : 0u;
        r[j] = el;
    }
    if (merge) {
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (r[j] < N) r[j] = merged_rank(sel, N, q[j]);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (e0 + 64u * (uint32_t)j + lane < N) {
            x[j] = a.src.x[q[j]];
            if (D == 2) y[j] = a.src.y[q[j]];
            c0[j] = a.src.cx[q[j]]; c1[j] = a.src.cy[q[j]]; c2[j] = a.src.cz[q[j]];
            if (VR) ww[j] = a.src.w[q[j]];
            id[j] = a.src.id[q[j]];
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (e0 + 64u * (uint32_t)j + lane < N) {
            const uint32_t o = base + (r[j] < N ? r[j] : N - 1);
            a.s.x[o] = x[j];
            if (D == 2) a.s.y[o] = y[j];
            a.s.id[o] = id[j];
            const uint32_t rr = r[j] < N ? r[j] : N - 1;
            if (vx) {
                vx[rr] = c0[j]; vy[rr] = c1[j]; vz[rr] = c2[j];
                if (VR) w[rr] = ww[j];
            } else {
                a.s.cx[o] = c0[j]; a.s.cy[o] = c1[j]; a.s.cz[o] = c2[j];
                if (VR) a.s.w[o] = ww[j];
            }
        }
    }
}

// Whole gather of a walled cell: selection into sel (LDS or global scratch
// of at least N entries), then the particles into the new sequence at
// `base` (velocities and weights into LDS when vx is given, else into the
// new sequence too).
template <typename R, bool VR, int D>
__device__ __forceinline__ void gather_cell(const CollideArgs<R> &a, uint32_t cell, uint32_t base, uint32_t N,
                                            uint32_t *sel, R *vx, R *vy, R *vz, R *w) {
    uint32_t n_near = select_near<R, D>(a, cell, N, sel);
    if (n_near > N) {
        if (lane_id() == 0) set_error(a.st, DSMC_ECAPACITY);
        n_near = N;
    }
    const bool merge = n_near < N;
    if (merge) select_far(a, cell, n_near, N, sel);
    __syncthreads();
    uint32_t e0 = 0;
    for (; e0 + 256 <= N; e0 += 256) gather_j<R, VR, D, 4>(a, base, e0, N, sel, merge, vx, vy, vz, w);
    const uint32_t left = N - e0;
    if (left > 192) gather_j<R, VR, D, 4>(a, base, e0, N, sel, merge, vx, vy, vz, w);
    else if (left > 128) gather_j<R, VR, D, 3>(a, base, e0, N, sel, merge, vx, vy, vz, w);
    else if (left > 64) gather_j<R, VR, D, 2>(a, base, e0, N, sel, merge, vx, vy, vz, w);
    else if (left > 0) gather_j<R, VR, D, 1>(a, base, e0, N, sel, merge, vx, vy, vz, w);
}

// LDS kernel body: one wave per cell.  Homogeneous instances (D 0) collide
// in place in storage order; walled cells (D 1, 2) are gathered into the new
// sequence first.
template <typename R, bool VR, int D, bool LEARNED>
__device__ __forceinline__ void collide_lds_body(const CollideArgs<R> &a, unsigned char *smem, uint32_t cell) {
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
    const CellPrefetch pf = prefetch_cell<R, VR, true>(a, cell);
    const int cap = a.cap;
    R *vx = (R *)smem, *vy = vx + cap, *vz = vy + cap;
    R *w = VR ? vz + cap : nullptr;
    uint32_t *owner = (uint32_t *)(VR ? w + cap : vz + cap);  // cap + 4 entries
    if (D > 0) {
        gather_cell<R, VR, D>(a, cell, base, N, owner, vx, vy, vz, w);  // the owner array holds the selection
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
    // the sampling writes the cell back and reduces its sums through the
    // cell's LDS area
    if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf, (double *)smem, base);
    else process_cell<R, VR>(a, view, cell, N, step, pf, (double *)smem, base);
    __syncthreads();
}

// Global-memory kernel for cells larger than the LDS capacity: walled cells
// are gathered into the new sequence (selection in a global scratch array),
// then every cell is operated on in place.
template <typename R, bool VR, int D, bool LEARNED>
__device__ __forceinline__ void collide_big_body(const CollideArgs<R> &a) {
    const int lane = lane_id();
    const uint32_t step = (uint32_t)a.st->step_cur;
    const uint32_t nbig = a.st->big_count;
    for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const uint32_t cell = a.big_list[q];
        const uint32_t base = a.start[cell];
        const uint32_t N = a.start[cell + 1] - base;
        if (D > 0) {
            gather_cell<R, VR, D>(a, cell, base, N, a.perm_g + base, (R *)nullptr, (R *)nullptr, (R *)nullptr,
                                  (R *)nullptr);
            __syncthreads();
        }
        const GlobalView<R> view{a.s.cx + base, a.s.cy + base, a.s.cz + base,
                                 VR ? a.s.w + base : nullptr, nullptr, a.owner_g + base};
        for (uint32_t r = lane; r < N; r += 64) view.clear_own(r);
        __syncthreads();
        const CellPrefetch pf = prefetch_cell<R, VR, false>(a, cell);
        if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf);
        else process_cell<R, VR>(a, view, cell, N, step, pf);
        if (lane == 0) diag_add(a.st, kDiagBig, 1ull);
        __syncthreads();
    }
}

// At least five waves per SIMD: the register budget that the LDS footprint
// of a typical walled cell with weights also allows.
template <typename R, bool VR, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_collide(CollideArgs<R> a) {
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
