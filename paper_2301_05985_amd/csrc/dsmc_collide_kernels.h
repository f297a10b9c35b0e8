// dsmc_collide_kernels.h -- the collision kernels: cells staged in LDS (one
// wave per cell, two walled cells per wave, or a workgroup of waves per large
// homogeneous instance) and, for cells above the LDS capacity, a
// global-memory variant; each with the exact or the learned majorant (the
// two-cell kernel with the exact one).
#pragma once
#include "dsmc_collide.h"
#include "dsmc_learned.h"

namespace dsmc {

// ------------------------------------------------ gather of a walled cell
// Cell t of the new sequence holds, in order, the particles of the previous
// sequence whose new cell is t (a stable counting sort).  In ascending
// position these are the movers from cells before t, the particles that
// stayed in t (found from t's own range of code bytes), and the movers from
// cells after t: the movers, listed by the streaming pass in no particular
// order, are sorted across the wave and split at t's range.  Overflow movers
// (beyond the slot list, rare) are appended and the whole selection is then
// merged by position.

// Lane v ^ J of a 64-lane value (J a power of two).
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    else if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)v, 32, 64);
}

// One compare-exchange stage of a bitonic sort (block size K, distance J):
// ascending blocks keep the minimum on the lower lane.
template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_stage(uint32_t v, uint32_t lane) {
    const uint32_t o = xor_lane<J>(v);
    const bool keep_min = ((lane & J) == 0) == ((lane & K) == 0 || K == 64);
    const uint32_t lo = v < o ? v : o, hi = v < o ? o : v;
    return keep_min ? lo : hi;
}
template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_merge(uint32_t v, uint32_t lane) {
    v = bitonic_stage<K, J>(v, lane);
    if constexpr (J > 1) v = bitonic_merge<K, J / 2>(v, lane);
    return v;
}
// Ascending sort of one value per lane over the first W lanes (W 32 or 64).
template <int W>
__device__ __forceinline__ uint32_t bitonic_sort(uint32_t v, uint32_t lane) {
    v = bitonic_merge<2, 1>(v, lane);
    v = bitonic_merge<4, 2>(v, lane);
    v = bitonic_merge<8, 4>(v, lane);
    v = bitonic_merge<16, 8>(v, lane);
    v = bitonic_merge<(W == 32 ? 64 : 32), 16>(v, lane);  // W 32: the last stage, ascending
    if constexpr (W == 64) v = bitonic_merge<64, 32>(v, lane);
    return v;
}

// Ascending sort of C values per lane (element lane + L r in register r,
// L C elements; L = 64 a wave, 32 a half-wave cell with `lane` its cell
// lane): the same bitonic network, with the stages of distance L and more
// exchanging registers within a lane.
template <int C, int K, int J, int L = 64>
__device__ __forceinline__ void bitonic_stage_regs(uint32_t (&v)[4], uint32_t lane) {
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const bool asc = ((lane + (uint32_t)L * (uint32_t)r) & (uint32_t)K) == 0u;
        if constexpr (J >= L) {
            constexpr int R = J / L;
            if ((r & R) == 0) {
                const uint32_t a = v[r], b = v[r | R];
                const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                v[r] = asc ? lo : hi;
                v[r | R] = asc ? hi : lo;
            }
        } else {
            const uint32_t o = xor_lane<J>(v[r]);
            const bool keep_min = ((lane & (uint32_t)J) == 0u) == asc;
            const uint32_t lo = v[r] < o ? v[r] : o, hi = v[r] < o ? o : v[r];
            v[r] = keep_min ? lo : hi;
        }
    }
}
template <int C, int K, int J, int L = 64>
__device__ __forceinline__ void bitonic_merge_regs(uint32_t (&v)[4], uint32_t lane) {
    bitonic_stage_regs<C, K, J, L>(v, lane);
    if constexpr (J > 1) bitonic_merge_regs<C, K, J / 2, L>(v, lane);
}
template <int C, int K, int L = 64>
__device__ __forceinline__ void bitonic_sort_regs(uint32_t (&v)[4], uint32_t lane) {
    if constexpr (K > 2) bitonic_sort_regs<C, K / 2, L>(v, lane);
    bitonic_merge_regs<C, K, K / 2, L>(v, lane);
}

// Work bound of the merge of overflow movers (N x overflow entries): a cell
// above it reports DSMC_ECAPACITY and is not merged, so that a pathological
// state (say every particle at a NaN position, all in cell 0) costs bounded
// time.
constexpr uint64_t kMergeBudget = 1ull << 28;

// Selection of `cell`: source entries 2 p + flown (p the source position,
// flown set where the wall kernel already stored the final position) written
// to sel[0..N) (sel holds at least N entries).  Returns N, or, when overflow
// movers must still be merged by position, the length S of the ascending
// prefix sel[0..S) (the movers of the slot list and the stays; the overflow
// movers follow it in list order).  Any mismatch with the cell's count is
// reported, and sel is filled with valid positions.  T = 64: the wave;
// T = 32: the cell's half of a wave (at most 128 mover slots), whose mover
// sort is sized by m_wave, the larger mover count of the wave's two cells,
// so that both halves take the same branch.
template <typename R, int T = 64>
__device__ __forceinline__ uint32_t select_cell(const CollideArgs<R> &a, uint32_t cell, uint32_t N,
                                                uint32_t *sel, uint32_t m_wave = 0u) {
    constexpr uint32_t L = (uint32_t)T;
    constexpr int P = 128 / T;  // chunks of codes loaded at once
    const uint32_t lane = (uint32_t)cell_lane<T>();
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (N == 0) return 0u;  // nothing lands here (and the sequence may be empty)
    const uint32_t b = a.src_start[cell], e = a.src_start[cell + 1];
    const uint32_t mc = a.rg.mcount[cell];
    const uint32_t K = a.rg.slots;
    const uint32_t nm = mc < K ? mc : K;
    const uint32_t *ml = a.rg.movers + (size_t)cell * K;
    uint32_t v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t el = lane + L * (uint32_t)r;
        v[r] = 0xFFFFFFFFu;
        if (r == 0 || nm > L * (uint32_t)r) v[r] = el < nm ? ml[el] : 0xFFFFFFFFu;  // uniform test
    }
    // the codes of the cell's own range, the first chunks loaded at once;
    // every load below is issued from an in-bounds address (the sequence is
    // not empty) and masked afterwards
    const uint32_t last = e > b ? e - 1u : (b > 0u ? b - 1u : 0u);
    uint32_t ic[P];
    uint8_t cc[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
        ic[t] = b + L * (uint32_t)t + lane;
        cc[t] = a.rg.code[ic[t] < e ? ic[t] : last];
    }
    if constexpr (T == 64) {
        if (nm <= 32) v[0] = bitonic_sort<32>(v[0], lane);
        else if (nm <= 64) v[0] = bitonic_sort<64>(v[0], lane);
        else if (nm <= 128) bitonic_sort_regs<2, 128>(v, lane);
        else bitonic_sort_regs<4, 256>(v, lane);
    } else {
        const uint32_t ns = m_wave > nm ? (m_wave < K ? m_wave : K) : nm;  // padded entries sort last
        if (ns <= 32) v[0] = bitonic_sort<32>(v[0], lane);
        else if (ns <= 64) bitonic_sort_regs<2, 64, 32>(v, lane);
        else bitonic_sort_regs<4, 128, 32>(v, lane);
    }
    uint32_t nlow = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r > 0 && nm <= L * (uint32_t)r) break;
        const uint32_t el = lane + L * (uint32_t)r;
        nlow += (uint32_t)__popcll(cell_ballot<T>(el < nm && v[r] < 2u * b));  // entries sort by position
    }
    uint32_t nstay = 0;
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const bool m = ic[t] < e && (cc[t] & kStay) != 0;
        const unsigned long long bal = cell_ballot<T>(m);
        const uint32_t pos = nlow + nstay + (uint32_t)__popcll(bal & lt);
        if (m && pos < N) sel[pos] = 2u * ic[t] + ((cc[t] & kFlown) ? 1u : 0u);
        nstay += (uint32_t)__popcll(bal);
    }
    for (uint32_t c = b + 128u; c < e; c += L) {
        const uint32_t i = c + lane;
        const uint8_t ci = i < e ? a.rg.code[i] : (uint8_t)0;
        const bool m = (ci & kStay) != 0;
        const unsigned long long bal = cell_ballot<T>(m);
        const uint32_t pos = nlow + nstay + (uint32_t)__popcll(bal & lt);
        if (m && pos < N) sel[pos] = 2u * i + ((ci & kFlown) ? 1u : 0u);
        nstay += (uint32_t)__popcll(bal);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r > 0 && nm <= L * (uint32_t)r) break;
        const uint32_t el = lane + L * (uint32_t)r;
        if (el < nm) {
            const uint32_t pos = el < nlow ? el : el + nstay;
            if (pos < N) sel[pos] = v[r];
        }
    }
    const uint32_t S = nstay + nm;  // the ascending prefix (uniform over the cell)
    const bool over = mc > K;
    const uint32_t F = N > S ? N - S : 0u;
    const bool merge = over && (uint64_t)N * (uint64_t)F <= kMergeBudget;
    if (lane == 0) {
        uint32_t m = S;
        if (over) {
            if (merge) {
                // overflow movers from the list, merged by position afterwards
                uint32_t q = a.rg.far_head[cell];
                while (q != kEmpty && m < N) {
                    sel[m++] = a.rg.far_src[q];
                    q = a.rg.far_next[q];
                }
                if (q != kEmpty) set_error(a.st, DSMC_ECAPACITY);
            } else {
                set_error(a.st, DSMC_ECAPACITY);
            }
            a.rg.far_head[cell] = kEmpty;
        }
        if (m != N) set_error(a.st, DSMC_ECAPACITY);
        while (m < N) sel[m++] = 2u * last;  // valid positions only (b itself may be the end of the sequence)
        if (mc) a.rg.mcount[cell] = 0u;
    }
    return merge && S < N ? S : N;
}

// Position in the merged order of entry i (value q) of sel[0..N), whose
// prefix sel[0..S) ascends and whose rest holds the overflow movers: the
// number of smaller entries (the entries are distinct positions), that is i
// or the lower bound of q in the prefix, plus the smaller overflow entries.
__device__ __forceinline__ uint32_t merged_rank(const uint32_t *sel, uint32_t S, uint32_t N, uint32_t i,
                                                uint32_t q) {
    uint32_t r = i;
    if (i >= S) {
        uint32_t lo = 0, hi = S;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sel[mid] < q) lo = mid + 1u;
            else hi = mid;
        }
        r = lo;
    }
    for (uint32_t t = S; t < N; ++t) r += sel[t] < q ? 1u : 0u;
    return r;
}

// J elements per lane (e0 + T j + lane, T the cell's lanes): every load
// issued before the first store.  Positions, ids go straight to the new
// sequence; velocities and weights to LDS at the element's rank.  A particle
// the wall kernel did not fly is moved to its end point x + c dt here.
template <typename R, bool VR, int D, int J, int T = 64>
__device__ __forceinline__ void gather_j(const CollideArgs<R> &a, uint32_t base, uint32_t e0, uint32_t N,
                                         const uint32_t *sel, uint32_t S, Vel4<R> *vel, BoxKeys *box) {
    const uint32_t lane = (uint32_t)cell_lane<T>();
    uint32_t q[J], r[J], id[J];
    R x[J], y[J], c0[J], c1[J], c2[J], ww[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t el = e0 + (uint32_t)T * (uint32_t)j + lane;
        q[j] = el < N ? sel[el] : 0u;
        r[j] = el;
    }
    if (S < N) {
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (r[j] < N) r[j] = merged_rank(sel, S, N, r[j], q[j]);
    }
    bool flown[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        flown[j] = (q[j] & 1u) != 0u;
        if (e0 + (uint32_t)T * (uint32_t)j + lane < N) {
            const uint32_t p = bounds_ck(q[j] >> 1, a.n_total, a.st);
            x[j] = a.src.x[p];
            if (D == 2) y[j] = a.src.y[p];
            c0[j] = a.src.cx[p]; c1[j] = a.src.cy[p]; c2[j] = a.src.cz[p];
            if (VR) ww[j] = a.src.w[p];
            id[j] = a.src.id[p];
        }
    }
    const R tau = (R)a.dt;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (e0 + (uint32_t)T * (uint32_t)j + lane < N) {
            if (!flown[j]) {
                x[j] = x[j] + c0[j] * tau;
                if (D == 2) y[j] = y[j] + c1[j] * tau;
            }
            const uint32_t o = bounds_ck(base + (r[j] < N ? r[j] : N - 1), a.n_total, a.st);
            a.s.x[o] = x[j];
            if (D == 2) a.s.y[o] = y[j];
            a.s.id[o] = id[j];
            const uint32_t rr = r[j] < N ? r[j] : N - 1;
            if constexpr (sizeof(R) == 4) {
                if (box) box_keys_add(*box, c0[j], c1[j], c2[j]);
            }
            if (vel) {
                vel[rr] = Vel4<R>{c0[j], c1[j], c2[j], VR ? ww[j] : (R)1};
            } else {
                a.s.cx[o] = c0[j]; a.s.cy[o] = c1[j]; a.s.cz[o] = c2[j];
                if (VR) a.s.w[o] = ww[j];
            }
        }
    }
}

// Whole gather of a walled cell: selection into sel (LDS or global scratch
// of at least N entries), then the particles into the new sequence at
// `base` (velocities and weights into LDS when vel is given, else into the
// new sequence too).
// (box, FP32: this lane's running minima of the velocity keys, which the
// exact majorant takes instead of a pass of its own over the cell.)
// (WG_BARRIER false: called by one wave of a larger workgroup, which orders
// its own LDS accesses with a wave-scope fence instead of a barrier.  Half-wave
// cells: N_wave and m_wave are the larger cell size and mover count of the
// wave's two cells, from which the unrolling and the sort are chosen, so
// that the halves do not run two variants one after the other.)
template <typename R, bool VR, int D, int T = 64, bool WG_BARRIER = true>
__device__ __forceinline__ void gather_cell(const CollideArgs<R> &a, uint32_t cell, uint32_t base, uint32_t N,
                                            uint32_t *sel, Vel4<R> *vel, uint32_t N_wave = 0u,
                                            uint32_t m_wave = 0u, BoxKeys *box = nullptr) {
    constexpr uint32_t L = (uint32_t)T;
    const uint32_t S = select_cell<R, T>(a, cell, N, sel, m_wave);  // N: no merge
    if constexpr (WG_BARRIER) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t Nb = N_wave > N ? N_wave : N;  // elements at N and above are masked in gather_j
    uint32_t e0 = 0;
    for (; e0 + 4 * L <= Nb; e0 += 4 * L) gather_j<R, VR, D, 4, T>(a, base, e0, N, sel, S, vel, box);
    const uint32_t left = Nb - e0;
    if (left > 3 * L) gather_j<R, VR, D, 4, T>(a, base, e0, N, sel, S, vel, box);
    else if (left > 2 * L) gather_j<R, VR, D, 3, T>(a, base, e0, N, sel, S, vel, box);
    else if (left > L) gather_j<R, VR, D, 2, T>(a, base, e0, N, sel, S, vel, box);
    else if (left > 0) gather_j<R, VR, D, 1, T>(a, base, e0, N, sel, S, vel, box);
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
            const uint32_t q = atomicAdd(a.bigc, 1u);
            a.big_list[q] = cell;
        }
        return;
    }
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const auto pf = prefetch_cell<R, VR, true>(a, cell);
    const int cap = a.cap;
    constexpr bool kPacked = D == 0 && !VR;  // owner marks in the weight slots
    Vel4<R> *vel = (Vel4<R> *)smem;
    uint32_t *owner = kPacked ? nullptr : (uint32_t *)(vel + cap);  // cap + 4 entries
    if (D > 0) {
        gather_cell<R, VR, D>(a, cell, base, N, owner, vel);  // the owner array holds the selection
        __syncthreads();
    } else {
        // staged four rows of 64 at a time: all their loads are in flight
        // before the first LDS store
        for (uint32_t s0 = 0; s0 < N; s0 += 256) {
            Vel4<R> t[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t s = s0 + 64u * (uint32_t)j + (uint32_t)lane;
                if (s < N)
                    t[j] = Vel4<R>{a.s.cx[base + s], a.s.cy[base + s], a.s.cz[base + s],
                                   VR ? a.s.w[base + s] : (R)1};
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t s = s0 + 64u * (uint32_t)j + (uint32_t)lane;
                if (s < N) vel[s] = t[j];
            }
        }
    }
    const LdsView<R, kPacked> view{vel, owner, view_check((uint32_t)cap, a.st)};
    for (uint32_t r = lane; r < N; r += 64) view.clear_own(r);
    __syncthreads();
    // the sampling writes the cell back and reduces its sums through the
    // cell's LDS area
    if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf, (double *)smem, base);
    else process_cell<R, VR>(a, view, cell, N, step, pf, (double *)smem, base);
    __syncthreads();
}

// Two walled cells per wave, 32 lanes each: lanes 0-31 take schedule entry
// 2 b of workgroup b, lanes 32-63 entry 2 b + 1 (kNoCell: none).  Each half
// gathers, collides and samples its cell in its own LDS area of
// pair_area_bytes(cap) bytes by the same steps as the one-wave kernel, every
// cross-lane operation staying inside the half; a wave's 64 lanes then carry
// two windows of candidates instead of one mostly idle one.
constexpr uint32_t kNoCell = 0xFFFFFFFFu;
template <typename R>
__host__ __device__ constexpr size_t pair_area_bytes(int cap) {
    const size_t part = (size_t)cap * (sizeof(Vel4<R>) + 4) + 16 + 16;  // particles, owner marks (+4)
    const size_t red = (size_t)13 * 32 * 8;                             // moment transpose
    return ((part > red ? part : red) + 15) / 16 * 16;
}

template <typename R, bool VR, int D>
__device__ __forceinline__ void collide_pair_body(const CollideArgs<R> &a, unsigned char *smem) {
    constexpr int T = 32;
    const uint32_t half = (uint32_t)lane_id() >> 5;
    const uint32_t lane = cell_tid<T>();
    const uint32_t cell = a.sched[2 * blockIdx.x + half];
    const bool has = cell != kNoCell;
    const uint32_t base = has ? a.start[cell] : 0u;
    const uint32_t N = has ? a.start[cell + 1] - base : 0u;
    // the larger size and mover count of the wave's cells staged here (taken
    // while all 64 lanes are active): the gather's unrolling and mover sort
    // are chosen from them
    const bool staged = has && N <= (uint32_t)a.cap;
    const uint32_t Ns = staged ? N : 0u, ms = staged ? a.rg.mcount[cell] : 0u;
    const uint32_t N_wave = max(Ns, (uint32_t)__shfl_xor((int)Ns, 32, 64));
    const uint32_t m_wave = max(ms, (uint32_t)__shfl_xor((int)ms, 32, 64));
    if (!has) return;
    if (N > (uint32_t)a.cap) {
        if (lane == 0) {
            const uint32_t q = atomicAdd(a.bigc, 1u);
            a.big_list[q] = cell;
        }
        return;
    }
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const auto pf = prefetch_cell<R, VR, true, T>(a, cell);
    const int cap = a.cap;
    unsigned char *area = smem + (size_t)half * pair_area_bytes<R>(cap);
    Vel4<R> *vel = (Vel4<R> *)area;
    uint32_t *owner = (uint32_t *)(vel + cap);  // cap + 4 entries; first the gather's selection
    // FP32: the majorant's velocity box is taken while the gather holds the
    // velocities in registers
    constexpr bool kBox = sizeof(R) == 4;
    BoxKeys box = ~0u;
    gather_cell<R, VR, D, T>(a, cell, base, N, owner, vel, N_wave, m_wave, kBox ? &box : nullptr);
    __syncthreads();
    const LdsView<R, false> view{vel, owner, view_check((uint32_t)cap, a.st)};
    for (uint32_t r = lane; r < N; r += T) view.clear_own(r);
    __syncthreads();
    process_cell<R, VR, LdsView<R, false>, T>(a, view, cell, N, step, pf, (double *)area, base, nullptr, kBox, box);
    __syncthreads();
}

// Walled cells on a workgroup of kWideThreads threads each (four waves): the
// first wave selects and gathers the cell into LDS exactly as the one-wave
// kernel does, then the workgroup collides and samples it as a large
// homogeneous instance is (particle loops over 256 threads, windows of 256
// candidates).  For grids of few, populous cells, where one wave per cell
// would leave most of the GPU idle.
template <typename R, bool VR, int D>
__device__ __forceinline__ void collide_walled_wide_body(const CollideArgs<R> &a, unsigned char *smem) {
    constexpr int T = kWideThreads;
    const uint32_t tid = threadIdx.x;
    const uint32_t cell = a.sched ? a.sched[blockIdx.x] : blockIdx.x;
    const uint32_t base = a.start[cell];
    const uint32_t N = a.start[cell + 1] - base;
    if (N > (uint32_t)a.cap) {
        if (tid == 0) {
            const uint32_t q = atomicAdd(a.bigc, 1u);
            a.big_list[q] = cell;
        }
        return;  // the whole workgroup
    }
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const auto pf = prefetch_cell<R, VR, false>(a, cell);
    const int cap = a.cap;
    Vel4<R> *vel = (Vel4<R> *)smem;
    uint32_t *owner = (uint32_t *)(vel + cap);  // cap + 4 entries; first the gather's selection
    GroupScratch *gs = (GroupScratch *)(owner + cap + 4);
    if (tid < 64u) gather_cell<R, VR, D, 64, false>(a, cell, base, N, owner, vel);
    __syncthreads();
    const LdsView<R, false> view{vel, owner, view_check((uint32_t)cap, a.st)};
    for (uint32_t r = tid; r < N; r += T) view.clear_own(r);
    __syncthreads();
    process_cell<R, VR, LdsView<R, false>, T>(a, view, cell, N, step, pf, nullptr, base, gs);
}

// Global-memory kernel for cells larger than the LDS capacity: walled cells
// are gathered into the new sequence (selection in a global scratch array),
// then every cell is operated on in place.
template <typename R, bool VR, int D, bool LEARNED>
__device__ __forceinline__ void collide_big_body(const CollideArgs<R> &a) {
    const int lane = lane_id();
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const uint32_t nbig = *a.bigc;
    for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const uint32_t cell = a.big_list[q];
        const uint32_t base = a.start[cell];
        const uint32_t N = a.start[cell + 1] - base;
        if (D > 0) {
            gather_cell<R, VR, D>(a, cell, base, N, a.perm_g + base, (Vel4<R> *)nullptr);
            __syncthreads();
        }
        const GlobalView<R> view{a.s.cx + base, a.s.cy + base, a.s.cz + base,
                                 VR ? a.s.w + base : nullptr, nullptr, a.owner_g + base, view_check(N, a.st)};
        for (uint32_t r = lane; r < N; r += 64) view.clear_own(r);
        __syncthreads();
        const auto pf = prefetch_cell<R, VR, false>(a, cell);
        if (LEARNED) process_cell_learned<R, VR>(a, view, cell, N, step, pf);
        else process_cell<R, VR>(a, view, cell, N, step, pf);
        if (lane == 0) diag_add(a.st, kDiagBig, 1ull);
        __syncthreads();
    }
}

// At least OCC waves per SIMD (5 by default: the register budget that the
// LDS footprint of a typical walled cell with weights also allows; 6 is
// compiled too for homogeneous instances, where the autotuner picks one).
template <typename R, bool VR, int D, int OCC = 5>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) void k_collide(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_lds_body<R, VR, D, false>(a, smem, a.sched ? a.sched[blockIdx.x] : blockIdx.x);
}

// Two walled cells per wave: five waves per SIMD (the kernel fits their 96
// registers without spills; in FP32 the LDS of two cells of the pair
// capacity allows more).
template <typename R, bool VR, int D, int OCC = 5>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) void k_collide_pair(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_pair_body<R, VR, D>(a, smem);
}

template <typename R, bool VR, int D>
__global__ __launch_bounds__(kWideThreads) void k_collide_walled_wide(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_walled_wide_body<R, VR, D>(a, smem);
}

// Large homogeneous instances: one workgroup of kWideThreads threads per
// instance (the particle loops spread over its waves, NTC windows of
// kWideThreads consecutive candidates), so that an instance of a few
// thousand particles does not run on a single wave held by its LDS size.
template <typename R, bool VR, bool LEARNED>
__device__ __forceinline__ void collide_wide_body(const CollideArgs<R> &a, unsigned char *smem) {
    constexpr int T = kWideThreads;
    const uint32_t tid = threadIdx.x;
    const uint32_t cell = a.sched[blockIdx.x];
    const uint32_t base = a.start[cell];
    const uint32_t N = a.start[cell + 1] - base;
    if (N > (uint32_t)a.cap) {
        if (tid == 0) {
            const uint32_t q = atomicAdd(a.bigc, 1u);
            a.big_list[q] = cell;
        }
        return;
    }
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const auto pf = prefetch_cell<R, VR, false>(a, cell);
    const int cap = a.cap;
    constexpr bool kPacked = !VR;  // owner marks in the weight slots
    Vel4<R> *vel = (Vel4<R> *)smem;
    uint32_t *owner = kPacked ? nullptr : (uint32_t *)(vel + cap);
    // 16-byte aligned: cap is a multiple of 32
    GroupScratch *gs = kPacked ? (GroupScratch *)(vel + cap) : (GroupScratch *)(owner + cap + 4);
    for (uint32_t s0 = 0; s0 < N; s0 += 2 * T) {
        Vel4<R> t[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t s = s0 + (uint32_t)T * (uint32_t)j + tid;
            if (s < N)
                t[j] = Vel4<R>{a.s.cx[base + s], a.s.cy[base + s], a.s.cz[base + s], VR ? a.s.w[base + s] : (R)1};
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t s = s0 + (uint32_t)T * (uint32_t)j + tid;
            if (s < N) vel[s] = t[j];
        }
    }
    const LdsView<R, kPacked> view{vel, owner, view_check((uint32_t)cap, a.st)};
    for (uint32_t r = tid; r < N; r += T) view.clear_own(r);
    __syncthreads();
    if (LEARNED) process_cell_learned<R, VR, LdsView<R, kPacked>, T>(a, view, cell, N, step, pf, nullptr, base, gs);
    else process_cell<R, VR, LdsView<R, kPacked>, T>(a, view, cell, N, step, pf, nullptr, base, gs);
}

// Homogeneous instances above the LDS capacity: one kWideThreads workgroup
// each, operating on the instance in global memory (owner marks in the
// global scratch array, read and set by device-scope atomics).
template <typename R, bool VR, bool LEARNED>
__device__ __forceinline__ void collide_big_wide_body(const CollideArgs<R> &a) {
    constexpr int T = kWideThreads;
    __shared__ GroupScratch gs;
    const uint32_t step = (uint32_t)(a.st->step_cur + a.step_off);
    const uint32_t nbig = *a.bigc;
    for (uint32_t q = blockIdx.x; q < nbig; q += gridDim.x) {
        const uint32_t cell = a.big_list[q];
        const uint32_t base = a.start[cell];
        const uint32_t N = a.start[cell + 1] - base;
        const GlobalView<R> view{a.s.cx + base, a.s.cy + base, a.s.cz + base,
                                 VR ? a.s.w + base : nullptr, nullptr, a.owner_g + base, view_check(N, a.st)};
        for (uint32_t r = threadIdx.x; r < N; r += T) view.clear_own(r);
        __syncthreads();
        const auto pf = prefetch_cell<R, VR, false>(a, cell);
        if (LEARNED) process_cell_learned<R, VR, GlobalView<R>, T>(a, view, cell, N, step, pf, nullptr, 0, &gs);
        else process_cell<R, VR, GlobalView<R>, T>(a, view, cell, N, step, pf, nullptr, 0, &gs);
        if (threadIdx.x == 0) diag_add(a.st, kDiagBig, 1ull);
        __syncthreads();
    }
}

template <typename R, bool VR>
__global__ __launch_bounds__(kWideThreads) void k_collide_big_wide(CollideArgs<R> a) {
    collide_big_wide_body<R, VR, false>(a);
}

template <typename R, bool VR>
__global__ __launch_bounds__(kWideThreads) void k_collide_big_wide_learned(CollideArgs<R> a) {
    collide_big_wide_body<R, VR, true>(a);
}

template <typename R, bool VR>
__global__ __launch_bounds__(kWideThreads) void k_collide_wide(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_wide_body<R, VR, false>(a, smem);
}

template <typename R, bool VR>
__global__ __launch_bounds__(kWideThreads) void k_collide_wide_learned(CollideArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    collide_wide_body<R, VR, true>(a, smem);
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
        if (lane_id() == 0) k = atomicAdd(&a.queue[q * kQueueStride], 1u);
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
        if (lane_id() == 0) pending = atomicAdd(&a.queue[q * kQueueStride], 1u);
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
            if (lane_id() == 0) k = atomicAdd(&a.queue[q * kQueueStride], 1u);
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
// pairs, in double); -inf for cells with fewer than two particles.  A
// workgroup of kCollectThreads per cell: the pairs are spread over all its
// threads (the maximum does not depend on the order), the O(N) features and
// bound are taken on the first wave.  Optionally log2 of the exact bound and
// log2 of the 65th largest r_p + r_(1) (radii about the velocity box
// midpoint, as in the verification; -inf when N <= 64): a proposal passes
// the verification's limit |S| <= 64 exactly when its verification
// threshold is at least that value.  It is found by bisection on the
// threshold (60 halvings of [0, 2 r_(1)], counting the members above it).
constexpr int kCollectThreads = 256;

template <typename R>
__global__ __launch_bounds__(kCollectThreads) void k_collect_features(CollideArgs<R> a, int ncell, float *feat,
                                                                      float *label, float *bound, float *slim) {
    __shared__ double wave_best[kCollectThreads / 64];
    const int lane = lane_id();
    const uint32_t tid = threadIdx.x;
    const uint32_t cell = blockIdx.x;
    if ((int)cell >= ncell) return;
    const uint32_t base = a.start[cell];
    const uint32_t N = a.start[cell + 1] - base;
    const GlobalView<R> v{a.s.cx + base, a.s.cy + base, a.s.cz + base, nullptr, nullptr, nullptr};
    if (N < 2) {
        if (tid < 6) feat[(size_t)cell * 6 + tid] = 0.0f;
        if (tid == 0) label[cell] = -INFINITY;
        if (tid == 0 && bound) bound[cell] = -INFINITY;
        if (tid == 0 && slim) slim[cell] = -INFINITY;
        return;
    }
    double best = 0.0;
    for (uint32_t r = tid; r < N; r += kCollectThreads) {
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
    if (lane == 0) wave_best[tid >> 6] = best;
    __syncthreads();
    if (tid >= 64) return;
#pragma unroll
    for (int w = 1; w < kCollectThreads / 64; ++w) best = fmax(best, wave_best[w]);
    const double V = a.volume ? a.volume[cell] : a.Vuni;
    const Features F = cell_features<R>(v, N, a.FN, V);
    if (lane < 6) feat[(size_t)cell * 6 + lane] = F.f[lane == 0 ? 0 : lane == 1 ? 1 : lane == 2 ? 2 : lane == 3 ? 3 : lane == 4 ? 4 : 5];
    if (lane == 0) label[cell] = (float)log2(sqrt(best));
    if (bound || slim) {
        double rt, mid[3];
        const double gb = exact_bound<R>(v, N, rt, nullptr, mid);
        if (lane == 0 && bound) bound[cell] = (float)log2(gb);
        if (slim) {
            float out = -INFINITY;
            if (N > 64u) {
                const auto above = [&](double thr) {
                    uint32_t cnt = 0;
                    for (uint32_t r = lane; r < N; r += 64) {
                        R x, y, z;
                        v.get(r, x, y, z);
                        const double dx = (double)x - mid[0], dy = (double)y - mid[1], dz = (double)z - mid[2];
                        cnt += (sqrt((dx * dx + dy * dy) + dz * dz) + rt > thr) ? 1u : 0u;
                    }
                    return wave_sum_u32(cnt);
                };
                double lo = 0.0, hi = 2.0 * rt * (1.0 + 0x1.0p-40) + 1e-300;
                for (int it = 0; it < 60; ++it) {
                    const double m = 0.5 * (lo + hi);
                    if (above(m) <= 64u) hi = m; else lo = m;
                }
                out = (float)log2(hi);
            }
            if (lane == 0) slim[cell] = out;
        }
    }
}

}  // namespace dsmc
