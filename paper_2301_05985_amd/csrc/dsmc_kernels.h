// dsmc_kernels.h -- the per-step kernels of the DSMC hot path on gfx950.
//
// One time step (Bird 1994, direct simulation Monte Carlo), walled runs:
//   k_stream_code     end points of the particles that stay in the box (the
//                     positions themselves are advanced by the gather), new
//                     cell counted, one code byte each, movers listed; the others go
//                     to the wall list                       [grid over particles]
//   k_stream_walls    exact flight with wall conditions of the wall list
//   k_scan_lookback   exclusive scan of the counts into the new cell ranges,
//                     step bookkeeping                   [decoupled look-back]
//   k_collide         per cell (dsmc_collide_kernels.h; k_collide_pair takes
//                     two cells per wave): gather the cell's
//                     particles from the previous sequence (stays and movers),
//                     majorant, NTC candidates in conflict-free wave batches,
//                     importance weights, FP64 moment sums [one wave per cell]
// Homogeneous instances (dims == 0) run k_begin_step and k_collide only.
#pragma once
#include "dsmc_device.h"
#include "../../include/dsmc.h"

namespace dsmc {

// Diagnostic counters are striped over kDiagStripes cache lines (workgroup
// index modulo the stripe count): thousands of workgroups adding to one
// address would serialize in a single L2 channel.  The host sums the stripes.
constexpr int kDiagStripes = 1024;
constexpr int kDiagPerStripe = 8;
// One queue per XCD (workgroups are dealt to the eight XCDs round-robin), so
// that the queue atomics of one step spread over eight addresses.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;
constexpr int kStepSlots = 8;

struct DevState {
    unsigned long long step_next;   // index of the next step to stream
    unsigned long long step_cur;    // index of the step being collided
    unsigned long long n_samples;   // sampled steps since the last reset
    unsigned int error;             // first device error (positive code), 0 = none
    unsigned int big_count;         // walled runs: cells queued for the global-memory collision kernel
    unsigned int far_count;         // entries of this step's overflow mover list
    unsigned int wall_count;        // entries of this step's wall list
    unsigned int max_cell;          // set-up: the largest initial cell
    unsigned long long pad[3];
    unsigned long long diag[kDiagStripes * kDiagPerStripe];
    // Homogeneous runs record up to kStepSlots steps per graph with a single
    // bookkeeping launch in front; step k of the batch uses slot k: its
    // big-instance count and the work-unit queues of the persistent
    // collision kernel (one 128-byte line each: queue q hands out the units
    // q, q + kQueues, q + 2 kQueues, ...).
    unsigned int big_slot[kStepSlots];
    unsigned int queue[kStepSlots * kQueues * kQueueStride];
};
enum { kDiagOvershoot = 0, kDiagWallHits, kDiagLearned, kDiagFallback, kDiagSkip, kDiagVrNonfinite,
       kDiagBig, kDiagBounds };

__device__ __forceinline__ void diag_add(DevState *st, int which, unsigned long long v) {
    atomicAdd(&st->diag[(blockIdx.x & (kDiagStripes - 1)) * kDiagPerStripe + which], v);
}

// Index check of the bounds-checking build (compiled with
// -DDSMC_BOUNDS_CHECK): an index outside [0, n) is counted in the
// diagnostics and replaced by 0, so that the access stays inside the array.
// The release build returns the index unchanged.
__device__ __forceinline__ uint32_t bounds_ck(uint32_t i, uint32_t n, DevState *st) {
#ifdef DSMC_BOUNDS_CHECK
    if (i >= n) {
        diag_add(st, kDiagBounds, 1ull);
        return 0u;
    }
#else
    (void)n;
    (void)st;
#endif
    return i;
}

__device__ __forceinline__ void set_error(DevState *st, int code) {
    atomicCAS(&st->error, 0u, (unsigned int)(-code));
}

struct Geo {
    int dims, nx, ny, max_hits;
    double Lx, Ly, dt, invx, invy;
    int kind[4];
    double Tw[4];
    double ux[4], uy[4], uz[4];  // wall velocities by component
    double T0;
    uint32_t k0, k1;
};

template <typename R>
struct Soa {
    R *x, *y, *cx, *cy, *cz, *w;
    uint32_t *id;
};

// ------------------------------------------------------------ diffuse wall
// Outgoing velocity drawn from the wall's normalized flux Maxwellian:
// normal speed sqrt(-2 Tw ln(1-U1)), tangential Box-Muller pair from
// (U2, U3) scaled by sqrt(Tw).  Double: U1, U2 from block 0 (two words
// each), U3 from block 1; float: U1..U3 from words 0..2 of block 0.
__device__ __forceinline__ void wall_draw(float Tw, uint32_t hit, uint32_t pid, uint32_t step,
                                          uint32_t k0, uint32_t k1, float &cn, float &t1, float &t2) {
    const u32x4 b = draw(hit, kTagWall, 0, pid, step, k0, k1);
    const float U1 = unif24(b.v[0]), U2 = unif24(b.v[1]), U3 = unif24(b.v[2]);
    const float rad = sqrtf(-2.0f * logf(1.0f - U2));
    const float th = 6.28318530717958647692f * U3;
    const float sT = sqrtf(Tw);
    cn = sqrtf((-2.0f * Tw) * logf(1.0f - U1));
    t1 = sT * (rad * cosf(th));
    t2 = sT * (rad * sinf(th));
}
__device__ __forceinline__ void wall_draw(double Tw, uint32_t hit, uint32_t pid, uint32_t step,
                                          uint32_t k0, uint32_t k1, double &cn, double &t1, double &t2) {
    const u32x4 b0 = draw(hit, kTagWall, 0, pid, step, k0, k1);
    const u32x4 b1 = draw(hit, kTagWall, 1, pid, step, k0, k1);
    const double U1 = unif53(b0.v[0], b0.v[1]), U2 = unif53(b0.v[2], b0.v[3]);
    const double U3 = unif53(b1.v[0], b1.v[1]);
    const double rad = sqrt(-2.0 * log(1.0 - U2));
    const double th = 6.28318530717958647692 * U3;
    const double sT = sqrt(Tw);
    cn = sqrt((-2.0 * Tw) * log(1.0 - U1));
    t1 = sT * (rad * cos(th));
    t2 = sT * (rad * sin(th));
}

// Importance-weight factor at a diffuse wall: flux Maxwellian of the
// reference equilibrium (T0, at rest) over that of the wall (Tw, uw).
__device__ __forceinline__ double wall_weight_ratio(double vx, double vy, double vz, double Tw,
                                                    const double *uw, double T0) {
    const double c2_0 = (vx * vx + vy * vy) + vz * vz;
    const double dx = vx - uw[0], dy = vy - uw[1], dz = vz - uw[2];
    const double c2_w = (dx * dx + dy * dy) + dz * dz;
    const double ex = c2_w / (2.0 * Tw) - c2_0 / (2.0 * T0);
    return ((Tw * Tw) / (T0 * T0)) * exp(ex);
}

// Element w of a 4-entry argument array by selects (a dynamic index into a
// kernel-argument array would copy the array to scratch memory).
template <typename T>
__device__ __forceinline__ T pick4(const T (&a)[4], int w) {
    return w == 0 ? a[0] : (w == 1 ? a[1] : (w == 2 ? a[2] : a[3]));
}

// ------------------------------------------------------------ free flight
// The free end point x + c tau is tried first: inside the closed box the
// particle simply moves there (no division).  Otherwise exact times of flight
// to the walls the particle moves toward decide the wall met first; a hit
// snaps the particle onto the wall, applies the wall condition and continues
// with the remaining time; on a tie the x wall goes first.  Returns 0 or
// DSMC_EWALLHITS.  The particle id is read only when a diffuse wall is hit.
// cz is only written (at diffuse walls); w is read from wsrc[p] at the
// first diffuse hit.  diffuse reports whether one happened.
template <typename R, int D, bool WANT_W>
__device__ __forceinline__ int fly(const Geo &g, R &x, R &y, R &cx, R &cy, R &cz, R &w,
                                   const uint32_t *ids, const R *wsrc, int64_t p, uint32_t step, uint32_t &hits,
                                   bool &diffuse) {
    const R Lx = (R)g.Lx, Ly = (R)g.Ly, zero = (R)0;
    const R inf = (R)INFINITY;
    R tau = (R)g.dt;
    hits = 0;
    diffuse = false;
    uint32_t pid = 0;
    bool have_pid = false;
    for (;;) {
        const R xe = x + cx * tau;
        const R ye = D == 2 ? y + cy * tau : zero;
        if (xe >= zero && xe <= Lx && (D < 2 || (ye >= zero && ye <= Ly))) {
            x = xe;
            if (D == 2) y = ye;
            return 0;
        }
        R tx = inf, ty = inf;
        if (cx > zero) tx = (Lx - x) / cx;
        else if (cx < zero) tx = (zero - x) / cx;
        if (D == 2) {
            if (cy > zero) ty = (Ly - y) / cy;
            else if (cy < zero) ty = (zero - y) / cy;
        }
        R t = tx <= ty ? tx : ty;
        if (t < zero) t = zero;
        if (t >= tau) {
            x = x + cx * tau;
            if (D == 2) y = y + cy * tau;
            return 0;
        }
        const bool xwall = tx <= ty;
        x = x + cx * t;
        if (D == 2) y = y + cy * t;
        tau = tau - t;
        int wall;
        if (xwall) { wall = cx > zero ? 1 : 0; x = wall ? Lx : zero; }
        else       { wall = cy > zero ? 3 : 2; y = wall == 3 ? Ly : zero; }
        if ((int)hits >= g.max_hits) return DSMC_EWALLHITS;
        const int kind = pick4(g.kind, wall);
        if (kind == DSMC_WALL_PERIODIC) {
            if (xwall) x = wall ? zero : Lx;
            else       y = wall == 3 ? zero : Ly;
        } else if (kind == DSMC_WALL_SPECULAR) {
            if (xwall) cx = -cx; else cy = -cy;
        } else {
            if (!have_pid) {
                pid = ids[p];
                have_pid = true;
                if (WANT_W) w = wsrc[p];
            }
            diffuse = true;
            R dn, d1, d2;
            const double Tw = pick4(g.Tw, wall);
            wall_draw((R)Tw, hits, pid, step, g.k0, g.k1, dn, d1, d2);
            const R sign = (wall & 1) ? (R)-1 : (R)1;
            const double uw[3] = {pick4(g.ux, wall), pick4(g.uy, wall), pick4(g.uz, wall)};
            if (xwall) { cx = sign * dn; cy = d1 + (R)uw[1]; cz = d2 + (R)uw[2]; }
            else       { cy = sign * dn; cx = d1 + (R)uw[0]; cz = d2 + (R)uw[2]; }
            if (WANT_W) {
                const double ratio = wall_weight_ratio((double)cx, (double)cy, (double)cz, Tw, uw, g.T0);
                w = (R)((double)w * ratio);
            }
        }
        hits++;
    }
}

// Cell coordinates floor(x nx / Lx), floor(y ny / Ly), each clamped to the
// grid (NaN to 0), in double; 2-D cells are numbered iy * nx + ix.  The
// product is clamped to [0, n - 1] first (max returns 0 for NaN), where
// truncation equals floor.
__device__ __forceinline__ int cell_coord(double t, int n) {
    return (int)fmin(fmax(t, 0.0), (double)(n - 1));
}
__device__ __forceinline__ void cell_coords(const Geo &g, double x, double y, int &ix, int &iy) {
    ix = cell_coord(x * g.invx, g.nx);
    iy = g.dims == 2 ? cell_coord(y * g.invy, g.ny) : 0;
}
__device__ __forceinline__ uint32_t cell_index(const Geo &g, double x, double y) {
    int ix, iy;
    cell_coords(g, x, y, ix, iy);
    return (uint32_t)iy * (uint32_t)g.nx + (uint32_t)ix;
}

// ------------------------------------------------------------ regrouping
// The particle sequence is regrouped every step by a stable counting sort on
// the new cell.  Streaming marks each particle that stays in its cell
// (code byte with kStay) and appends the position of each particle that changes
// cell (a mover) to a list of its new cell: 64, 128 or 256 slots per cell, the
// rest (rare) linked into a per-cell overflow list.  The collision wave of
// cell t then has, in ascending position, the movers from cells before t,
// the particles that stayed in t, and the movers from cells after t: the
// stays are found from t's own codes, the movers by sorting t's short list.
//
// Particles whose end point lies in the box keep their stored position: the
// gather, which loads every particle anyway, moves them to x + c dt (the
// same float operations as the streaming kernel's end point).  Particles of
// the wall list are flown exactly by the second kernel, which stores their
// final position and flags it: kFlown in the code byte, and bit 0 of the list
// entry, which holds position p as 2 p + flown (the entries still sort by
// position).
constexpr uint8_t kStay = 1;
constexpr uint8_t kMoved = 0;
constexpr uint8_t kFlown = 2;
constexpr uint32_t kMaxMoverSlots = 256;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

struct Regroup {
    uint8_t *code;        // [n] kStay or kMoved, with kFlown, per position of the streamed sequence
    uint32_t *mcount;     // [ncell] movers into each cell this step (reset by the collision wave)
    uint32_t *movers;     // [ncell][slots] 2 p + flown for their positions p, in no particular order
    uint32_t *far_head;   // [ncell] overflow list heads (reset by the collision wave)
    uint32_t *far_src, *far_next;
    uint32_t slots;       // mover slots per cell: 64, 128 or 256
    uint32_t n, ncell;    // particles and cells (the sizes of the lists above)
};

// (e: the list entry, 2 p + flown)
__device__ __forceinline__ void push_mover(const Regroup &rg, uint32_t e, uint32_t cell, uint32_t slot,
                                           DevState *st) {
    if (slot < rg.slots) {
        rg.movers[(size_t)bounds_ck(cell, rg.ncell, st) * rg.slots + slot] = e;
    } else {
        const uint32_t q = bounds_ck(atomicAdd(&st->far_count, 1u), rg.n, st);
        rg.far_src[q] = e;
        rg.far_next[q] = atomicExch(&rg.far_head[cell], q);
    }
}

// Streaming, in sequence order and in place, in two kernels.  The first
// takes every particle whose free end point x + c dt lies inside the closed
// box (the rule the flight itself applies first): it writes the code byte,
// counts the new cell and lists the movers (the gather moves the particle).  Particles
// that would leave the box go to a list that the second kernel flies
// exactly, wall conditions included, and finishes in the same way.  Keeping
// the rare wall path out of the first kernel keeps its register use, and so
// the number of loads in flight, at the level of a plain streaming kernel.
template <typename R, int D>
__device__ __forceinline__ void finish_move(const Geo &g, int64_t p, int fx, int fy, R x, R y, const Regroup &rg,
                                            uint32_t *count, DevState *st) {
    int tx, ty;
    cell_coords(g, (double)x, D == 2 ? (double)y : 0.0, tx, ty);
    const uint32_t cell = (uint32_t)ty * (uint32_t)g.nx + (uint32_t)tx;
    const bool stay = tx == fx && ty == fy;
    rg.code[p] = (stay ? kStay : kMoved) | kFlown;
    atomicAdd(&count[cell], 1u);
    if (!stay) push_mover(rg, 2u * (uint32_t)p + 1u, cell, atomicAdd(&rg.mcount[cell], 1u), st);
}

template <typename R>
__device__ __forceinline__ void load4(const R *p, R (&v)[4]) {
    if constexpr (sizeof(R) == 4) {
        const float4 t = *(const float4 *)p;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
        const double2 a = ((const double2 *)p)[0], b = ((const double2 *)p)[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}
template <typename R>
__device__ __forceinline__ void store4(R *p, const R (&v)[4]) {
    if constexpr (sizeof(R) == 4) {
        *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        ((double2 *)p)[0] = make_double2(v[0], v[1]);
        ((double2 *)p)[1] = make_double2(v[2], v[3]);
    }
}

// Workgroup of 256 threads, 4 consecutive particles per thread (vector loads
// and stores; one 32-bit store of the four code bytes).  New-cell counts and
// mover counts go to LDS bins covering the cells base .. base + 2047, base
// one row and one cell before the old cell of the workgroup's first
// particle: the sequence is grouped by cell, so the workgroup's particles
// come from a few consecutive cells and, apart from far and wrapped moves,
// land within one row of them.  Each bin is added to the global counters
// once per workgroup (the mover count returning the bin's first slot);
// cells outside the window are counted directly.
constexpr int kStreamBins = 2048;

template <typename R, int D>
__global__ __launch_bounds__(256) void k_stream_code(Geo g, Soa<R> s, int64_t n, Regroup rg, uint32_t *count,
                                                     uint32_t *wall_list, DevState *st) {
    __shared__ uint4 bins4[kStreamBins / 4];   // new-cell counts
    __shared__ uint4 mbins4[kStreamBins / 4];  // movers per new cell, then their first slot
    __shared__ uint32_t base_sh;
    uint32_t *bins = (uint32_t *)bins4, *mbins = (uint32_t *)mbins4;
    const uint32_t tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * 1024 + 4 * tid;  // first particle of this thread
    const int64_t left = n - p0;
    const int nv = left >= 4 ? 4 : (left > 0 ? (int)left : 0);
    const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
    bins4[tid] = zero4;
    bins4[tid + 256] = zero4;
    mbins4[tid] = zero4;
    mbins4[tid + 256] = zero4;
    const R tau = (R)g.dt, Lx = (R)g.Lx, Ly = (R)g.Ly, zero = (R)0;
    R x[4], y[4], cx[4], cy[4];
    if (nv == 4) {
        load4(s.x + p0, x);
        load4(s.cx + p0, cx);
        if (D == 2) {
            load4(s.y + p0, y);
            load4(s.cy + p0, cy);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool a = k < nv;
            x[k] = a ? s.x[p0 + k] : zero;
            cx[k] = a ? s.cx[p0 + k] : zero;
            if (D == 2) {
                y[k] = a ? s.y[p0 + k] : zero;
                cy[k] = a ? s.cy[p0 + k] : zero;
            }
        }
    }
    if (D < 2) {
#pragma unroll
        for (int k = 0; k < 4; ++k) { y[k] = zero; cy[k] = zero; }
    }
    uint32_t cell[4];
    bool in[4], stay[4];
    uint32_t codes = 0;
    int fx0 = 0, fy0 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const R xe = x[k] + cx[k] * tau;
        const R ye = D == 2 ? y[k] + cy[k] * tau : zero;
        in[k] = k < nv && xe >= zero && xe <= Lx && (D < 2 || (ye >= zero && ye <= Ly));
        int fx, fy;
        cell_coords(g, (double)x[k], D == 2 ? (double)y[k] : 0.0, fx, fy);
        if (k == 0) {
            fx0 = fx;
            fy0 = fy;
        }
        int tx, ty;
        cell_coords(g, (double)xe, D == 2 ? (double)ye : 0.0, tx, ty);
        cell[k] = (uint32_t)ty * (uint32_t)g.nx + (uint32_t)tx;
        stay[k] = tx == fx && ty == fy;
        // particles of the wall list get their code from the second kernel
        codes |= (uint32_t)(in[k] && stay[k] ? kStay : kMoved) << (8 * k);
    }
    // every position stays as stored (the gather advances it)
    if (nv == 4) {
        *(uint32_t *)(rg.code + p0) = codes;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nv) rg.code[p0 + k] = (uint8_t)(codes >> (8 * k));
    }
    if (tid == 0) base_sh = (uint32_t)fy0 * (uint32_t)g.nx + (uint32_t)fx0 - (D == 2 ? (uint32_t)g.nx : 0u) - 1u;
    __syncthreads();
    const uint32_t base = base_sh;  // modulo 2^32: cell - base is the bin
    uint32_t local[4];              // slot of each mover inside its bin
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        local[k] = 0;
        if (in[k]) {
            const uint32_t b = cell[k] - base;
            if (b < (uint32_t)kStreamBins) {
                atomicAdd(&bins[b], 1u);
                if (!stay[k]) local[k] = atomicAdd(&mbins[b], 1u);
            } else {
                atomicAdd(&count[cell[k]], 1u);
                if (!stay[k]) push_mover(rg, 2u * (uint32_t)(p0 + k), cell[k], atomicAdd(&rg.mcount[cell[k]], 1u), st);
            }
        }
        // particles that meet a wall: one list slot each, one atomic per wave
        const bool wall = k < nv && !in[k];
        const unsigned long long bal = __ballot(wall);
        if (bal) {
            const int lane = lane_id();
            const int leader = __ffsll((long long)bal) - 1;
            uint32_t b0 = 0;
            if (lane == leader) b0 = atomicAdd(&st->wall_count, (uint32_t)__popcll(bal));
            b0 = (uint32_t)__shfl((int)b0, leader, 64);
            if (wall)
                wall_list[bounds_ck(b0 + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull)), (uint32_t)n, st)] =
                    (uint32_t)(p0 + k);
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint4 c = bins4[tid + 256 * h];
        uint4 m = mbins4[tid + 256 * h];
        const uint32_t b = base + 4u * (tid + 256u * h);
        if (c.x) atomicAdd(&count[b], c.x);
        if (c.y) atomicAdd(&count[b + 1u], c.y);
        if (c.z) atomicAdd(&count[b + 2u], c.z);
        if (c.w) atomicAdd(&count[b + 3u], c.w);
        if (m.x) m.x = atomicAdd(&rg.mcount[b], m.x);
        if (m.y) m.y = atomicAdd(&rg.mcount[b + 1u], m.y);
        if (m.z) m.z = atomicAdd(&rg.mcount[b + 2u], m.z);
        if (m.w) m.w = atomicAdd(&rg.mcount[b + 3u], m.w);
        mbins4[tid + 256 * h] = m;  // first slot of each bin (a zero base is a base too)
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t b = cell[k] - base;
        if (in[k] && !stay[k] && b < (uint32_t)kStreamBins)
            push_mover(rg, 2u * (uint32_t)(p0 + k), cell[k], mbins[b] + local[k], st);
    }
}

// The particles of the wall list: exact flight with wall conditions from
// their unmodified state, then the same finish as in the first kernel.
// Grid-stride over the list length of this step.
template <typename R, int D, bool VR>
__global__ __launch_bounds__(256) void k_stream_walls(Geo g, Soa<R> s, Regroup rg, uint32_t *count,
                                                      const uint32_t *wall_list, DevState *st) {
    const uint32_t nw = st->wall_count;
    const uint32_t step = (uint32_t)st->step_next;
    uint32_t hsum = 0;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < nw; t += gridDim.x * 256) {
        const int64_t p = wall_list[t];
        R x = s.x[p], y = D == 2 ? s.y[p] : (R)0, cx = s.cx[p], cy = s.cy[p], cz = (R)0, w = (R)0;
        int fx, fy;
        cell_coords(g, (double)x, D == 2 ? (double)y : 0.0, fx, fy);
        uint32_t hits;
        bool diffuse;
        const int rc = fly<R, D, VR>(g, x, y, cx, cy, cz, w, s.id, s.w, p, step, hits, diffuse);
        if (rc) set_error(st, rc);
        s.x[p] = x;
        if (D == 2) s.y[p] = y;
        if (hits) {
            s.cx[p] = cx;
            s.cy[p] = cy;
            if (diffuse) {
                s.cz[p] = cz;
                if (VR) s.w[p] = w;
            }
        }
        finish_move<R, D>(g, p, fx, fy, x, y, rg, count, st);
        hsum += hits;
    }
    hsum = wave_sum_u32(hsum);
    if (lane_id() == 0 && hsum) diag_add(st, kDiagWallHits, (unsigned long long)hsum);
}

// Set-up of the initial sequence (grouped by the cell of the initial
// position, ascending particle id inside a cell): count the cells of the
// current positions, place every particle in its cell's range (arbitrary
// order), then rank each cell by id.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_count_cells(Geo g, Soa<R> s, int64_t n, uint32_t *count) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = p < n;
    uint32_t cell = 0;
    if (act) cell = cell_index(g, (double)s.x[p], D == 2 ? (double)s.y[p] : 0.0);
    wave_aggregated_add(count, cell, act);
}

template <typename R, int D, bool VR>
__global__ __launch_bounds__(256) void k_place(Geo g, Soa<R> src, Soa<R> dst, int64_t n, uint32_t *cursor,
                                               DevState *st) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = p < n;
    uint32_t cell = 0;
    if (act) cell = cell_index(g, (double)src.x[p], D == 2 ? (double)src.y[p] : 0.0);
    const uint32_t slot = wave_aggregated_inc(cursor, cell, act);
    if (act && (int64_t)slot >= n) {
        set_error(st, DSMC_ECAPACITY);
        return;
    }
    if (act) {
        dst.x[slot] = src.x[p];
        if (D == 2) dst.y[slot] = src.y[p];
        dst.cx[slot] = src.cx[p]; dst.cy[slot] = src.cy[p]; dst.cz[slot] = src.cz[p];
        if (VR) dst.w[slot] = src.w[p];
        dst.id[slot] = src.id[p];
    }
}

// Largest cell of the ranges start[0..ncell] (atomic maximum into
// st->max_cell, zero before the launch; set-up only).
__global__ __launch_bounds__(256) void k_max_cell(const uint32_t *start, int64_t ncell, DevState *st) {
    uint32_t m = 0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * 256) {
        const uint32_t n = start[c + 1] - start[c];
        m = n > m ? n : m;
    }
    m = ~wave_min_u32(~m);
    if (lane_id() == 0 && m) atomicMax(&st->max_cell, m);
}

template <typename R, int D, bool VR>
__global__ __launch_bounds__(64) void k_canonical(Soa<R> src, Soa<R> dst, const uint32_t *start) {
    const uint32_t cell = blockIdx.x;
    const uint32_t base = start[cell], N = start[cell + 1] - base;
    for (uint32_t q = lane_id(); q < N; q += 64) {
        const uint32_t me = src.id[base + q];
        uint32_t r = 0;
        for (uint32_t t = 0; t < N; ++t) r += src.id[base + t] < me ? 1u : 0u;
        if (r >= N) r = N - 1;  // ids are distinct; never write outside the cell
        const uint32_t o = base + r;
        dst.x[o] = src.x[base + q];
        if (D == 2) dst.y[o] = src.y[base + q];
        dst.cx[o] = src.cx[base + q]; dst.cy[o] = src.cy[base + q]; dst.cz[o] = src.cz[base + q];
        if (VR) dst.w[o] = src.w[base + q];
        dst.id[o] = me;
    }
}

// Exclusive scan of the per-cell counts as a single-pass decoupled
// look-back scan (Merrill & Garland 2016): each workgroup of 256 threads
// scans a tile of 1024 cells, publishes its tile total (flag AGG) and, once
// its prefix is known, its inclusive prefix (flag INC); a tile's prefix is
// found by walking back over earlier tiles' flags, 64 at a time (one per
// lane of the first wave).  Workgroups are dispatched in index order, so
// every tile it waits on is resident or finished; the walk still gives up
// (and reports an error) after a bounded number of polls.  A flag is one
// 64-bit word: status (2 bits), the launch's epoch (30 bits) and the value
// (32 bits); a flag of an earlier launch has another epoch and reads as not
// yet published, so flags are never cleared.  done[0] counts finished
// workgroups, done[1] holds the last launch's epoch; the last workgroup to
// finish resets the one, advances the other and, when `advance` is set
// (every step; not at set-up), advances the step bookkeeping.
constexpr int kScanTile = 1024;
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62, kFlagStatus = 3ull << 62;
constexpr uint32_t kEpochMask = (1u << 30) - 1u;

__global__ __launch_bounds__(256) void k_scan_lookback(uint32_t *count, uint32_t *offset, uint32_t *cursor,
                                                       int ncell, uint64_t *flags, uint32_t *done,
                                                       DevState *st, int advance) {
    __shared__ uint32_t wave_tot[4];
    __shared__ uint32_t tile_prefix;
    __shared__ bool last;
    const int t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    const int tile = blockIdx.x;
    const int c0 = tile * kScanTile + t * 4;
    uint4 q = make_uint4(0, 0, 0, 0);
    if (c0 + 3 < ncell) {
        q = *(const uint4 *)(count + c0);
    } else {
        if (c0 < ncell) q.x = count[c0];
        if (c0 + 1 < ncell) q.y = count[c0 + 1];
        if (c0 + 2 < ncell) q.z = count[c0 + 2];
    }
    const uint32_t local = (q.x + q.y) + (q.z + q.w);
    uint32_t inc = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(inc, off, 64);
        if (lane >= off) inc += v;
    }
    if (lane == 63) wave_tot[wv] = inc;
    __syncthreads();
    const uint32_t w0 = wave_tot[0], w1 = wave_tot[1], w2 = wave_tot[2], w3 = wave_tot[3];
    const uint32_t tile_total = (w0 + w1) + (w2 + w3);
    const uint32_t wave_excl = wv == 0 ? 0u : (wv == 1 ? w0 : (wv == 2 ? w0 + w1 : (w0 + w1) + w2));
    if (wv == 0) {
        // wave-wide look-back: lane l inspects tile j - l, 64 predecessors per
        // round; the window is summed up to the nearest inclusive prefix once
        // every tile before it has published its total.  A flag carries its
        // value in the same 64-bit word, so relaxed device-scope atomics
        // suffice (release/acquire would write back and invalidate L2 on
        // every store and poll)
        uint32_t prefix = 0;
        const uint64_t epoch = (uint64_t)((done[1] + 1u) & kEpochMask) << 32;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&flags[0], kFlagInc | epoch | (uint64_t)tile_total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&flags[tile], kFlagAgg | epoch | (uint64_t)tile_total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int j = tile - 1;
            uint32_t polls = 0;
            while (j >= 0) {
                const int idx = j - lane;
                // before tile 0: an inclusive prefix of zero ends the window;
                // a flag of another launch counts as unpublished
                uint64_t f = idx >= 0 ? __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                      : kFlagInc | epoch;
                if ((f & ((uint64_t)kEpochMask << 32)) != epoch) f = 0;
                const unsigned long long incm = __ballot((f & kFlagStatus) == kFlagInc);
                const int first = incm ? __ffsll((long long)incm) - 1 : 64;
                const unsigned long long need = first >= 63 ? ~0ull : ((1ull << (first + 1)) - 1ull);
                const unsigned long long waiting = __ballot((f & kFlagStatus) == 0) & need;
                if (waiting) {
                    if (++polls > (1u << 24)) {
                        if (lane == 0) set_error(st, DSMC_EHIP);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += wave_sum_u32(lane <= first ? (uint32_t)f : 0u);
                if (first < 64) break;
                j -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&flags[tile], kFlagInc | epoch | (uint64_t)(prefix + tile_total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) tile_prefix = prefix;
    }
    __syncthreads();
    uint32_t run = tile_prefix + wave_excl + inc - local;
    uint4 r;
    r.x = run; run += q.x;
    r.y = run; run += q.y;
    r.z = run; run += q.z;
    r.w = run; run += q.w;
    if (c0 + 3 < ncell) {
        *(uint4 *)(offset + c0) = r;
        *(uint4 *)(cursor + c0) = r;
        *(uint4 *)(count + c0) = make_uint4(0, 0, 0, 0);
    } else {
        const uint32_t rv[4] = {r.x, r.y, r.z, r.w};
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncell) { offset[c0 + k] = rv[k]; cursor[c0 + k] = rv[k]; count[c0 + k] = 0u; }
    }
    if (c0 <= ncell - 1 && ncell - 1 <= c0 + 3) offset[ncell] = run;
    // last workgroup out: next epoch, advance the step
    __syncthreads();
    if (t == 0) {
        const uint32_t d = atomicAdd(&done[0], 1u);
        last = d == gridDim.x - 1;
    }
    __syncthreads();
    if (last) {
        if (t == 0) {
            // every workgroup read done[1] before its arrival was counted
            done[0] = 0u;
            done[1] = (done[1] + 1u) & kEpochMask;
            if (advance) {
                st->step_cur = st->step_next;
                st->step_next = st->step_next + 1;
                st->n_samples = st->n_samples + 1;
                st->big_count = 0;
                st->far_count = 0;
                st->wall_count = 0;
            }
        }
    }
}

// Step bookkeeping for homogeneous instances (no sort pass), once for a
// batch of nsteps <= kStepSlots steps: step k of the batch has index
// step_cur + k and uses slot k.
__global__ void k_begin_step(DevState *st, int nsteps) {
    if (threadIdx.x == 0) {
        st->step_cur = st->step_next;
        st->step_next = st->step_next + (unsigned long long)nsteps;
        st->n_samples = st->n_samples + (unsigned long long)nsteps;
    }
    if (threadIdx.x < kStepSlots) st->big_slot[threadIdx.x] = 0;
    if (threadIdx.x < kStepSlots * kQueues) st->queue[threadIdx.x * kQueueStride] = 0;
}

}  // namespace dsmc
