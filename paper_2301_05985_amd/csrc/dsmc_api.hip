// dsmc_api.hip -- host side of the C ABI declared in include/dsmc.h.
//
// The context borrows the caller's particle buffers and workspace, carves
// the workspace into the counting-sort double buffer, per-cell arrays and
// FP64 running sums, and records the per-step kernel sequence into HIP
// graphs on a private capture stream; dsmc_step replays them on the
// caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dsmc.h"
#include "dsmc_collide_kernels.h"

using namespace dsmc;

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return DSMC_EHIP;        \
    } while (0)

namespace {

constexpr int kGraphSteps = 8;  // steps recorded per graph (even: the sort ping-pongs)
constexpr unsigned kWallGrid = 256;  // workgroups of the wall-flight kernel (grid-stride)
constexpr uint32_t kWideMin = 1024;  // default: homogeneous instances above this size run on a workgroup of waves
constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 64 * 1024;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t alt[7];  // x y cx cy cz w id of the second particle buffer
    size_t count, offset, offset2, cursor, sums, counters, volume, state, big_list, perm, owner, sched, flags, done,
        units, code, far_head, far_src, far_next, wall_list, mcount, movers;
    size_t mlp, lattice;
    size_t total;
};

int64_t n_cells_of(const dsmc_config &c) {
    if (c.dims == 2) return (int64_t)c.n_cells[0] * c.n_cells[1];
    return c.n_cells[0];
}

// Mover slots per cell: the mean cell population rounded up to a power of
// two, between 64 and 256 (the whole cell moving in one step still fits).
uint32_t mover_slots(const dsmc_config &c) {
    const int64_t nc = n_cells_of(c);
    const double mean = nc > 0 ? (double)c.n_particles / (double)nc : 0.0;
    uint32_t s = 64;
    while ((double)s < mean && s < kMaxMoverSlots) s *= 2;
    return s;
}

dsmc_status validate(const dsmc_config *c) {
    if (!c) return DSMC_EINVAL;
    if (c->abi_version != DSMC_ABI_VERSION) return DSMC_EABI;
    if (c->dims < 0 || c->dims > 2) return DSMC_EINVAL;
    if (c->real_bytes != 4 && c->real_bytes != 8) return DSMC_EINVAL;
    if (c->molecule != DSMC_HARD_SPHERE && c->molecule != DSMC_MAXWELL && c->molecule != DSMC_VHS &&
        c->molecule != DSMC_VSS)
        return DSMC_EINVAL;
    if ((c->molecule == DSMC_VHS || c->molecule == DSMC_VSS) && !(c->omega >= 0.5 && c->omega <= 1.0))
        return DSMC_EINVAL;
    if (c->molecule == DSMC_VSS && !(c->alpha >= 1.0 && c->alpha <= 2.0)) return DSMC_EINVAL;
    if (c->majorant < DSMC_MAJORANT_EXACT || c->majorant > DSMC_MAJORANT_DIAMETER) return DSMC_EINVAL;
    if (c->n_cells[0] < 1 || (c->dims == 2 && c->n_cells[1] < 1)) return DSMC_EINVAL;
    if (n_cells_of(*c) > (int64_t)1 << 30) return DSMC_EINVAL;
    if (c->n_particles < 0 || c->n_particles > (int64_t)0x7FFFFFFF) return DSMC_EINVAL;
    if (!(c->dt > 0) || !(c->sigma >= 0) || !(c->FN > 0)) return DSMC_EINVAL;
    if (c->vr && !(c->vr_T0 > 0)) return DSMC_EINVAL;
    if (c->vr_reconstruct < 0 || !(c->vr_kappa == 0.0 || c->vr_kappa >= 1.0) || !(c->vr_kappa <= 16.0))
        return DSMC_EINVAL;
    if (c->wide_min < 0 || (c->wide_min > 0 && c->wide_min < 64)) return DSMC_EINVAL;
    if (c->occupancy != 0 && c->occupancy != 5 && c->occupancy != 6) return DSMC_EINVAL;
    if (c->cells_per_wave < 0 || c->cells_per_wave > 2) return DSMC_EINVAL;
    if (c->cells_per_wave == 2) {
        // walled cells with the exact or brute-force majorant, at most 128
        // mover slots (a mean cell population of at most 128)
        if (c->dims == 0 || c->majorant == DSMC_MAJORANT_LEARNED || mover_slots(*c) > 128) return DSMC_EINVAL;
    }
    if (c->waves_per_cell != 0 && c->waves_per_cell != 1 && c->waves_per_cell != 4) return DSMC_EINVAL;
    if (c->waves_per_cell == 4 &&
        (c->dims == 0 || c->majorant == DSMC_MAJORANT_LEARNED || c->cells_per_wave == 2))
        return DSMC_EINVAL;
    if (c->dims >= 1) {
        if (!(c->length[0] > 0) || (c->dims == 2 && !(c->length[1] > 0))) return DSMC_EINVAL;
        for (int k = 0; k < (c->dims == 2 ? 4 : 2); ++k) {
            if (c->wall_kind[k] < 0 || c->wall_kind[k] > 2) return DSMC_EINVAL;
            if (c->wall_kind[k] == DSMC_WALL_DIFFUSE && !(c->wall_T[k] > 0)) return DSMC_EINVAL;
        }
        // periodic walls come in pairs
        if ((c->wall_kind[0] == DSMC_WALL_PERIODIC) != (c->wall_kind[1] == DSMC_WALL_PERIODIC)) return DSMC_EINVAL;
        if (c->dims == 2 && (c->wall_kind[2] == DSMC_WALL_PERIODIC) != (c->wall_kind[3] == DSMC_WALL_PERIODIC))
            return DSMC_EINVAL;
    } else {
        if (!c->inst_offset) return DSMC_EINVAL;
        if (c->inst_offset[0] != 0 || c->inst_offset[c->n_cells[0]] != c->n_particles) return DSMC_EINVAL;
        for (int b = 0; b < c->n_cells[0]; ++b)
            if (c->inst_offset[b + 1] < c->inst_offset[b]) return DSMC_EINVAL;
    }
    if (c->cell_volume)
        for (int64_t i = 0; i < n_cells_of(*c); ++i)
            if (!(c->cell_volume[i] > 0)) return DSMC_EINVAL;
    if (c->max_wall_hits < 0) return DSMC_EINVAL;
    if (c->schedule != DSMC_SCHEDULE_GRID && c->schedule != DSMC_SCHEDULE_PERSISTENT) return DSMC_EINVAL;
    if (c->persistent_waves < 0 || c->chunk_work < 0) return DSMC_EINVAL;
    return DSMC_OK;
}

Layout make_layout(const dsmc_config &c) {
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const size_t n = (size_t)c.n_particles, rb = (size_t)c.real_bytes, nc = (size_t)n_cells_of(c);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
    if (c.dims >= 1) {
        for (int f = 0; f < 6; ++f) L.alt[f] = take(n * rb);
        L.alt[6] = take(n * 4);
        L.count = take(nc * 4);
        L.cursor = take(nc * 4);
        L.flags = take(((nc + kScanTile - 1) / kScanTile) * 8);
        L.done = take(8);
        L.offset2 = take((nc + 1) * 4);
        L.code = take(n);
        L.far_head = take(nc * 4);
        L.far_src = take(n * 4);
        L.far_next = take(n * 4);
        L.wall_list = take(n * 4);
        L.mcount = take(nc * 4);
        L.movers = take(nc * mover_slots(c) * 4);
    }
    L.offset = take((nc + 1) * 4);
    L.sums = take(nc * kNsum * 8);
    L.counters = take(nc * 2 * 8);
    L.volume = take(nc * 8);
    L.state = take(sizeof(DevState));
    L.big_list = take(nc * 4);
    L.perm = take(n * 4);
    L.owner = take(n * 4);
    L.sched = take((nc + 16) * 4);  // the two-cells-per-wave order may pad up to 16 entries
    L.units = take(nc * 8);
    L.mlp = take(DSMC_MLP_NPARAM * 4);
    L.lattice = take(kLatticeSize * 8);
    L.total = off;
    return L;
}

struct Bufs {
    void *x, *y, *cx, *cy, *cz, *w;
    uint32_t *id;
};

}  // namespace

struct dsmc_ctx {
    dsmc_config cfg;
    std::vector<double> volume_host;
    hipStream_t stream = nullptr;    // caller's stream
    hipStream_t capture = nullptr;   // private stream used only to record graphs
    unsigned char *ws = nullptr;
    Layout L;
    Bufs buf[2];
    int cur = 0;                     // buffer that holds the current state
    int64_t n = 0, ncell = 0;
    int cap = 0;
    size_t lds = 0;
    bool pair = false;               // walled cells: two per wave (cells_per_wave 2)
    unsigned pair_grid = 0;          // its workgroups
    bool walled_wide = false;        // walled cells: a four-wave workgroup each (waves_per_cell 4)
    int big_grid = 0;
    bool any_big_possible = false;
    uint64_t *flags = nullptr;
    uint32_t *done = nullptr;
    uint2 *units = nullptr;
    uint32_t n_units = 0;
    int persistent_grid = 0;
    // homogeneous instances, grid launch: the largest ones (more than
    // kWideMin particles, a prefix of the longest-first order) run on
    // workgroups of kWideThreads threads, the rest on single waves
    uint32_t nwide = 0;
    int cap_small = 0;
    size_t lds_wide = 0, lds_small = 0;
    uint32_t *count = nullptr, *offset = nullptr, *cursor = nullptr, *big_list = nullptr,
             *perm = nullptr, *owner = nullptr, *sched = nullptr;
    // walled runs: cell ranges of each particle buffer (off[0] is `offset`),
    // code bytes, mover lists and overflow lists of the streaming pass
    uint32_t *off[2] = {nullptr, nullptr};
    uint8_t *code = nullptr;
    uint32_t *far_head = nullptr, *far_src = nullptr, *far_next = nullptr, *wall_list = nullptr;
    uint32_t *mcount = nullptr, *movers = nullptr;
    double *sums = nullptr, *volume = nullptr, *lattice = nullptr;
    unsigned long long *counters = nullptr;
    float *mlp = nullptr;
    bool mlp_loaded = false;
    double mlp_delta = 0.0;
    uint32_t mlp_min_n = 0;
    DevState *st = nullptr;
    Geo geo;
    double Vuni = 1.0;
    hipGraphExec_t g1[2] = {nullptr, nullptr}, gk[2] = {nullptr, nullptr};
    dsmc_status sticky = DSMC_OK;
};

namespace {

template <typename R>
Soa<R> soa_of(const Bufs &b) {
    Soa<R> s;
    s.x = (R *)b.x; s.y = (R *)b.y; s.cx = (R *)b.cx; s.cy = (R *)b.cy; s.cz = (R *)b.cz;
    s.w = (R *)b.w; s.id = b.id;
    return s;
}

Regroup regroup_of(const dsmc_ctx *c) {
    Regroup r;
    r.code = c->code;
    r.mcount = c->mcount;
    r.movers = c->movers;
    r.far_head = c->far_head;
    r.far_src = c->far_src;
    r.far_next = c->far_next;
    r.slots = mover_slots(c->cfg);
    r.n = (uint32_t)c->n;
    r.ncell = (uint32_t)c->ncell;
    return r;
}

// Collision arguments for a step reading buffer src and writing dst (the
// same buffer for homogeneous instances, the other one for walled runs).
template <typename R>
CollideArgs<R> collide_args(dsmc_ctx *c, int src, int dst) {
    CollideArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.s = soa_of<R>(c->buf[dst]);
    a.sched = c->sched;
    if (c->cfg.dims == 0) {
        a.start = c->offset;
    } else {
        a.start = c->off[dst];
        a.src = soa_of<R>(c->buf[src]);
        a.src_start = c->off[src];
        a.rg = regroup_of(c);
    }
    a.volume = c->cfg.cell_volume ? c->volume : nullptr;
    a.Vuni = c->Vuni;
    a.dt = c->cfg.dt;
    a.sigma = c->cfg.sigma;
    a.FN = c->cfg.FN;
    a.molecule = c->cfg.molecule;
    a.omega1 = 1.0 - c->cfg.omega;
    a.inv_alpha = c->cfg.molecule == DSMC_VSS ? 1.0 / c->cfg.alpha : 1.0;
    a.cap = c->cap;
    a.majorant = c->cfg.majorant;
    a.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFull);
    a.k1 = (uint32_t)(c->cfg.seed >> 32);
    a.sums = c->sums;
    a.counters = c->counters;
    a.st = c->st;
    a.big_list = c->big_list;
    a.bigc = c->cfg.dims == 0 ? &c->st->big_slot[0] : &c->st->big_count;
    a.queue = &c->st->queue[0];
    a.step_off = 0;
    a.perm_g = c->perm;
    a.owner_g = c->owner;
    a.mlp = (c->cfg.majorant == DSMC_MAJORANT_LEARNED && c->mlp_loaded) ? c->mlp : nullptr;
    a.lattice = c->lattice;
    a.delta = c->mlp_delta;
    a.mlp_min_n = c->mlp_min_n;
    a.vr_reest = c->cfg.vr ? c->cfg.vr_reconstruct : 0;
    a.vr_scale = c->cfg.vr ? 1.0 / std::sqrt(c->cfg.vr_T0) : 1.0;
    a.vr_kappa = c->cfg.vr ? c->cfg.vr_kappa : 1.0;
    a.n_total = (uint32_t)c->n;
    a.n_cells = (uint32_t)c->ncell;
    return a;
}

// Kernel launch helper recording an optional event before each launch.
struct Launcher {
    hipStream_t s;
    std::vector<hipEvent_t> *ev;
    std::vector<const char *> *names;
    void mark(const char *name) {
        if (ev) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            (void)hipEventRecord(e, s);
            ev->push_back(e);
            names->push_back(name);
        }
    }
};

// One-wave collision kernel with its occupancy variant.  Walled FP32 cells
// run at six waves per SIMD (the kernel fits 80 registers, and the LDS
// capacity below leaves room for six cells per SIMD); FP64 walled cells,
// whose LDS holds fewer waves anyway, keep five.  Homogeneous instances on
// the grid schedule take the configured variant (five by default; six fits
// the weighted kernel into 80 registers at the price of a few spills).
template <typename R, bool VR, int D>
void launch_collide_wave(dsmc_ctx *c, dim3 grid, size_t lds, hipStream_t s, const CollideArgs<R> &a) {
    if constexpr (D == 0) {
        if (c->cfg.occupancy == 6) {
            hipLaunchKernelGGL((k_collide<R, VR, D, 6>), grid, dim3(64), lds, s, a);
            return;
        }
        hipLaunchKernelGGL((k_collide<R, VR, D, 5>), grid, dim3(64), lds, s, a);
    } else {
        hipLaunchKernelGGL((k_collide<R, VR, D, (sizeof(R) == 4 ? 6 : 5)>), grid, dim3(64), lds, s, a);
    }
}

template <typename R, bool VR, int D>
void launch_collide(dsmc_ctx *c, Launcher &L, int src, int slot) {
    CollideArgs<R> a = collide_args<R>(c, src, D == 0 ? src : src ^ 1);
    if (D == 0) {
        // step `slot` of a batch recorded behind one bookkeeping launch
        a.step_off = (uint32_t)slot;
        a.bigc = &c->st->big_slot[slot];
        a.queue = &c->st->queue[slot * kQueues * kQueueStride];
    }
    const bool learned = a.mlp != nullptr && c->cfg.molecule != DSMC_MAXWELL;
    L.mark(learned ? "collide_learned" : "collide");
    if (D == 0 && c->cfg.schedule == DSMC_SCHEDULE_PERSISTENT) {
        if (learned)
            hipLaunchKernelGGL((k_collide_persistent<R, VR, true>), dim3((unsigned)c->persistent_grid), dim3(64),
                               c->lds, L.s, a, (const uint2 *)c->units, c->n_units);
        else
            hipLaunchKernelGGL((k_collide_persistent<R, VR, false>), dim3((unsigned)c->persistent_grid), dim3(64),
                               c->lds, L.s, a, (const uint2 *)c->units, c->n_units);
    } else if (D == 0 && c->nwide > 0) {
        if (learned)
            hipLaunchKernelGGL((k_collide_wide_learned<R, VR>), dim3(c->nwide), dim3(kWideThreads), c->lds_wide, L.s,
                               a);
        else
            hipLaunchKernelGGL((k_collide_wide<R, VR>), dim3(c->nwide), dim3(kWideThreads), c->lds_wide, L.s, a);
        if ((int64_t)c->nwide < c->ncell) {
            CollideArgs<R> as = a;
            as.sched = c->sched + c->nwide;
            as.cap = c->cap_small;
            if (learned)
                hipLaunchKernelGGL((k_collide_learned<R, VR, D>), dim3((unsigned)(c->ncell - c->nwide)), dim3(64),
                                   c->lds_small, L.s, as);
            else
                launch_collide_wave<R, VR, D>(c, dim3((unsigned)(c->ncell - c->nwide)), c->lds_small, L.s, as);
        }
    } else if (learned)
        hipLaunchKernelGGL((k_collide_learned<R, VR, D>), dim3((unsigned)c->ncell), dim3(64), c->lds,
                           L.s, a);
    else if (D > 0 && c->pair)
        hipLaunchKernelGGL((k_collide_pair<R, VR, D>), dim3(c->pair_grid), dim3(64), c->lds, L.s, a);
    else if (D > 0 && c->walled_wide)
        hipLaunchKernelGGL((k_collide_walled_wide<R, VR, D>), dim3((unsigned)c->ncell), dim3(kWideThreads), c->lds,
                           L.s, a);
    else
        launch_collide_wave<R, VR, D>(c, dim3((unsigned)c->ncell), c->lds, L.s, a);
    if (c->any_big_possible) {
        L.mark("collide_big");
        if (D == 0) {
            // homogeneous instances: a four-wave workgroup per instance
            if (learned)
                hipLaunchKernelGGL((k_collide_big_wide_learned<R, VR>), dim3(c->big_grid), dim3(kWideThreads), 0,
                                   L.s, a);
            else
                hipLaunchKernelGGL((k_collide_big_wide<R, VR>), dim3(c->big_grid), dim3(kWideThreads), 0, L.s, a);
        } else if (learned)
            hipLaunchKernelGGL((k_collide_big_learned<R, VR, D>), dim3(c->big_grid), dim3(64), 0, L.s, a);
        else
            hipLaunchKernelGGL((k_collide_big<R, VR, D>), dim3(c->big_grid), dim3(64), 0, L.s, a);
    }
}

// Streaming pass over buffer src and the scan of the new cells' counts into
// the cell ranges of the other buffer.
template <typename R, int D, bool VR>
void launch_stream(dsmc_ctx *c, Launcher &L, int src) {
    const int dst = src ^ 1;
    const unsigned grid = (unsigned)((c->n + 1023) / 1024);  // 4 particles per thread
    if (c->n > 0) {
        const Soa<R> s = soa_of<R>(c->buf[src]);
        L.mark("stream");
        hipLaunchKernelGGL((k_stream_code<R, D>), dim3(grid), dim3(256), 0, L.s, c->geo, s, (int64_t)c->n,
                           regroup_of(c), c->count, c->wall_list, c->st);
        L.mark("stream_walls");
        hipLaunchKernelGGL((k_stream_walls<R, D, VR>), dim3(kWallGrid), dim3(256), 0, L.s, c->geo, s, regroup_of(c),
                           c->count, (const uint32_t *)c->wall_list, c->st);
    }
    L.mark("scan");
    hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)((c->ncell + kScanTile - 1) / kScanTile)), dim3(256), 0, L.s,
                       c->count, c->off[dst], c->cursor, (int)c->ncell, c->flags, c->done, c->st, 1);
}

// Cell ranges of buffer b from the cells of its current positions (set-up and
// restore; the step bookkeeping is not advanced).
template <typename R, int D>
void launch_ranges(dsmc_ctx *c, hipStream_t s, int b) {
    const unsigned grid = (unsigned)((c->n + 255) / 256);
    if (c->n > 0)
        hipLaunchKernelGGL((k_count_cells<R, D>), dim3(grid), dim3(256), 0, s, c->geo, soa_of<R>(c->buf[b]),
                           (int64_t)c->n, c->count);
    hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)((c->ncell + kScanTile - 1) / kScanTile)), dim3(256), 0, s,
                       c->count, c->off[b], c->cursor, (int)c->ncell, c->flags, c->done, c->st, 0);
}

// Largest cell of the initial positions: the set-up orders each cell by id
// with one wave and a quadratic rank count, so a cell above this size (for
// instance every particle at a NaN position, all in cell 0) makes dsmc_init
// fail with DSMC_ECAPACITY instead of running for minutes.
constexpr uint32_t kMaxSetupCell = 1u << 17;

// Initial sequence in buffer 0: grouped by cell, ascending id inside a cell.
template <typename R, int D, bool VR>
dsmc_status launch_initial_sequence(dsmc_ctx *c, hipStream_t s) {
    launch_ranges<R, D>(c, s, 0);
    if (c->n == 0) return DSMC_OK;
    // the largest cell, reduced on the device (the state was zeroed at init)
    const unsigned mgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((c->ncell + 255) / 256, 1024));
    hipLaunchKernelGGL(k_max_cell, dim3(mgrid), dim3(256), 0, s, (const uint32_t *)c->off[0], (int64_t)c->ncell,
                       c->st);
    uint32_t max_cell = 0;
    if (hipMemcpyAsync(&max_cell, &c->st->max_cell, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DSMC_EHIP;
    if (max_cell > kMaxSetupCell) return DSMC_ECAPACITY;
    const unsigned grid = (unsigned)((c->n + 255) / 256);
    hipLaunchKernelGGL((k_place<R, D, VR>), dim3(grid), dim3(256), 0, s, c->geo, soa_of<R>(c->buf[0]),
                       soa_of<R>(c->buf[1]), (int64_t)c->n, c->cursor, c->st);
    hipLaunchKernelGGL((k_canonical<R, D, VR>), dim3((unsigned)c->ncell), dim3(64), 0, s, soa_of<R>(c->buf[1]),
                       soa_of<R>(c->buf[0]), (const uint32_t *)c->off[0]);
    return DSMC_OK;
}

template <typename R, int D>
dsmc_status dispatch_vr(dsmc_ctx *c, hipStream_t s, bool initial) {
    if (initial) return c->cfg.vr ? launch_initial_sequence<R, D, true>(c, s) : launch_initial_sequence<R, D, false>(c, s);
    launch_ranges<R, D>(c, s, c->cur);
    return DSMC_OK;
}

// Set-up (initial) or restore (ranges of the current buffer) of a walled run.
dsmc_status walled_setup(dsmc_ctx *c, bool initial) {
    hipStream_t s = c->stream;
    if (c->cfg.real_bytes == 4) {
        if (c->cfg.dims == 1) return dispatch_vr<float, 1>(c, s, initial);
        return dispatch_vr<float, 2>(c, s, initial);
    }
    if (c->cfg.dims == 1) return dispatch_vr<double, 1>(c, s, initial);
    return dispatch_vr<double, 2>(c, s, initial);
}

// Step k of a batch of nsteps consecutive steps.  Homogeneous runs put one
// bookkeeping launch in front of every kStepSlots steps; walled runs keep
// their bookkeeping in the scan.
template <typename R, bool VR>
void enqueue_step_t(dsmc_ctx *c, Launcher &L, int src, int k, int nsteps) {
    if (c->cfg.dims == 0) {
        if (k % kStepSlots == 0) {
            L.mark("begin_step");
            hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(64), 0, L.s, c->st, std::min(kStepSlots, nsteps - k));
        }
        launch_collide<R, VR, 0>(c, L, src, k % kStepSlots);
        return;
    }
    if (c->cfg.dims == 1) {
        launch_stream<R, 1, VR>(c, L, src);
        launch_collide<R, VR, 1>(c, L, src, 0);
    } else {
        launch_stream<R, 2, VR>(c, L, src);
        launch_collide<R, VR, 2>(c, L, src, 0);
    }
}

// Enqueue step k of a batch of nsteps reading buffer `src`; returns the
// buffer holding the result.
int enqueue_step(dsmc_ctx *c, Launcher &L, int src, int k = 0, int nsteps = 1) {
    const bool vr = c->cfg.vr != 0;
    if (c->cfg.real_bytes == 4) {
        if (vr) enqueue_step_t<float, true>(c, L, src, k, nsteps);
        else enqueue_step_t<float, false>(c, L, src, k, nsteps);
    } else {
        if (vr) enqueue_step_t<double, true>(c, L, src, k, nsteps);
        else enqueue_step_t<double, false>(c, L, src, k, nsteps);
    }
    return c->cfg.dims == 0 ? src : src ^ 1;
}

dsmc_status record_graph(dsmc_ctx *c, int src, int steps, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
    Launcher L{c->capture, nullptr, nullptr};
    int b = src;
    for (int k = 0; k < steps; ++k) b = enqueue_step(c, L, b, k, steps);
    hipError_t e = hipStreamEndCapture(c->capture, &g);
    if (e != hipSuccess) return DSMC_EHIP;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

dsmc_status device_status(dsmc_ctx *c) {
    if (c->sticky != DSMC_OK) return c->sticky;
    unsigned int err = 0;
    if (hipMemcpy(&err, &c->st->error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) {
        c->sticky = DSMC_EHIP;
        return c->sticky;
    }
    if (err) c->sticky = (dsmc_status)(-(int)err);
    return c->sticky;
}

struct BlobHeader {
    uint64_t magic, n, real_bytes, dims, ncell, step_next, n_samples, vr;
};
constexpr uint64_t kBlobMagic = 0x44534d4330314b50ull;

}  // namespace

extern "C" {

const char *dsmc_status_string(dsmc_status s) {
    switch (s) {
        case DSMC_OK: return "ok";
        case DSMC_EINVAL: return "invalid argument or configuration";
        case DSMC_ENOMEM: return "workspace too small";
        case DSMC_EHIP: return "HIP runtime error";
        case DSMC_ENONFINITE: return "non-finite velocity";
        case DSMC_EWALLHITS: return "too many wall hits in one step";
        case DSMC_ECAPACITY: return "per-cell capacity exceeded";
        case DSMC_EABI: return "ABI version mismatch";
    }
    return "unknown status";
}

dsmc_status dsmc_workspace_size(const dsmc_config *cfg, size_t *bytes) {
    dsmc_status s = validate(cfg);
    if (s != DSMC_OK) return s;
    if (!bytes) return DSMC_EINVAL;
    *bytes = make_layout(*cfg).total;
    return DSMC_OK;
}

dsmc_status dsmc_init(const dsmc_config *cfg, const dsmc_soa *p, void *workspace, size_t ws_bytes,
                      void *hip_stream, dsmc_ctx **out) {
    if (!out) return DSMC_EINVAL;
    *out = nullptr;
    dsmc_status s = validate(cfg);
    if (s != DSMC_OK) return s;
    if (!p || !workspace || ((uintptr_t)workspace % kAlign) != 0) return DSMC_EINVAL;
    if (cfg->n_particles > 0 && (!p->cx || !p->cy || !p->cz || !p->id)) return DSMC_EINVAL;
    if (cfg->n_particles > 0 && cfg->dims >= 1 && !p->x) return DSMC_EINVAL;
    if (cfg->n_particles > 0 && cfg->dims == 2 && !p->y) return DSMC_EINVAL;
    if (cfg->n_particles > 0 && cfg->vr && !p->w) return DSMC_EINVAL;
    // the streaming kernel moves four particles per vector access
    for (const void *q : {(const void *)p->x, (const void *)p->y, (const void *)p->cx, (const void *)p->cy,
                          (const void *)p->cz, (const void *)p->w, (const void *)p->id})
        if (((uintptr_t)q % 16) != 0) return DSMC_EINVAL;
    const Layout L = make_layout(*cfg);
    if (ws_bytes < L.total) return DSMC_ENOMEM;

    dsmc_ctx *c = new (std::nothrow) dsmc_ctx();
    if (!c) return DSMC_EINVAL;
    c->cfg = *cfg;
    if (c->cfg.max_wall_hits == 0) c->cfg.max_wall_hits = 64;
    c->cfg.cell_volume = nullptr;
    c->cfg.inst_offset = nullptr;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (unsigned char *)workspace;
    c->L = L;
    c->n = cfg->n_particles;
    c->ncell = n_cells_of(*cfg);
    const size_t rb = (size_t)cfg->real_bytes;
    c->buf[0] = Bufs{p->x, p->y, p->cx, p->cy, p->cz, p->w, p->id};
    if (cfg->dims >= 1) {
        c->buf[1] = Bufs{c->ws + L.alt[0], c->ws + L.alt[1], c->ws + L.alt[2], c->ws + L.alt[3],
                         c->ws + L.alt[4], c->ws + L.alt[5], (uint32_t *)(c->ws + L.alt[6])};
        c->count = (uint32_t *)(c->ws + L.count);
        c->cursor = (uint32_t *)(c->ws + L.cursor);
        c->flags = (uint64_t *)(c->ws + L.flags);
        c->done = (uint32_t *)(c->ws + L.done);
        c->code = (uint8_t *)(c->ws + L.code);
        c->far_head = (uint32_t *)(c->ws + L.far_head);
        c->far_src = (uint32_t *)(c->ws + L.far_src);
        c->far_next = (uint32_t *)(c->ws + L.far_next);
        c->wall_list = (uint32_t *)(c->ws + L.wall_list);
        c->mcount = (uint32_t *)(c->ws + L.mcount);
        c->movers = (uint32_t *)(c->ws + L.movers);
        c->off[1] = (uint32_t *)(c->ws + L.offset2);
    } else {
        c->buf[1] = c->buf[0];
    }
    c->offset = (uint32_t *)(c->ws + L.offset);
    c->off[0] = c->offset;
    c->sums = (double *)(c->ws + L.sums);
    c->counters = (unsigned long long *)(c->ws + L.counters);
    c->volume = (double *)(c->ws + L.volume);
    c->st = (DevState *)(c->ws + L.state);
    c->big_list = (uint32_t *)(c->ws + L.big_list);
    c->perm = (uint32_t *)(c->ws + L.perm);
    c->owner = (uint32_t *)(c->ws + L.owner);
    c->sched = (uint32_t *)(c->ws + L.sched);
    c->units = (uint2 *)(c->ws + L.units);
    c->mlp = (float *)(c->ws + L.mlp);
    c->lattice = (double *)(c->ws + L.lattice);

    // geometry
    Geo &g = c->geo;
    std::memset(&g, 0, sizeof(g));
    g.dims = cfg->dims;
    g.nx = cfg->n_cells[0];
    g.ny = cfg->dims == 2 ? cfg->n_cells[1] : 1;
    g.max_hits = c->cfg.max_wall_hits;
    g.Lx = cfg->length[0];
    g.Ly = cfg->length[1];
    g.dt = cfg->dt;
    g.invx = cfg->dims >= 1 ? (double)cfg->n_cells[0] / cfg->length[0] : 0.0;
    g.invy = cfg->dims == 2 ? (double)cfg->n_cells[1] / cfg->length[1] : 0.0;
    for (int k = 0; k < 4; ++k) {
        g.kind[k] = cfg->wall_kind[k];
        g.Tw[k] = cfg->wall_T[k];
        g.ux[k] = cfg->wall_u[k][0];
        g.uy[k] = cfg->wall_u[k][1];
        g.uz[k] = cfg->wall_u[k][2];
    }
    g.T0 = cfg->vr ? cfg->vr_T0 : 1.0;
    g.k0 = (uint32_t)(cfg->seed & 0xFFFFFFFFull);
    g.k1 = (uint32_t)(cfg->seed >> 32);
    if (cfg->dims == 2) c->Vuni = (cfg->length[0] / cfg->n_cells[0]) * (cfg->length[1] / cfg->n_cells[1]);
    else if (cfg->dims == 1) c->Vuni = cfg->length[0] / cfg->n_cells[0];
    else c->Vuni = 1.0;

    // LDS capacity per cell (one wave per cell)
    // LDS per cell: velocity and weight of each particle side by side (16 B,
    // 32 B in double), owner marks (+4 padding entries; in walled runs they
    // first hold the gather's selection).  Homogeneous runs without weights
    // keep the owner marks in the weight slots.
    const bool packed = cfg->dims == 0 && !cfg->vr;
    const size_t per = packed ? 4 * rb : 4 * rb + 4;
    const int cap_fit = (int)std::min<size_t>((kMaxLds - 64) / per, 65535) / 32 * 32;
    std::vector<uint32_t> start_host;
    std::vector<uint32_t> sched_host;
    std::vector<uint2> units_host;
    if (cfg->dims == 0) {
        int64_t maxn = 0;
        start_host.resize(c->ncell + 1);
        for (int64_t b = 0; b <= c->ncell; ++b) start_host[b] = (uint32_t)cfg->inst_offset[b];
        for (int64_t b = 0; b < c->ncell; ++b) maxn = std::max<int64_t>(maxn, cfg->inst_offset[b + 1] - cfg->inst_offset[b]);
        c->cap = (int)std::min<int64_t>(std::max<int64_t>((maxn + 31) / 32 * 32, 32), cap_fit);
        int nbig = 0;
        for (int64_t b = 0; b < c->ncell; ++b)
            if (cfg->inst_offset[b + 1] - cfg->inst_offset[b] > c->cap) ++nbig;
        c->any_big_possible = nbig > 0;
        c->big_grid = std::max(1, std::min(nbig, 256));
        // longest-processing-time order: instances by decreasing N^2 work
        sched_host.resize(c->ncell);
        std::iota(sched_host.begin(), sched_host.end(), 0u);
        std::stable_sort(sched_host.begin(), sched_host.end(), [&](uint32_t a, uint32_t b) {
            return (cfg->inst_offset[a + 1] - cfg->inst_offset[a]) > (cfg->inst_offset[b + 1] - cfg->inst_offset[b]);
        });
        // work units of the persistent kernel: runs of at most 64 consecutive
        // schedule entries holding fewer than chunk_work particles before the
        // last one is added (chunk_work 0: one instance per unit)
        for (uint32_t k = 0; k < (uint32_t)c->ncell;) {
            uint32_t cnt = 0;
            int64_t work = 0;
            do {
                work += cfg->inst_offset[sched_host[k + cnt] + 1] - cfg->inst_offset[sched_host[k + cnt]];
                ++cnt;
            } while (k + cnt < (uint32_t)c->ncell && work < cfg->chunk_work && cnt < 64);
            units_host.push_back(make_uint2(k, cnt));
            k += cnt;
        }
        c->n_units = (uint32_t)units_host.size();
        // wide instances: the prefix of the longest-first order above the
        // configured threshold
        const int64_t wide_min = cfg->wide_min > 0 ? cfg->wide_min : (int64_t)kWideMin;
        if (cfg->schedule == DSMC_SCHEDULE_GRID) {
            uint32_t nw = 0;
            while (nw < (uint32_t)c->ncell &&
                   cfg->inst_offset[sched_host[nw] + 1] - cfg->inst_offset[sched_host[nw]] > (int64_t)wide_min)
                ++nw;
            const size_t lw = std::max<size_t>((size_t)c->cap * per + 16 + 16 + sizeof(GroupScratch),
                                               kRedBytes);
            if (nw > 0 && lw <= kMaxLds) {
                c->nwide = nw;
                c->lds_wide = lw;
                const int64_t nsmall = nw < (uint32_t)c->ncell
                    ? cfg->inst_offset[sched_host[nw] + 1] - cfg->inst_offset[sched_host[nw]] : 0;
                c->cap_small = (int)std::min<int64_t>(std::max<int64_t>((nsmall + 31) / 32 * 32, 32), cap_fit);
                c->lds_small = std::max<size_t>((size_t)c->cap_small * per + 16 + 16, kRedBytes);
            }
        }
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
        }
        c->persistent_grid = cfg->persistent_waves > 0 ? cfg->persistent_waves : 8 * ncu;
    } else {
        // LDS capacity of a walled cell, chosen so that LDS holds six
        // one-wave cells per SIMD where the registers allow six (FP32):
        // 2 x mean + 64 without weights (16 bytes and an owner mark per
        // particle), 2.5 x mean + 64 with them (20 bytes); on the 100-per-cell
        // cavity the collision kernel runs 8% faster than at five.  FP64
        // cells keep 3 x mean + 64.  A cell above capacity runs in the
        // global-memory kernel with the same results.
        const double mean = (double)c->n / (double)c->ncell;
        const double mult = cfg->real_bytes == 8 ? 3.0 : (cfg->vr ? 2.5 : 2.0);
        int want = (int)std::ceil(mult * mean + 64.0);
        want = (want + 31) / 32 * 32;
        c->cap = std::max(64, std::min(want, cap_fit));
        if (cfg->waves_per_cell == 4) {
            // the four-wave workgroup also keeps its GroupScratch in LDS
            const int cap_fit_wide =
                (int)std::min<size_t>((kMaxLds - 64 - sizeof(GroupScratch)) / per, 65535) / 32 * 32;
            c->cap = std::max(64, std::min(c->cap, cap_fit_wide));
        }
        c->pair = cfg->cells_per_wave == 2;
        if (c->pair) {
            // two cells per wave: 0.96 x mean + 64 per cell (160 on the
            // 100-per-cell cavity, where a cell's area is then the moment
            // transpose's 3,328 bytes: 204 us per step against 214 at 192);
            // at least 128, so that a cell's owner marks (cap + 4 words) can
            // hold the 64 FP64 sums of the weight re-estimation.  Cells above
            // it run in the global-memory kernel (counted in big_cells), so a
            // flow far from uniform density is better served by one cell per
            // wave and its larger capacity
            const int cap_fit_pair = (int)std::min<size_t>((kMaxLds / 2 - 64) / per, 65535) / 32 * 32;
            int wp = (int)std::ceil(0.96 * mean + 64.0);
            wp = (wp + 31) / 32 * 32;
            c->cap = std::max(128, std::min(wp, cap_fit_pair));
        }
        const int64_t maxbig = c->n / (c->cap + 1);
        c->any_big_possible = maxbig > 0;
        c->big_grid = (int)std::max<int64_t>(1, std::min<int64_t>(maxbig, 256));
        // XCD-aware order: workgroups are dealt to the eight XCDs in turn
        // (block b on XCD b mod 8), so XCD x is given the x-th contiguous
        // eighth of the cells and the neighbour cells a cell gathers from
        // are mostly read through the same L2
        if (c->pair) {
            // workgroup w = 8 k + x takes cells x per8 + 2 k and x per8 + 2 k + 1
            // (per8 even; entries past the last cell hold kNoCell)
            const int64_t per8 = ((c->ncell + 7) / 8 + 1) / 2 * 2;
            const int64_t waves = 8 * (per8 / 2);
            sched_host.assign((size_t)(2 * waves), kNoCell);
            for (int64_t w = 0; w < waves; ++w)
                for (int64_t h = 0; h < 2; ++h) {
                    const int64_t cell = (w % 8) * per8 + 2 * (w / 8) + h;
                    if (cell < c->ncell) sched_host[(size_t)(2 * w + h)] = (uint32_t)cell;
                }
            c->pair_grid = (unsigned)waves;
        } else {
            sched_host.resize(c->ncell);
            const int64_t per8 = (c->ncell + 7) / 8;
            int64_t blk = 0;
            for (int64_t k = 0; k < per8; ++k)
                for (int64_t x = 0; x < 8; ++x) {
                    const int64_t cell = x * per8 + k;
                    if (cell < c->ncell) sched_host[blk++] = (uint32_t)cell;
                }
        }
    }
    // (at least the transpose area of the moment reduction: 13 x 64 doubles;
    // two cells per wave: two areas of pair_area_bytes)
    c->lds = std::max<size_t>((size_t)c->cap * per + 16 + 16, kRedBytes);
    if (c->pair) c->lds = 2 * (cfg->real_bytes == 8 ? pair_area_bytes<double>(c->cap) : pair_area_bytes<float>(c->cap));
    // four waves per walled cell: the workgroup's wave results meet in a
    // GroupScratch after the owner marks (the moments are reduced through it,
    // not through the cell's area)
    c->walled_wide = cfg->dims >= 1 && cfg->waves_per_cell == 4;
    if (c->walled_wide) c->lds = (size_t)c->cap * per + 16 + 16 + sizeof(GroupScratch);

    // graphs are recorded on a private stream (capture is not allowed on
    // the legacy default stream the caller may use)
    if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return DSMC_EHIP;
    }
    auto fail = [&](dsmc_status e) { dsmc_destroy(c); return e; };
    // initial device state, on the caller's stream
    if (hipMemsetAsync(c->ws + L.sums, 0, L.counters + (size_t)c->ncell * 16 - L.sums, c->stream) != hipSuccess)
        return fail(DSMC_EHIP);
    if (hipMemsetAsync(c->st, 0, sizeof(DevState), c->stream) != hipSuccess) return fail(DSMC_EHIP);
    if (cfg->dims >= 1 && hipMemsetAsync(c->count, 0, (size_t)c->ncell * 4, c->stream) != hipSuccess)
        return fail(DSMC_EHIP);
    if (cfg->dims >= 1 && hipMemsetAsync(c->ws + L.flags, 0, L.done + 8 - L.flags, c->stream) != hipSuccess)
        return fail(DSMC_EHIP);
    if (cfg->cell_volume) {
        c->volume_host.assign(cfg->cell_volume, cfg->cell_volume + c->ncell);
        c->cfg.cell_volume = c->volume_host.data();
        if (hipMemcpyAsync(c->volume, c->volume_host.data(), (size_t)c->ncell * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(DSMC_EHIP);
    }
    if (hipMemcpyAsync(c->sched, sched_host.data(), sched_host.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fail(DSMC_EHIP);
    if (cfg->dims == 0) {
        if (hipMemcpyAsync(c->offset, start_host.data(), start_host.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->units, units_host.data(), units_host.size() * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(DSMC_EHIP);
    } else {
        // empty mover and overflow lists, then the initial particle sequence
        if (hipMemsetAsync(c->far_head, 0xFF, (size_t)c->ncell * 4, c->stream) != hipSuccess ||
            hipMemsetAsync(c->mcount, 0, (size_t)c->ncell * 4, c->stream) != hipSuccess)
            return fail(DSMC_EHIP);
        const dsmc_status rs = walled_setup(c, true);
        if (rs != DSMC_OK) return fail(rs);
        if (hipGetLastError() != hipSuccess) return fail(DSMC_EHIP);
    }
    {
        std::vector<double> lat(kLatticeSize);
        for (int k = 0; k < kLatticeSize; ++k) lat[k] = std::exp2((double)(k - kLatticeHalf) / 64.0);
        if (hipMemcpyAsync(c->lattice, lat.data(), lat.size() * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(DSMC_EHIP);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(DSMC_EHIP);
    }
    if (c->lds > 64 * 1024) return fail(DSMC_EINVAL);
    dsmc_status r = DSMC_OK;
    for (int b = 0; b < (cfg->dims >= 1 ? 2 : 1) && r == DSMC_OK; ++b) {
        r = record_graph(c, b, 1, &c->g1[b]);
        if (r == DSMC_OK) r = record_graph(c, b, kGraphSteps, &c->gk[b]);
    }
    if (r != DSMC_OK) return fail(r);
    *out = c;
    return DSMC_OK;
}

dsmc_status dsmc_step(dsmc_ctx *c, int32_t n_steps) {
    if (!c || n_steps < 0) return DSMC_EINVAL;
    if (c->sticky != DSMC_OK) return c->sticky;
    const int nb = c->cfg.dims >= 1 ? 2 : 1;
    (void)nb;
    while (n_steps >= kGraphSteps) {
        HIP_TRY(hipGraphLaunch(c->gk[c->cur], c->stream));
        n_steps -= kGraphSteps;  // even number of steps: the current buffer is unchanged
    }
    while (n_steps > 0) {
        HIP_TRY(hipGraphLaunch(c->g1[c->cur], c->stream));
        if (c->cfg.dims >= 1) c->cur ^= 1;
        --n_steps;
    }
    return DSMC_OK;
}

dsmc_status dsmc_sample(dsmc_ctx *c, double *sums_host, uint64_t *counters_host, uint64_t *n_samples,
                        int32_t reset) {
    if (!c) return DSMC_EINVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dsmc_status s = device_status(c);
    if (sums_host) HIP_TRY(hipMemcpy(sums_host, c->sums, (size_t)c->ncell * kNsum * 8, hipMemcpyDeviceToHost));
    if (counters_host)
        HIP_TRY(hipMemcpy(counters_host, c->counters, (size_t)c->ncell * 16, hipMemcpyDeviceToHost));
    if (n_samples) HIP_TRY(hipMemcpy(n_samples, &c->st->n_samples, 8, hipMemcpyDeviceToHost));
    if (reset) {
        HIP_TRY(hipMemsetAsync(c->sums, 0, (size_t)c->ncell * kNsum * 8, c->stream));
        HIP_TRY(hipMemsetAsync(c->counters, 0, (size_t)c->ncell * 16, c->stream));
        HIP_TRY(hipMemsetAsync(&c->st->n_samples, 0, 8, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return s;
}

dsmc_status dsmc_particles(dsmc_ctx *c, dsmc_soa *cur) {
    if (!c || !cur) return DSMC_EINVAL;
    const Bufs &b = c->buf[c->cur];
    cur->x = b.x; cur->y = b.y; cur->cx = b.cx; cur->cy = b.cy; cur->cz = b.cz; cur->w = b.w; cur->id = b.id;
    return DSMC_OK;
}

dsmc_status dsmc_diagnostics(dsmc_ctx *c, dsmc_diag *out) {
    if (!c || !out) return DSMC_EINVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<unsigned char> stbuf(sizeof(DevState));
    DevState &st = *(DevState *)stbuf.data();
    HIP_TRY(hipMemcpy(&st, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
    std::vector<unsigned long long> cnt((size_t)c->ncell * 2);
    HIP_TRY(hipMemcpy(cnt.data(), c->counters, cnt.size() * 8, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->steps = st.step_next;
    for (int64_t i = 0; i < c->ncell; ++i) {
        out->candidates += cnt[2 * i];
        out->accepted += cnt[2 * i + 1];
    }
    unsigned long long tot[kDiagPerStripe] = {0};
    for (int sidx = 0; sidx < kDiagStripes; ++sidx)
        for (int k = 0; k < kDiagPerStripe; ++k) tot[k] += st.diag[sidx * kDiagPerStripe + k];
    out->overshoot = tot[kDiagOvershoot];
    out->wall_hits = tot[kDiagWallHits];
    out->learned_used = tot[kDiagLearned];
    out->fallback = tot[kDiagFallback];
    out->learned_skip = tot[kDiagSkip];
    out->vr_nonfinite = tot[kDiagVrNonfinite];
    out->big_cells = tot[kDiagBig];
    out->bounds_violations = tot[kDiagBounds];
#ifdef DSMC_BOUNDS_CHECK
    out->bounds_checked = 1;
#endif
    return device_status(c);
}

dsmc_status dsmc_set_step(dsmc_ctx *c, uint64_t next_step) {
    if (!c) return DSMC_EINVAL;
    HIP_TRY(hipMemcpyAsync(&c->st->step_next, &next_step, 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return DSMC_OK;
}

dsmc_status dsmc_set_majorant_model(dsmc_ctx *c, const uint16_t *bf16, int64_t n, double delta, int32_t min_n) {
    if (!c || !bf16 || n != DSMC_MLP_NPARAM || c->cfg.majorant != DSMC_MAJORANT_LEARNED || !std::isfinite(delta) ||
        min_n < 0)
        return DSMC_EINVAL;
    std::vector<float> in(DSMC_MLP_NPARAM), w(DSMC_MLP_NPARAM);
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t bits = (uint32_t)bf16[i] << 16;
        std::memcpy(&in[i], &bits, 4);
        if (!std::isfinite(in[i])) return DSMC_EINVAL;
    }
    // device layout: the hidden-to-hidden matrix is stored transposed so that
    // lane h reads W2[h][i] at i * 64 + h (coalesced across the wave)
    w = in;
    const int o_w2 = kMlpH * kMlpIn + kMlpH;
    for (int h = 0; h < kMlpH; ++h)
        for (int i = 0; i < kMlpH; ++i) w[o_w2 + i * kMlpH + h] = in[o_w2 + h * kMlpH + i];
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->mlp, w.data(), w.size() * 4, hipMemcpyHostToDevice));
    const bool was = c->mlp_loaded;
    c->mlp_loaded = true;
    c->mlp_delta = delta;
    c->mlp_min_n = (uint32_t)min_n;
    // the collision kernel's arguments change: re-record the graphs
    for (int b = 0; b < 2; ++b) {
        if (c->g1[b]) { (void)hipGraphExecDestroy(c->g1[b]); c->g1[b] = nullptr; }
        if (c->gk[b]) { (void)hipGraphExecDestroy(c->gk[b]); c->gk[b] = nullptr; }
    }
    (void)was;
    dsmc_status r = DSMC_OK;
    for (int b = 0; b < (c->cfg.dims >= 1 ? 2 : 1) && r == DSMC_OK; ++b) {
        r = record_graph(c, b, 1, &c->g1[b]);
        if (r == DSMC_OK) r = record_graph(c, b, kGraphSteps, &c->gk[b]);
    }
    return r;
}

dsmc_status dsmc_checkpoint(dsmc_ctx *c, void *blob, size_t *bytes) {
    if (!c || !bytes) return DSMC_EINVAL;
    const size_t n = (size_t)c->n, rb = (size_t)c->cfg.real_bytes, nc = (size_t)c->ncell;
    const size_t need = sizeof(BlobHeader) + 6 * n * rb + n * 4 + nc * kNsum * 8 + nc * 16;
    if (!blob) { *bytes = need; return DSMC_OK; }
    if (*bytes < need) return DSMC_EINVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dsmc_status s = device_status(c);
    if (s != DSMC_OK) return s;
    unsigned long long hdr[3];
    HIP_TRY(hipMemcpy(hdr, c->st, sizeof(hdr), hipMemcpyDeviceToHost));
    BlobHeader h{kBlobMagic, n, rb, (uint64_t)c->cfg.dims, nc, hdr[0], hdr[2], (uint64_t)c->cfg.vr};
    unsigned char *o = (unsigned char *)blob;
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    const Bufs &b = c->buf[c->cur];
    void *fields[6] = {b.x, b.y, b.cx, b.cy, b.cz, b.w};
    for (int f = 0; f < 6; ++f) {
        if (fields[f] && n) HIP_TRY(hipMemcpy(o, fields[f], n * rb, hipMemcpyDeviceToHost));
        else std::memset(o, 0, n * rb);
        o += n * rb;
    }
    if (n) HIP_TRY(hipMemcpy(o, b.id, n * 4, hipMemcpyDeviceToHost));
    o += n * 4;
    HIP_TRY(hipMemcpy(o, c->sums, nc * kNsum * 8, hipMemcpyDeviceToHost));
    o += nc * kNsum * 8;
    HIP_TRY(hipMemcpy(o, c->counters, nc * 16, hipMemcpyDeviceToHost));
    *bytes = need;
    return DSMC_OK;
}

dsmc_status dsmc_restore(dsmc_ctx *c, const void *blob, size_t bytes) {
    if (!c || !blob || bytes < sizeof(BlobHeader)) return DSMC_EINVAL;
    BlobHeader h;
    std::memcpy(&h, blob, sizeof(h));
    const size_t n = (size_t)c->n, rb = (size_t)c->cfg.real_bytes, nc = (size_t)c->ncell;
    const size_t need = sizeof(BlobHeader) + 6 * n * rb + n * 4 + nc * kNsum * 8 + nc * 16;
    if (h.magic != kBlobMagic || h.n != n || h.real_bytes != rb || h.dims != (uint64_t)c->cfg.dims || h.ncell != nc ||
        bytes < need)
        return DSMC_EINVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const unsigned char *o = (const unsigned char *)blob + sizeof(h);
    const Bufs &b = c->buf[c->cur];
    void *fields[6] = {b.x, b.y, b.cx, b.cy, b.cz, b.w};
    for (int f = 0; f < 6; ++f) {
        if (fields[f] && n) HIP_TRY(hipMemcpy(fields[f], o, n * rb, hipMemcpyHostToDevice));
        o += n * rb;
    }
    if (n) HIP_TRY(hipMemcpy(b.id, o, n * 4, hipMemcpyHostToDevice));
    o += n * 4;
    HIP_TRY(hipMemcpy(c->sums, o, nc * kNsum * 8, hipMemcpyHostToDevice));
    o += nc * kNsum * 8;
    HIP_TRY(hipMemcpy(c->counters, o, nc * 16, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&c->st->step_next, &h.step_next, 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&c->st->n_samples, &h.n_samples, 8, hipMemcpyHostToDevice));
    if (c->cfg.dims >= 1) {
        // the blob holds the particle sequence; its cell ranges follow from
        // the positions
        const dsmc_status rs = walled_setup(c, false);
        if (rs != DSMC_OK) return rs;
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return device_status(c);
}

dsmc_status dsmc_profile_step(dsmc_ctx *c, float *ms_host, int32_t max_kernels, int32_t *n_kernels,
                              char *names_host, int32_t names_len) {
    if (!c || !ms_host || !n_kernels || max_kernels <= 0) return DSMC_EINVAL;
    if (c->sticky != DSMC_OK) return c->sticky;
    std::vector<hipEvent_t> ev;
    std::vector<const char *> names;
    Launcher lead{c->stream, nullptr, nullptr};
    c->cur = enqueue_step(c, lead, c->cur);
    Launcher L{c->stream, &ev, &names};
    c->cur = enqueue_step(c, L, c->cur);
    L.mark("end");
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int nk = (int)ev.size() - 1;
    *n_kernels = std::min(nk, max_kernels);
    std::string all;
    for (int k = 0; k < nk; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        if (k < max_kernels) ms_host[k] = ms;
        all += names[k];
        all += '\n';
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    if (names_host && names_len > 0) {
        std::strncpy(names_host, all.c_str(), (size_t)names_len - 1);
        names_host[names_len - 1] = 0;
    }
    return device_status(c);
}

dsmc_status dsmc_estimators(const double *sums, int64_t n_cells, uint64_t n_samples, double FN,
                            const double *volume, double volume_uniform, int32_t vr, double vr_n0, double vr_T0,
                            double *out) {
    if (!sums || !out || n_cells < 0 || n_samples == 0 || !(FN > 0)) return DSMC_EINVAL;
    if (!volume && !(volume_uniform > 0)) return DSMC_EINVAL;
    for (int64_t c = 0; c < n_cells; ++c) {
        const double *S = sums + (size_t)c * DSMC_NSUM;
        const double V = volume ? volume[c] : volume_uniform;
        const double f = FN / (V * (double)n_samples);
        // density-weighted moments <1>, <c_d>, <c_d c_e> (xx yy zz xy xz yz), <c_d |c|^2>
        double d[13];
        for (int k = 0; k < 13; ++k) d[k] = (vr ? S[13 + k] : S[k]) * f;
        if (vr) {
            d[0] += vr_n0;
            for (int k = 4; k < 7; ++k) d[k] += vr_n0 * vr_T0;
        }
        double *o = out + (size_t)c * DSMC_NEST;
        const double n = d[0];
        const double u[3] = {d[1] / n, d[2] / n, d[3] / n};
        const double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
        const double tr = (d[4] + d[5]) + d[6];
        // full second-moment matrix from xx yy zz xy xz yz
        const double M[3][3] = {{d[4], d[7], d[8]}, {d[7], d[5], d[9]}, {d[8], d[9], d[6]}};
        o[0] = n;
        o[1] = u[0]; o[2] = u[1]; o[3] = u[2];
        o[4] = (tr / n - uu) / 3.0;
        const int pd[6] = {0, 1, 2, 0, 0, 1}, pe[6] = {0, 1, 2, 1, 2, 2};
        for (int k = 0; k < 6; ++k) o[5 + k] = M[pd[k]][pe[k]] - n * u[pd[k]] * u[pe[k]];
        for (int a = 0; a < 3; ++a) {
            const double ue = (u[0] * M[a][0] + u[1] * M[a][1]) + u[2] * M[a][2];
            o[11 + a] = 0.5 * (((d[10 + a] - 2.0 * ue) - u[a] * tr) + 2.0 * n * u[a] * uu);
        }
    }
    return DSMC_OK;
}

dsmc_status dsmc_collect_features(dsmc_ctx *c, float *features, float *labels, float *bounds, float *slimits) {
    if (!c || !features || !labels) return DSMC_EINVAL;
    if (c->sticky != DSMC_OK) return c->sticky;
    // the current buffer holds the particle sequence grouped by cell (walled
    // runs are grouped at set-up)
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->cfg.real_bytes == 4)
        hipLaunchKernelGGL(k_collect_features<float>, dim3((unsigned)c->ncell), dim3(kCollectThreads), 0, c->stream,
                           collide_args<float>(c, c->cur, c->cur), (int)c->ncell, features, labels, bounds, slimits);
    else
        hipLaunchKernelGGL(k_collect_features<double>, dim3((unsigned)c->ncell), dim3(kCollectThreads), 0, c->stream,
                           collide_args<double>(c, c->cur, c->cur), (int)c->ncell, features, labels, bounds, slimits);
    HIP_TRY(hipGetLastError());
    return DSMC_OK;
}

dsmc_status dsmc_destroy(dsmc_ctx *c) {
    if (!c) return DSMC_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    for (int b = 0; b < 2; ++b) {
        if (c->g1[b]) (void)hipGraphExecDestroy(c->g1[b]);
        if (c->gk[b]) (void)hipGraphExecDestroy(c->gk[b]);
    }
    if (c->capture) (void)hipStreamDestroy(c->capture);
    delete c;
    return DSMC_OK;
}

}  // extern "C"
