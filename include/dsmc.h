/*
 * dsmc.h -- C ABI of the MI355X (gfx950) direct simulation Monte Carlo hot path.
 *
 * The cited paper (arXiv 2301.05985) contains no Monte Carlo method; the
 * operations below follow the standard published DSMC method:
 * Bird, "Molecular Gas Dynamics and the Direct Simulation of Gas Flows" (1994)
 * for free flight, diffuse/specular/periodic walls, cell indexing, the
 * no-time-counter (NTC) collision scheme and cell sampling; Salmon et al.
 * (SC'11) for the Philox4x32-10 counter-based generator; Al-Mohssen &
 * Hadjiconstantinou (ESAIM M2AN 2010) for the importance-weight variance
 * reduction.  The problem solved is the spatially homogeneous or 1-D/2-D
 * Boltzmann equation for a simple gas, df/dt + c . grad_x f = Q(f, f), with
 * kinetic wall conditions; units take Boltzmann's constant and the molecular
 * mass as 1.
 *
 * Conventions for every call:
 *   - Every function returns dsmc_status (0 = DSMC_OK, negative = error).  No
 *     C++ exception and no abort crosses the ABI.
 *   - Pointers named "device" are HIP device pointers (e.g. torch tensor
 *     data pointers); pointers named "host" are ordinary host memory.
 *   - The caller owns every buffer passed in (particles, workspace, host
 *     arrays).  The context borrows device buffers until dsmc_destroy and
 *     copies host arrays during the call.  The library owns only the context
 *     object and the HIP graph it records; it never allocates device memory.
 *   - Work is enqueued asynchronously on the HIP stream given to dsmc_init.
 *     Device-side errors (too many wall hits, non-finite velocities, a cell
 *     larger than the kernels can hold) are recorded on the device and
 *     reported by the next synchronising call (dsmc_sample, dsmc_diagnostics,
 *     dsmc_checkpoint); the first error is sticky until dsmc_destroy.
 *   - One context is driven by one host thread at a time.
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSMC_ABI_VERSION 5
#define DSMC_NSUM 26          /* FP64 running sums per cell (see dsmc_sample) */
#define DSMC_MLP_NPARAM 4673  /* learned-majorant network 6-64-64-1 */

typedef struct dsmc_ctx dsmc_ctx; /* opaque, owned by the library */

typedef enum {
    DSMC_OK = 0,
    DSMC_EINVAL = -1,      /* invalid argument or configuration; nothing was launched */
    DSMC_ENOMEM = -2,      /* workspace smaller than dsmc_workspace_size reports */
    DSMC_EHIP = -3,        /* a HIP runtime call failed */
    DSMC_ENONFINITE = -4,  /* a velocity became NaN or infinite */
    DSMC_EWALLHITS = -5,   /* a particle hit walls more than max_wall_hits times in one step */
    DSMC_ECAPACITY = -6,   /* a per-cell candidate count (at most 2^24 per step) or cell size
                              exceeded the kernels' limits: also a walled cell of more than
                              131,072 particles at dsmc_init, or one whose overflow movers
                              (beyond the per-cell mover slots) times its particles exceed
                              2^28 in one step */
    DSMC_EABI = -7         /* abi_version mismatch */
} dsmc_status;

enum { DSMC_WALL_DIFFUSE = 0, DSMC_WALL_SPECULAR = 1, DSMC_WALL_PERIODIC = 2 };
/* Molecular models: hard spheres (sigma_T constant), Maxwell molecules
 * (sigma_T g constant), variable hard spheres (sigma_T = sigma g^(1 - 2 omega),
 * omega in [0.5, 1]; acceptance (g / g_max)^(2 - 2 omega) evaluated by a fixed
 * sequence of double operations, isotropic scattering) and variable soft
 * spheres (Koura & Matsumoto 1991: the VHS cross-section and acceptance, and
 * a deflection chi about the relative velocity with cos chi = 2 B^(1/alpha) - 1,
 * B uniform, alpha in [1, 2]; B and the azimuth are taken from the pair's
 * isotropic unit vector n as B = (1 + n_z)/2 and the direction of (n_x, n_y),
 * the turn computed in double in a fixed order). */
enum { DSMC_HARD_SPHERE = 0, DSMC_MAXWELL = 1, DSMC_VHS = 2, DSMC_VSS = 3 };
/* Majorant of the relative speed used by the NTC scheme in each cell:
 *   EXACT    (r_(1) + r_(2)) (1 + eps): radii about the velocity bounding-box
 *            midpoint; a bound on every pair, O(N) per cell;
 *   LEARNED  network proposal, used where proven to bound every pair,
 *            otherwise EXACT;
 *   DIAMETER the largest pair speed itself (1 + eps), O(N^2) per cell. */
enum { DSMC_MAJORANT_EXACT = 0, DSMC_MAJORANT_LEARNED = 1, DSMC_MAJORANT_DIAMETER = 2 };

/* Run configuration.  Cells: dims == 1 divides [0, length[0]] into n_cells[0]
 * equal cells; dims == 2 divides [0, length[0]] x [0, length[1]] into
 * n_cells[0] x n_cells[1] cells numbered iy * n_cells[0] + ix; dims == 0 is a
 * batch of n_cells[0] independent spatially homogeneous cells ("instances"),
 * instance b owning particles inst_offset[b] .. inst_offset[b+1]-1. */
typedef struct {
    int32_t abi_version;      /* must equal DSMC_ABI_VERSION */
    int32_t dims;             /* 0, 1 or 2 */
    int32_t real_bytes;       /* 4: FP32 positions/velocities/weights, 8: FP64 */
    int32_t molecule;         /* DSMC_HARD_SPHERE, DSMC_MAXWELL (sigma * g = const), DSMC_VHS or
                                 DSMC_VSS */
    int32_t n_cells[2];       /* (nx, ny); dims 1: ny ignored; dims 0: (n_instances, 1) */
    int32_t majorant;         /* DSMC_MAJORANT_EXACT, _LEARNED or _DIAMETER */
    int32_t vr;               /* 1: importance-weight variance reduction */
    double length[2];         /* domain extents (dims >= 1) */
    double dt;                /* time step */
    double sigma;             /* hard sphere: total cross-section; Maxwell: the constant sigma*g */
    double FN;                /* real molecules per simulated particle */
    double vr_T0;             /* temperature of the reference equilibrium (at rest) */
    int32_t wall_kind[4];     /* walls x-, x+, y-, y+: DSMC_WALL_* */
    double wall_T[4];         /* diffuse wall temperatures */
    double wall_u[4][3];      /* wall velocities (tangential components are used) */
    uint64_t seed;            /* Philox key: (low word, high word) */
    int64_t n_particles;
    const double *cell_volume;   /* host [n_cells] volumes, or NULL: uniform cell volume
                                    (dims 1: dx * 1 * 1, dims 2: dx * dy * 1, dims 0: 1) */
    const int64_t *inst_offset;  /* host [n_cells[0] + 1], dims == 0 only, ascending */
    int32_t max_wall_hits;    /* wall interactions allowed per particle per step (0 -> 64; a
                                 particle in a corner may bounce between two walls many times) */
    int32_t schedule;         /* homogeneous instances: DSMC_SCHEDULE_GRID or _PERSISTENT */
    int32_t persistent_waves; /* waves of the persistent kernel (0 -> 8 per compute unit) */
    int32_t vr_reconstruct;   /* vr == 1: re-estimate the weights in every step whose index is a
                                 multiple of this (0: never); see dsmc_step */
    int64_t chunk_work;       /* persistent kernel: up to 64 consecutive instances of the
                                 schedule form one work unit while they hold fewer than this
                                 many particles (0 -> one instance per unit) */
    double omega;             /* DSMC_VHS, DSMC_VSS: viscosity index in [0.5, 1]; sigma is the
                                 total cross-section at unit relative speed */
    double alpha;             /* DSMC_VSS: scattering exponent in [1, 2] (1: isotropic) */
    double vr_kappa;          /* vr == 1: factor (1 <= kappa <= 16; 0 reads as 1) applied to the
                                 relative-speed majorant, so that the acceptance probability p of
                                 every candidate is at most 1 / kappa and the weight update's
                                 1 / (1 - p) at most kappa / (kappa - 1) */
    int32_t wide_min;         /* homogeneous instances, grid schedule: instances of more than this
                                 many particles run on a workgroup of four waves (0 -> 1024, else
                                 at least 64; DSMC_EINVAL otherwise).  Changes no result. */
    int32_t occupancy;        /* homogeneous instances, grid schedule: waves per SIMD the one-wave
                                 collision kernel is compiled for, 5 or 6 (0 -> 5; DSMC_EINVAL
                                 otherwise).  Changes no result. */
    int32_t cells_per_wave;   /* walled runs (dims 1, 2): 2 -> each wave collides two cells, 32
                                 lanes each (exact or brute-force majorant, mean cell population
                                 at most 128; DSMC_EINVAL otherwise); 0 or 1 -> one cell per wave.
                                 Changes no result; with 2, cells above 0.96 x mean + 64 particles
                                 (at least 128) take the slower global-memory path. */
    int32_t waves_per_cell;   /* walled runs (dims 1, 2): 4 -> each cell collides on a workgroup
                                 of four waves (exact or brute-force majorant, one cell per wave
                                 otherwise; DSMC_EINVAL if combined with cells_per_wave 2); 0 or
                                 1 -> one wave.  For grids of few, populous cells.  Changes no
                                 result. */
} dsmc_config;

/* How homogeneous instances are distributed over the GPU.  Both process the
 * instances longest first (decreasing N, i.e. decreasing N^2 work) and give
 * identical results; only the speed differs.
 *   GRID        one workgroup (one wave) per instance, the hardware dispatcher
 *               handing out instances in that order as slots free up;
 *   PERSISTENT  a fixed grid of waves taking work units (one large instance,
 *               or a run of small ones) from eight device queues, one per XCD,
 *               a wave moving on to the other queues once its own is empty.
 * Walled runs (dims 1, 2) ignore the field and launch one wave per cell. */
enum { DSMC_SCHEDULE_GRID = 0, DSMC_SCHEDULE_PERSISTENT = 1 };

/* Structure-of-arrays particle state (device pointers).  Element type is
 * float (real_bytes 4) or double (real_bytes 8).  y is used only when
 * dims == 2, x only when dims >= 1, w only when vr == 1 (may be NULL
 * otherwise).  id holds a unique persistent particle number < 2^32.
 * Collision order inside a cell: storage order for dims == 0.  Walled runs
 * (dims >= 1) keep the particles as one sequence grouped by cell: at set-up
 * by the cell of the initial position with ascending id inside a cell, and
 * after each step's free flight regrouped by the new cell with the relative
 * order of the previous sequence kept (a stable counting sort); a cell's
 * particles collide in sequence order.  The storage order of the buffers is
 * that sequence.  Every non-NULL pointer must be 16-byte aligned (any
 * hipMalloc or torch allocation is); dsmc_init returns EINVAL otherwise. */
typedef struct {
    void *x, *y, *cx, *cy, *cz, *w;
    uint32_t *id;
} dsmc_soa;

typedef struct {
    uint64_t steps;           /* steps taken so far (the next step's index) */
    uint64_t candidates;      /* NTC candidates since the last reset of the samples */
    uint64_t accepted;        /* accepted collisions since the last reset */
    uint64_t overshoot;       /* candidates with relative speed above the majorant in use */
    uint64_t wall_hits;       /* wall interactions */
    uint64_t learned_used;    /* cell-steps that used the verified learned majorant */
    uint64_t fallback;        /* cell-steps whose learned proposal failed verification */
    uint64_t learned_skip;    /* cell-steps whose proposal was not below the exact bound */
    uint64_t vr_nonfinite;    /* cell samples with non-finite weighted sums (weight divergence) */
    uint64_t big_cells;       /* cell-steps processed by the global-memory collision kernel */
    uint64_t bounds_violations; /* kernel index checks that failed (bounds-checking build only) */
    uint64_t bounds_checked;  /* 1 if the library was built with kernel index checks
                                 (-DDSMC_BOUNDS_CHECK), else 0 */
} dsmc_diag;

/* Where a cell is collided.  A cell (or instance) is staged in the 64 KiB of
 * LDS a workgroup may hold if it has at most `cap` particles, and is collided
 * in global memory otherwise (counted in big_cells); both give the same
 * results.  With fit = floor(65472 / (4 real_bytes + 4)) rounded down to a
 * multiple of 32 (3264 in FP32, 1792 in FP64; homogeneous runs without
 * weights, whose owner marks share the weight slots: floor(65472 /
 * (4 real_bytes)) rounded down, 4064 in FP32, 2016 in FP64):
 *   dims == 0:  cap = the largest instance rounded up to a multiple of 32
 *               (at least 32), at most fit;
 *   dims >= 1:  cap = 3 x (mean particles per cell) + 64 rounded up to a
 *               multiple of 32, at least 64, at most fit. */

/* Bytes of device workspace the configuration needs (second particle
 * buffer of the regrouping, per-cell ranges, code bytes and mover lists,
 * FP64 running sums, counters, scratch).  EINVAL on an invalid
 * configuration. */
dsmc_status dsmc_workspace_size(const dsmc_config *cfg, size_t *bytes);

/* Validate the configuration, bind the particle buffers (device, caller
 * owned, n_particles each) and the workspace (device, >= workspace size,
 * 256-byte aligned), zero the running sums, and record the per-step HIP
 * graph on `hip_stream` (a hipStream_t; NULL = default stream).  For
 * dims == 0 the particle counts per instance come from inst_offset.  For
 * dims >= 1 the particles are rearranged in place into the initial sequence
 * (grouped by cell, ascending id inside a cell; the workspace's second
 * buffer is used in between); a cell of more than 131,072 initial particles
 * returns DSMC_ECAPACITY (the ordering by id is quadratic in the cell size).
 * No device allocation. */
dsmc_status dsmc_init(const dsmc_config *cfg, const dsmc_soa *particles, void *workspace,
                      size_t ws_bytes, void *hip_stream, dsmc_ctx **out);

/* Enqueue n_steps time steps (asynchronous).  Each step runs, in order:
 * free flight with wall conditions, new cell and code byte of every
 * particle (dims >= 1), the scan of the new cells' counts, then per cell the
 * gather of its particles into the new sequence (dims >= 1), NTC collisions
 * with the majorant chosen by cfg->majorant, the importance-weight update
 * (vr == 1), the re-estimation of the weights (vr == 1, vr_reconstruct > 0,
 * steps whose index is a multiple of vr_reconstruct), and accumulation of the
 * cell moments into the running sums.
 *
 * Weight re-estimation (the reconstruction step of Al-Mohssen &
 * Hadjiconstantinou 2010 in this library's form): in a cell of at least 26
 * particles the deviations W - 1 are replaced by their least-squares
 * projection onto the 13 functions 1, v, v_d v_e, v_d |v|^2 of
 * v = c / sqrt(vr_T0), the functions whose weighted sums the cell samples.
 * Every sampled weighted sum of the cell keeps its value (to rounding), unit
 * weights stay exactly 1, and the per-particle noise that the collision
 * update multiplies is removed.  A cell whose normal equations have a pivot
 * not above 1e-12 times its diagonal entry keeps its weights.  The weights
 * stay finite where the raw update diverges when collisions per particle and
 * step are few (about 0.1); with many collisions per step, or with a
 * reference temperature far from the flow's, the weights can still diverge
 * (vr_nonfinite counts the cells). */
dsmc_status dsmc_step(dsmc_ctx *ctx, int32_t n_steps);

/* Synchronise the stream and copy out the running sums (host
 * [n_cells][DSMC_NSUM] doubles, may be NULL), the per-cell counters (host
 * [n_cells][2] uint64: NTC candidates, accepted collisions; may be NULL) and
 * the number of sampled steps (may be NULL).  Sums, per cell:
 *   [0] N, [1..3] sum c, [4..9] sum c_d c_e (xx yy zz xy xz yz),
 *   [10..12] sum c_d |c|^2, and [13..25] the same 13 sums weighted by (1 - W)
 *   when vr == 1 (zero otherwise).
 * reset != 0 zeroes sums, counters and the sample count after copying. */
dsmc_status dsmc_sample(dsmc_ctx *ctx, double *sums_host, uint64_t *counters_host,
                        uint64_t *n_samples, int32_t reset);

/* Cell estimates from the running sums of dsmc_sample (host arithmetic in
 * FP64, no GPU work; Bird 1994 ratio estimators of time-summed moments).
 * sums_host [n_cells][DSMC_NSUM], n_samples sampled steps, F_N, cell
 * volumes (host [n_cells], or NULL for volume_uniform).  Plain (vr == 0):
 * with <Q> = S_Q F_N / (V n_samples),
 *   n = <1>, u = <c> / n, T = (tr <c c> / n - |u|^2) / 3,
 *   P_de = <c_d c_e> - n u_d u_e,
 *   q_d = 1/2 (<c_d |c|^2> - 2 u_e <c_d c_e> - u_d tr <c c> + 2 n u_d |u|^2);
 * weighted (vr == 1): every <Q> is the reference equilibrium's (vr_n0, at
 * rest, vr_T0) plus the (1 - W)-weighted sums scaled the same way.  Writes
 * out_host [n_cells][DSMC_NEST] = n, u_x, u_y, u_z, T, P_xx, P_yy, P_zz,
 * P_xy, P_xz, P_yz, q_x, q_y, q_z (NaN in a cell without particles).
 * EINVAL on NULL pointers, n_cells < 0 or n_samples == 0. */
#define DSMC_NEST 14
dsmc_status dsmc_estimators(const double *sums_host, int64_t n_cells, uint64_t n_samples, double FN,
                            const double *volume_host, double volume_uniform, int32_t vr, double vr_n0,
                            double vr_T0, double *out_host);

/* Device pointers of the buffers that hold the current particle state, in
 * sequence order (walled runs alternate between the caller's buffers and
 * the workspace).  Valid until the next dsmc_step. */
dsmc_status dsmc_particles(dsmc_ctx *ctx, dsmc_soa *current);

/* Synchronise and report diagnostics (host struct); returns the sticky
 * device error, if any. */
dsmc_status dsmc_diagnostics(dsmc_ctx *ctx, dsmc_diag *out);

/* Set the index of the next step (checkpoint/resume: the random stream is
 * keyed by step, so resuming at the same step continues the same run). */
dsmc_status dsmc_set_step(dsmc_ctx *ctx, uint64_t next_step);

/* Load the learned-majorant network: n == DSMC_MLP_NPARAM bfloat16 values
 * (host) in the order W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3; the
 * output is log2 of the predicted largest relative speed of the cell, and the
 * proposal is the lattice value 2^(k/64), k = ceil(64 (y + delta)).  The
 * proposal is used only where the kernel proves it bounds every pair of the
 * cell (every pair speed at most 2^(k/64) (1 - eps), eps = 2^-20 in FP32,
 * 2^-50 in FP64); elsewhere the exact bound is used, so results keep the law
 * of the exact method.  Under either majorant a pair that an earlier collision
 * of the same step made faster than the cell's majorant is accepted with
 * probability 1 instead of g / g_max (counted in dsmc_diag.overshoot; the
 * tighter learned majorant has a somewhat higher count).  Cells of fewer
 * than min_n particles skip the network and use the exact bound (counted as
 * learned_skip): a size gate for cells whose possible saving of candidates
 * cannot repay the network and the verification (see dsmc_mlp_calibrate).
 * EINVAL if n is wrong, min_n < 0 or cfg->majorant is not LEARNED. */
dsmc_status dsmc_set_majorant_model(dsmc_ctx *ctx, const uint16_t *bf16_weights_host, int64_t n,
                                    double delta, int32_t min_n);

/* Checkpoint: with host_blob == NULL, *bytes receives the size needed;
 * otherwise the particle state (in sequence order), step index, running
 * sums and counters are copied into host_blob (synchronising).  Restore
 * copies them back into the context's buffers; a run restored at step s
 * continues bit for bit like the uninterrupted run. */
dsmc_status dsmc_checkpoint(dsmc_ctx *ctx, void *host_blob, size_t *bytes);
dsmc_status dsmc_restore(dsmc_ctx *ctx, const void *host_blob, size_t bytes);

/* Run two steps: the first untimed (it keeps the GPU busy while the second
 * is enqueued, so that no launch waits on the host), the second with every
 * kernel launched separately and timed with HIP events on the context's
 * stream; ms_host receives up to max_kernels per-kernel durations
 * (milliseconds) of the second step in launch order, *n_kernels their number
 * and names_host (may be NULL) a '\n'-separated list of kernel names (at
 * most names_len bytes).  Synchronising.  Used for roofline reports. */
dsmc_status dsmc_profile_step(dsmc_ctx *ctx, float *ms_host, int32_t max_kernels,
                              int32_t *n_kernels, char *names_host, int32_t names_len);

/* Release the context and its HIP graph (the caller's buffers stay valid). */
dsmc_status dsmc_destroy(dsmc_ctx *ctx);

/* Static text for a status code. */
const char *dsmc_status_string(dsmc_status status);

/* ---------------------------------------------------------------------
 * Learned majorant: training-data collection and network training.
 * ------------------------------------------------------------------ */

/* For every cell (dims 0: instance) of the current state, write the six
 * FP32 input features of the learned majorant (device [n_cells][6]), the
 * label log2 of the exact largest pairwise relative speed (device [n_cells]
 * float; -inf marks cells with fewer than two particles), if bounds_dev is
 * not NULL log2 of the EXACT-mode bound, and if slimits_dev is not NULL
 * log2 of the 65th largest r_p + r_(1) (the verification's set S holds at
 * most 64 members exactly when the proposal's threshold is at least this;
 * -inf when the cell has at most 64 particles) (device [n_cells] float).
 * Features: log2(number density), u_x/sqrt(T), u_y/sqrt(T), log2(T),
 * P_xx/p - 1, P_xy/p, from FP64 moments of the cell (walled runs: the
 * particles currently grouped in the cell).  Asynchronous. */
dsmc_status dsmc_collect_features(dsmc_ctx *ctx, float *features_dev, float *labels_dev, float *bounds_dev,
                                  float *slimits_dev);

/* Forward pass of the 6-64-64-1 ReLU network in FP32 (params device
 * [DSMC_MLP_NPARAM] float, layout as in dsmc_set_majorant_model; x device
 * [n][6]; y device [n]).  Asynchronous on hip_stream. */
dsmc_status dsmc_mlp_forward(const float *params_dev, const float *x_dev, int64_t n,
                             float *y_dev, void *hip_stream);

/* Mean expectile loss  L = (1/n) sum |tau - 1[r < 0]| r^2,  r = label - y,
 * and its gradient with respect to every parameter (device
 * [DSMC_MLP_NPARAM] float, overwritten) and the loss (device float [1]).
 * Rows with a non-finite label are skipped.  scratch_dev must hold
 * dsmc_mlp_scratch_floats(n) floats (8-byte aligned); n at most
 * 65535 x 128, else EINVAL.  Asynchronous. */
dsmc_status dsmc_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *label_dev,
                               int64_t n, double tau, float *grad_dev, float *loss_dev,
                               float *scratch_dev, void *hip_stream);
int64_t dsmc_mlp_scratch_floats(int64_t n);

/* dsmc_mlp_loss_grad without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): it allocates nothing and uses a scratch
 * array of the library's own, about 5.5 MB per device, held from library
 * load to process end.  Same arguments, results and asynchrony as
 * dsmc_mlp_loss_grad; n at most DSMC_MLP_NOALLOC_MAX, else EINVAL.  The
 * stream must belong to the current device (EINVAL otherwise; NULL is the
 * current device's default stream).  All calls on one device share the
 * array: calls whose work overlaps on one device (different streams, or
 * host threads racing) corrupt each other's results; calls queued on one
 * stream are safe. */
#define DSMC_MLP_NOALLOC_MAX 4096
dsmc_status dsmc_mlp_loss_grad_noalloc(const float *params_dev, const float *x_dev, const float *label_dev,
                                       int64_t n, double tau, float *grad_dev, float *loss_dev, void *hip_stream);

/* Feature statistics and standardisation for training: over the rows with
 * a finite label, the means m_k and sample standard deviations s_k (at least
 * 1e-6) of the six features, the mean label and the row count, in FP64 and a
 * fixed order, into stats_dev (device, DSMC_MLP_NSTATS doubles: m[6], s[6],
 * mean label, count) and, if stats_host is not NULL, the same on the host
 * (then synchronising); xs_dev [n][6] receives (x - m) / s for every row.
 * Asynchronous otherwise. */
#define DSMC_MLP_NSTATS 14
dsmc_status dsmc_mlp_standardize(const float *x_dev, const float *label_dev, int64_t n, float *xs_dev,
                                 double *stats_dev, double *stats_host, void *hip_stream);

/* Fold the standardisation into the first layer of a network trained on
 * standardised inputs (params device, in place): W1[h][k] /= s_k,
 * b1[h] -= sum_k W1[h][k] m_k / s_k (stats_dev from dsmc_mlp_standardize),
 * so that the network takes the raw features.  Asynchronous. */
dsmc_status dsmc_mlp_fold_inputs(float *params_dev, const double *stats_dev, void *hip_stream);

/* bfloat16 bits of n floats (device to device), rounded to nearest with ties
 * to even (NaN stays NaN).  Asynchronous. */
dsmc_status dsmc_mlp_to_bf16(const float *params_dev, int64_t n, uint16_t *bits_dev, void *hip_stream);

/* Cost model of the learned majorant for dsmc_mlp_calibrate, hard spheres.
 * Costs are in candidate-equivalents (the time of one NTC candidate of the
 * exact method). */
typedef struct {
    double n_scale;       /* particles per unit number density in a cell: V / F_N */
    double cand_scale;    /* candidates per unit majorant and ordered pair: 0.5 F_N sigma dt / V */
    double eps;           /* the exact bound's rounding margin: 2^-20 (FP32 runs) or 2^-50 (FP64) */
    double cost_network;  /* per cell whose network is evaluated (features, network, lattice) */
    double cost_member;   /* per particle of a cell whose proposal is verified (membership of S) */
    double cost_verify;   /* per cell whose proposal is verified (collecting S, the pair check, and
                             the extra candidates of a fallback) */
} dsmc_calib_model;
#define DSMC_CALIB_NDELTA 128 /* margins delta_j = -0.64 + 0.01 j */
#define DSMC_CALIB_NBINS 8    /* cell sizes [2, 64), [64, 128), ..., [4096, inf) */
#define DSMC_CALIB_FIELDS 4   /* saved candidates, cost, cells using the proposal, fallbacks */

/* Choose the lattice margin delta and the size gate min_n of the learned
 * majorant on held-out cells (features, labels, bounds and slimits from
 * dsmc_collect_features; bits the network in bfloat16, device).  For each
 * margin and cell-size bin: a cell's proposal is verified when it is below
 * the exact bound, and used when its threshold 2^(k/64) (1 - eps) is at
 * least the largest pair speed and the cell's slimit; a used proposal saves
 * cand_scale N (N - 1) (bound - proposal) candidates; every cell pays
 * cost_network, every verified cell N cost_member + cost_verify.  Returns
 * the margin and gate (the smallest bin edge, or 0) of the largest net
 * saving; if no gate saves more than it costs, min_n = INT32_MAX (the
 * network is never used) and delta is the margin of the largest gross
 * saving.  table_host (may be NULL) receives [DSMC_CALIB_NDELTA]
 * [DSMC_CALIB_NBINS][DSMC_CALIB_FIELDS] doubles.  work_dev: device, 256-byte
 * aligned, at least dsmc_mlp_calib_work_bytes(n).  Synchronising. */
size_t dsmc_mlp_calib_work_bytes(int64_t n);
dsmc_status dsmc_mlp_calibrate(const uint16_t *bits_dev, const float *features_dev, const float *labels_dev,
                               const float *bounds_dev, const float *slimits_dev, int64_t n,
                               const dsmc_calib_model *model, void *work_dev, size_t work_bytes,
                               double *delta_out, int32_t *min_n_out, double *table_host, void *hip_stream);

/* One Adam update (Kingma & Ba 2015) of params in place from grad, with the
 * first and second moment buffers m, v (device [n_param] float) and the
 * 1-based step index t.  Asynchronous. */
dsmc_status dsmc_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                          int64_t n_param, int64_t t, double lr, double beta1, double beta2,
                          double eps, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_H */
