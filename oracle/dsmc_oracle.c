/*
 * dsmc_oracle.c -- plain, slow, single-threaded CPU oracle of the DSMC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant table with the HIP implementation; both are written
 * independently from the method description below.
 *
 * The cited paper (arXiv 2301.05985, on finite-element electrokinetics)
 * contains no Monte Carlo method, so every step here follows the standard
 * published method named in its comment:
 *   - Bird, "Molecular Gas Dynamics and the Direct Simulation of Gas Flows"
 *     (1994): no-time-counter (NTC) collision selection, hard-sphere
 *     isotropic scattering, diffuse wall reflection, cell sampling.
 *   - Salmon et al., SC'11: the Philox4x32-10 counter-based generator.
 *   - Marsaglia (1972): uniform point on the unit sphere.
 *   - Al-Mohssen & Hadjiconstantinou, ESAIM M2AN (2010): importance-weight
 *     variance reduction relative to a reference equilibrium.
 * Every choice the literature leaves open (keying of the random stream,
 * operation order, the exact majorant) is fixed by the project's reading and
 * is restated next to the code that implements it.
 *
 * The file is compiled twice: REAL=double with suffix _f64 and REAL=float
 * with suffix _f32.  The float build takes every decision (pair choice,
 * acceptance, wall hits, cell index) in single precision, the precision the
 * GPU path uses for its FP32 configurations; accumulations and per-cell
 * scalars stay in double in both builds.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, so
 * every rounding step is the one written here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#error "compile with -DREAL=double or -DREAL=float"
#endif
#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SFX)

#define IS_F32 (sizeof(REAL) == 4)

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 round
 * function with the two multipliers below, key bumped by the Weyl constants
 * between rounds. */
static void orc_philox_impl(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

#ifdef ORC_PRIMARY
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    orc_philox_impl(ctr, key, out);
}
#endif

/* Keying of the stream (project reading): counter = (c0 = sub-index such as
 * candidate number or wall-hit number, c1 = tag << 24 | block,
 * c2 = cell / instance / particle id, c3 = time step), key = the 64-bit seed
 * split in two words. */
enum { TAG_NCAND = 1, TAG_PAIR = 2, TAG_WALL = 3 };

static void draw(const uint32_t key[2], uint32_t c0, uint32_t tag, uint32_t block,
                 uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, (tag << 24) | block, c2, c3};
    orc_philox_impl(ctr, key, out);
}

/* 53-bit uniform on [0,1) from two words: top 32 bits of the first word,
 * top 21 bits of the second. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * (1.0 / 9007199254740992.0);
}
/* 24-bit uniform on [0,1) from the top 24 bits of one word. */
static float u24(uint32_t a)
{
    return (float)(a >> 8) * (1.0f / 16777216.0f);
}

/* Ordered distinct pair from two words by the multiply-shift map
 * (floor(r * n / 2^32), Lemire 2019, without rejection). */
static uint32_t mulhi32(uint32_t r, uint32_t n)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

/* ---------------------------------------------------------------- types */
typedef struct {
    int32_t dims, nx, ny, molecule;     /* molecule: 0 hard sphere, 1 Maxwell, 2 VHS, 3 VSS */
    int32_t vr, majorant, n_inst, max_wall_hits;
    double Lx, Ly, dt, sigma, FN, vr_T0;
    int32_t wall_kind[4];               /* 0 diffuse, 1 specular, 2 periodic; x-,x+,y-,y+ */
    double wall_T[4];
    double wall_u[12];                  /* wall velocity, 3 components per wall */
    uint32_t key[2];
    const double *cell_volume;          /* per cell, or NULL for uniform */
    const int64_t *inst_offset;         /* dims == 0: [n_inst + 1] */
    const float *mlp;                   /* learned majorant weights (FP32 copy of BF16), or NULL */
    double mlp_delta;                   /* lattice margin in log2 units */
    const int64_t *cell_ids;            /* dims == 0: random-stream id of each instance, or NULL (= index) */
    const int64_t *only_cells;          /* if not NULL: collide and sample only these cells ... */
    int64_t n_only;                     /* ... (sorted ascending, n_only of them) */
    double omega;                       /* molecules 2 (VHS), 3 (VSS): viscosity index in [0.5, 1] */
    double alpha;                       /* molecule 3 (VSS): scattering exponent in [1, 2] */
    int32_t vr_reconstruct;             /* K > 0: re-estimate the weights in steps s with s mod K == 0 */
    int32_t pad_;
    double vr_kappa;                    /* weighted runs: majorant factor (>= 1; 0 is read as 1) */
    int64_t mlp_min_n;                  /* learned majorant: cells of fewer particles use the exact bound */
} orc_cfg;

typedef struct {
    uint64_t overshoot;      /* candidates whose relative speed exceeded the majorant in use */
    uint64_t wall_hits;
    uint64_t learned_used;   /* cells where the verified learned majorant was used */
    uint64_t fallback;       /* cells where the learned proposal failed verification */
    uint64_t learned_skip;   /* cells where the proposal was not below the exact bound */
    uint64_t vr_nonfinite;   /* cell samples whose weighted sums were not finite */
    int64_t error;           /* 0, -4 non-finite, -5 too many wall hits, -6 capacity */
} orc_diag;

enum { ERR_NONFINITE = -4, ERR_WALLHITS = -5, ERR_CAPACITY = -6 };
#define NSUM 26

/* ------------------------------------------------------- exact majorant */
/* Exact per-cell majorant (project reading): m = midpoint of the velocity
 * bounding box, r_p = |c_p - m|, bound = (r_(1) + r_(2)) * (1 + eps).  By the
 * triangle inequality |c_i - c_j| <= r_i + r_j <= r_(1) + r_(2) for every
 * pair; eps covers the rounding of the bound and of the acceptance test. */
double FN(orc_exact_bound)(const REAL *cx, const REAL *cy, const REAL *cz,
                           const int64_t *list, int64_t n)
{
    if (n < 2) return 0.0;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        double v[3] = {(double)cx[p], (double)cy[p], (double)cz[p]};
        for (int d = 0; d < 3; ++d) {
            if (v[d] < lo[d]) lo[d] = v[d];
            if (v[d] > hi[d]) hi[d] = v[d];
        }
    }
    double m[3];
    for (int d = 0; d < 3; ++d) m[d] = 0.5 * (hi[d] + lo[d]);
    double r2a = 0.0, r2b = 0.0; /* largest and second largest r^2 */
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        double dx = (double)cx[p] - m[0], dy = (double)cy[p] - m[1], dz = (double)cz[p] - m[2];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 > r2a) { r2b = r2a; r2a = r2; }
        else if (r2 > r2b) { r2b = r2; }
    }
    double eps = IS_F32 ? 9.5367431640625e-07 /* 2^-20 */ : 8.8817841970012523e-16 /* 2^-50 */;
    return (sqrt(r2a) + sqrt(r2b)) * (1.0 + eps);
}

/* Brute-force largest pairwise relative speed (the true per-cell maximum).
 * Used as the training label of the learned majorant and by the tests. */
double FN(orc_diameter)(const REAL *cx, const REAL *cy, const REAL *cz,
                        const int64_t *list, int64_t n)
{
    double best = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        for (int64_t b = a + 1; b < n; ++b) {
            int64_t q = list ? list[b] : b;
            double dx = (double)cx[p] - (double)cx[q];
            double dy = (double)cy[p] - (double)cy[q];
            double dz = (double)cz[p] - (double)cz[q];
            double g2 = (dx * dx + dy * dy) + dz * dz;
            if (g2 > best) best = g2;
        }
    }
    return sqrt(best);
}

/* ------------------------------------------------- post-collision state */
/* Uniform unit vector by Marsaglia's method: u, v uniform on (-1, 1),
 * rejected unless 0 < s = u^2 + v^2 < 1, then
 * n = (2u sqrt(1-s), 2v sqrt(1-s), 1 - 2s).  Attempts come from blocks
 * 1, 2, ... of the candidate's PAIR stream: one attempt per block in double
 * (two 53-bit uniforms), two per block in float (four 24-bit uniforms).  After
 * 64 blocks without success (probability below 1e-40) n = (0, 0, 1). */
void FN(orc_direction)(const uint32_t key[2], uint32_t k, uint32_t cell, uint32_t step, REAL n[3])
{
    for (uint32_t b = 1; b <= 64; ++b) {
        uint32_t r[4];
        draw(key, k, TAG_PAIR, b, cell, step, r);
        int attempts = IS_F32 ? 2 : 1;
        for (int a = 0; a < attempts; ++a) {
            REAL u, v;
            if (IS_F32) {
                u = (REAL)2 * (REAL)u24(r[2 * a]) - (REAL)1;
                v = (REAL)2 * (REAL)u24(r[2 * a + 1]) - (REAL)1;
            } else {
                u = (REAL)2 * (REAL)u53(r[0], r[1]) - (REAL)1;
                v = (REAL)2 * (REAL)u53(r[2], r[3]) - (REAL)1;
            }
            REAL s = u * u + v * v;
            if (s < (REAL)1 && s > (REAL)0) {
                REAL h = IS_F32 ? (REAL)sqrtf((float)((REAL)1 - s)) : (REAL)sqrt((double)((REAL)1 - s));
                n[0] = ((REAL)2 * u) * h;
                n[1] = ((REAL)2 * v) * h;
                n[2] = (REAL)1 - (REAL)2 * s;
                return;
            }
        }
    }
    n[0] = 0; n[1] = 0; n[2] = 1;
}

/* Hard-sphere (and Maxwell-molecule) elastic collision with isotropic
 * scattering: centre-of-mass velocity kept, relative speed g kept, new
 * relative direction n.  c_i' = c_m + g/2 n, c_j' = c_m - g/2 n. */
void FN(orc_scatter)(REAL ci[3], REAL cj[3], REAL g2, const REAL n[3])
{
    REAL g = IS_F32 ? (REAL)sqrtf((float)g2) : (REAL)sqrt((double)g2);
    REAL hg = (REAL)0.5 * g;
    for (int d = 0; d < 3; ++d) {
        REAL cm = (REAL)0.5 * (ci[d] + cj[d]);
        REAL t = hg * n[d];
        ci[d] = cm + t;
        cj[d] = cm - t;
    }
}

/* Importance-weight update for one candidate (Al-Mohssen &
 * Hadjiconstantinou 2010).  With acceptance probability p of the simulated
 * process, the reference-equilibrium process accepts the same candidate with
 * probability p * W_partner, so the likelihood ratio of each particle's
 * history is multiplied by W_partner on acceptance and by
 * (1 - p W_partner) / (1 - p) on rejection.  Arithmetic in double. */
void FN(orc_vr_update)(int accepted, double p, REAL *wi, REAL *wj)
{
    double a = (double)*wi, b = (double)*wj;
    if (accepted) {
        double ab = a * b;
        *wi = (REAL)ab;
        *wj = (REAL)ab;
    } else {
        double q = 1.0 - p;
        if (q > 0.0) {
            *wi = (REAL)((a * (1.0 - p * b)) / q);
            *wj = (REAL)((b * (1.0 - p * a)) / q);
        }
    }
}

/* ------------------------------------------------------- wall sampler */
/* Diffuse (fully accommodating) wall at temperature Tw: the outgoing
 * velocity is drawn from the normalized flux Maxwellian.  Normal speed
 * c_n = sqrt(-2 Tw ln(1-U1)); tangential components by Box-Muller from
 * (U2, U3), scaled by sqrt(Tw).  Stream: WALL tag, c0 = hit number,
 * c2 = particle id, c3 = step; double uses blocks 0 and 1
 * (U1, U2 from block 0, U3 from block 1), float uses block 0 words 0..2. */
void FN(orc_wall_draw)(const uint32_t key[2], uint32_t hit, uint32_t pid, uint32_t step,
                       double Tw, REAL out[3] /* c_n, t1, t2 (unit-variance Gaussians scaled) */)
{
    uint32_t b0[4], b1[4];
    draw(key, hit, TAG_WALL, 0, pid, step, b0);
    if (IS_F32) {
        float U1 = u24(b0[0]), U2 = u24(b0[1]), U3 = u24(b0[2]);
        float T = (float)Tw;
        float cn = sqrtf((-2.0f * T) * logf(1.0f - U1));
        float rad = sqrtf(-2.0f * logf(1.0f - U2));
        float th = 6.28318530717958647692f * U3;
        float sT = sqrtf(T);
        out[0] = (REAL)cn;
        out[1] = (REAL)(sT * (rad * cosf(th)));
        out[2] = (REAL)(sT * (rad * sinf(th)));
    } else {
        draw(key, hit, TAG_WALL, 1, pid, step, b1);
        double U1 = u53(b0[0], b0[1]), U2 = u53(b0[2], b0[3]), U3 = u53(b1[0], b1[1]);
        double cn = sqrt((-2.0 * Tw) * log(1.0 - U1));
        double rad = sqrt(-2.0 * log(1.0 - U2));
        double th = 6.28318530717958647692 * U3;
        double sT = sqrt(Tw);
        out[0] = (REAL)cn;
        out[1] = (REAL)(sT * (rad * cos(th)));
        out[2] = (REAL)(sT * (rad * sin(th)));
    }
}

/* Weight factor at a diffuse wall: ratio of the reference-equilibrium
 * flux Maxwellian (T0, at rest) to the wall's flux Maxwellian (Tw, uw), both
 * of the form c_n / (2 pi T^2) exp(-|c - u|^2 / 2T). */
double FN(orc_wall_ratio)(const REAL c[3], double Tw, const double uw[3], double T0)
{
    double v0 = (double)c[0], v1 = (double)c[1], v2 = (double)c[2];
    double c2_0 = (v0 * v0 + v1 * v1) + v2 * v2;
    double d0 = v0 - uw[0], d1 = v1 - uw[1], d2 = v2 - uw[2];
    double c2_w = (d0 * d0 + d1 * d1) + d2 * d2;
    double ex = c2_w / (2.0 * Tw) - c2_0 / (2.0 * T0);
    return ((Tw * Tw) / (T0 * T0)) * exp(ex);
}

/* ----------------------------------------------------------- streaming */
typedef struct {
    REAL *x, *y, *cx, *cy, *cz, *w;
    const uint32_t *id;
} soa_t;

/* Move one particle for one time step with exact times of flight to the
 * walls it moves toward (Bird 1994, free molecular motion).  The free end
 * point x + c tau is computed first; if it lies in the closed box the particle
 * moves there without meeting a wall.  Otherwise the times of flight decide
 * which wall is met first; a hit snaps the particle onto the wall, applies
 * the wall's condition and continues with the remaining time.  On a corner
 * tie the x wall is taken first.  More than max_wall_hits hits in one step is
 * an error. */
static int stream_one(const orc_cfg *cfg, soa_t *s, int64_t p, uint32_t step, orc_diag *diag)
{
    const REAL Lx = (REAL)cfg->Lx, Ly = (REAL)cfg->Ly;
    REAL x = s->x[p], y = (cfg->dims == 2) ? s->y[p] : (REAL)0;
    REAL c[3] = {s->cx[p], s->cy[p], s->cz[p]};
    REAL tau = (REAL)cfg->dt;
    uint32_t hits = 0;
    int rc = 0;
    for (;;) {
        REAL xe = x + c[0] * tau;
        REAL ye = (cfg->dims == 2) ? y + c[1] * tau : (REAL)0;
        if (xe >= (REAL)0 && xe <= Lx && (cfg->dims < 2 || (ye >= (REAL)0 && ye <= Ly))) {
            x = xe;
            if (cfg->dims == 2) y = ye;
            break;
        }
        REAL tx = (REAL)INFINITY, ty = (REAL)INFINITY;
        if (c[0] > (REAL)0) tx = (Lx - x) / c[0];
        else if (c[0] < (REAL)0) tx = ((REAL)0 - x) / c[0];
        if (cfg->dims == 2) {
            if (c[1] > (REAL)0) ty = (Ly - y) / c[1];
            else if (c[1] < (REAL)0) ty = ((REAL)0 - y) / c[1];
        }
        REAL t = tx <= ty ? tx : ty;
        if (t < (REAL)0) t = (REAL)0;
        if (t >= tau) {
            x = x + c[0] * tau;
            if (cfg->dims == 2) y = y + c[1] * tau;
            break;
        }
        int xwall = tx <= ty;
        x = x + c[0] * t;
        if (cfg->dims == 2) y = y + c[1] * t;
        tau = tau - t;
        int wall;
        if (xwall) { wall = c[0] > (REAL)0 ? 1 : 0; x = wall ? Lx : (REAL)0; }
        else       { wall = c[1] > (REAL)0 ? 3 : 2; y = wall == 3 ? Ly : (REAL)0; }
        if ((int)hits >= cfg->max_wall_hits) { rc = ERR_WALLHITS; break; }
        int nd = xwall ? 0 : 1;            /* normal component */
        int t1 = xwall ? 1 : 0, t2 = 2;    /* tangential components */
        int kind = cfg->wall_kind[wall];
        if (kind == 2) {                   /* periodic: re-enter at the opposite face */
            if (xwall) x = wall ? (REAL)0 : Lx;
            else       y = wall == 3 ? (REAL)0 : Ly;
        } else if (kind == 1) {            /* specular */
            c[nd] = -c[nd];
        } else {                           /* diffuse */
            REAL d[3];
            double Tw = cfg->wall_T[wall];
            const double *uw = &cfg->wall_u[3 * wall];
            FN(orc_wall_draw)(cfg->key, hits, s->id[p], step, Tw, d);
            REAL sign = (wall & 1) ? (REAL)-1 : (REAL)1; /* inward normal */
            c[nd] = sign * d[0];
            c[t1] = d[1] + (REAL)uw[t1];
            c[t2] = d[2] + (REAL)uw[t2];
            if (cfg->vr) {
                double ratio = FN(orc_wall_ratio)(c, Tw, uw, cfg->vr_T0);
                s->w[p] = (REAL)((double)s->w[p] * ratio);
            }
        }
        hits++;
    }
    diag->wall_hits += hits;
    s->x[p] = x;
    if (cfg->dims == 2) s->y[p] = y;
    s->cx[p] = c[0]; s->cy[p] = c[1]; s->cz[p] = c[2];
    return rc;
}

/* Cell index: floor(x * n / L) clamped to [0, n-1], computed in double;
 * 2-D cells are numbered row-major, iy * nx + ix. */
static int64_t cell_of(const orc_cfg *cfg, REAL x, REAL y)
{
    double invx = (double)cfg->nx / cfg->Lx;
    double fx = floor((double)x * invx);
    int64_t ix = fx < 0.0 ? 0 : (fx > (double)(cfg->nx - 1) ? cfg->nx - 1 : (int64_t)fx);
    if (cfg->dims < 2) return ix;
    double invy = (double)cfg->ny / cfg->Ly;
    double fy = floor((double)y * invy);
    int64_t iy = fy < 0.0 ? 0 : (fy > (double)(cfg->ny - 1) ? cfg->ny - 1 : (int64_t)fy);
    return iy * cfg->nx + ix;
}

/* --------------------------------------------------- learned majorant */
/* MLP 6 -> 64 -> 64 -> 1 with ReLU, FP32 arithmetic in the fixed order that
 * decides the lattice index: hidden unit h accumulates its inputs in
 * ascending order with fused multiply-adds starting from its bias; the output
 * layer multiplies each hidden activation by its weight and sums the 64
 * products by the pairwise (butterfly) tree with strides 32, 16, 8, 4, 2, 1,
 * then adds the output bias.  Weight layout (4673 floats): W1[64][6], b1[64],
 * W2[64][64], b2[64], w3[64], b3. */
#define MLP_IN 6
#define MLP_H 64
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

float FN(orc_mlp_forward_f32)(const float *prm, const float in[MLP_IN])
{
    const float *W1 = prm, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H,
                *b2 = W2 + MLP_H * MLP_H, *w3 = b2 + MLP_H, *b3 = w3 + MLP_H;
    float a1[MLP_H], s[MLP_H];
    for (int h = 0; h < MLP_H; ++h) {
        float acc = b1[h];
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(W1[h * MLP_IN + i], in[i], acc);
        a1[h] = acc > 0.0f ? acc : 0.0f;
    }
    for (int h = 0; h < MLP_H; ++h) {
        float acc = b2[h];
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(W2[h * MLP_H + i], a1[i], acc);
        float a2 = acc > 0.0f ? acc : 0.0f;
        s[h] = w3[h] * a2;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        float t[MLP_H];
        for (int l = 0; l < MLP_H; ++l) t[l] = s[l] + s[l ^ off];
        memcpy(s, t, sizeof(t));
    }
    return s[0] + b3[0];
}

/* Input features of the learned majorant, from the pre-collision state of
 * the cell: FP64 moments, rounded once to float.
 *   f0 = log2(n) where n = N F_N / V (number density),
 *   f1, f2 = u_x / sqrt(T), u_y / sqrt(T),
 *   f3 = log2(T),
 *   f4 = P_xx / p - 1, f5 = P_xy / p  (p = n T). */
void FN(orc_features)(const REAL *cx, const REAL *cy, const REAL *cz, const int64_t *list,
                      int64_t n, double FNum, double V, float out[MLP_IN])
{
    double S1[3] = {0, 0, 0}, Sxx = 0, Syy = 0, Szz = 0, Sxy = 0;
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        double vx = (double)cx[p], vy = (double)cy[p], vz = (double)cz[p];
        S1[0] += vx; S1[1] += vy; S1[2] += vz;
        Sxx += vx * vx; Syy += vy * vy; Szz += vz * vz; Sxy += vx * vy;
    }
    double N = (double)n;
    double ux = S1[0] / N, uy = S1[1] / N, uz = S1[2] / N;
    double T = (((Sxx + Syy) + Szz) / N - ((ux * ux + uy * uy) + uz * uz)) / 3.0;
    if (!(T > 1e-300)) T = 1e-300;
    double dens = (N * FNum) / V;
    double Pxx = dens * (Sxx / N - ux * ux);
    double Pxy = dens * (Sxy / N - ux * uy);
    double pr = dens * T;
    double sT = sqrt(T);
    out[0] = (float)log2(dens);
    out[1] = (float)(ux / sT);
    out[2] = (float)(uy / sT);
    out[3] = (float)log2(T);
    out[4] = (float)(Pxx / pr - 1.0);
    out[5] = (float)(Pxy / pr);
}

/* Lattice of admissible majorants: g = 2^(k/64), k integer.  The proposal is
 * k = ceil(64 (y + delta)) where y is the network output (log2 units). */
static double lattice_value(int64_t k) { return exp2((double)k / 64.0); }

/* Learned majorant with exact verification (project design).  The proposal
 * is used only when it is below the exact bound and provably bounds every
 * pair: with g_v = g_pred (1 - eps), pairs whose speed can exceed g_v both lie
 * in S = {p : r_p + r_(1) > g_v}; if |S| > 64 the proposal is rejected,
 * otherwise all pairs of S are checked by brute force against g_v.  Cells of
 * fewer than mlp_min_n particles skip the proposal.  Otherwise the exact
 * bound is used.  Returns the majorant; *used = 1 learned, 0 skip, -1 fallback. */
double FN(orc_learned_majorant)(const orc_cfg *cfg, const REAL *cx, const REAL *cy, const REAL *cz,
                                const int64_t *list, int64_t n, double V, int *used)
{
    double gb = FN(orc_exact_bound)(cx, cy, cz, list, n);
    /* size gate: small cells cannot repay the network and the verification */
    if (n < cfg->mlp_min_n) { *used = 0; return gb; }
    float f[MLP_IN];
    FN(orc_features)(cx, cy, cz, list, n, cfg->FN, V, f);
    float y = FN(orc_mlp_forward_f32)(cfg->mlp, f);
    double kk = ceil(64.0 * ((double)y + cfg->mlp_delta));
    if (!(kk > -4096.0)) kk = -4096.0;
    if (kk > 4096.0) kk = 4096.0;
    double gp = lattice_value((int64_t)kk);
    if (!(gp < gb)) { *used = 0; return gb; }
    /* radii about the bounding-box midpoint, as for the exact bound */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        double v[3] = {(double)cx[p], (double)cy[p], (double)cz[p]};
        for (int d = 0; d < 3; ++d) { if (v[d] < lo[d]) lo[d] = v[d]; if (v[d] > hi[d]) hi[d] = v[d]; }
    }
    double m[3];
    for (int d = 0; d < 3; ++d) m[d] = 0.5 * (hi[d] + lo[d]);
    double r1 = 0.0;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list ? list[a] : a;
        double dx = (double)cx[p] - m[0], dy = (double)cy[p] - m[1], dz = (double)cz[p] - m[2];
        r[a] = sqrt((dx * dx + dy * dy) + dz * dz);
        if (r[a] > r1) r1 = r[a];
    }
    /* verification threshold: the proposal less the exact bound's rounding
     * margin, so that a verified pair stays below the proposal also after
     * both are rounded to the working precision of the acceptance test */
    double eps = IS_F32 ? 9.5367431640625e-07 /* 2^-20 */ : 8.8817841970012523e-16 /* 2^-50 */;
    double gv = gp * (1.0 - eps);
    int64_t S[64];
    int64_t ns = 0;
    int ok = 1;
    for (int64_t a = 0; a < n; ++a) {
        if (r[a] + r1 > gv) {
            if (ns == 64) { ok = 0; break; }
            S[ns++] = list ? list[a] : a;
        }
    }
    free(r);
    if (ok) {
        /* every pair with speed above g_v lies inside S; compare against g_v^2 */
        double gv2 = gv * gv;
        for (int64_t a = 0; a < ns && ok; ++a)
            for (int64_t b = a + 1; b < ns; ++b) {
                double dx = (double)cx[S[a]] - (double)cx[S[b]];
                double dy = (double)cy[S[a]] - (double)cy[S[b]];
                double dz = (double)cz[S[a]] - (double)cz[S[b]];
                double g2 = (dx * dx + dy * dy) + dz * dz;
                if (g2 > gv2) { ok = 0; break; }
            }
    }
    if (!ok) { *used = -1; return gb; }
    *used = 1;
    return gp;
}

/* ------------------------------------------------------ collide + sample */
static const uint32_t *g_sort_ids; /* single-threaded oracle: qsort context */
static int cmp_by_id(const void *a, const void *b)
{
    uint32_t ia = g_sort_ids[*(const int64_t *)a], ib = g_sort_ids[*(const int64_t *)b];
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* ------------------------------------------------------------ VHS power */
/* x^a for x >= 0, 0 <= a <= 1, as 2^(a log2 x), in a fixed sequence of IEEE
 * double operations (no library transcendental), so that a decision taken
 * on it is identical wherever the same sequence runs.
 *   log2: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
 *         s = (m - 1)/(m + 1), |s| < 0.1716, by its odd series through s^27
 *         (Horner in s^2); log2 x = e + ln m / ln 2.
 *   exp2: y = n + f, n = floor(y), f in [0, 1); 2^f = e^(f ln 2) by its
 *         Taylor series through degree 18 (Horner on the coefficients 1/k!,
 *         a multiply and an add per degree); scaled by 2^n exactly. */
static const double VHS_LN2 = 0.69314718055994530942;
static const double VHS_INV_LN2 = 1.44269504088896340736;
static double vhs_log2(double x)
{
    int e;
    double m = frexp(x, &e); /* m in [0.5, 1) */
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    double sv = (m - 1.0) / (m + 1.0);
    double s2 = sv * sv;
    double t = 1.0 / 27.0;
    for (int k = 25; k >= 1; k -= 2) t = t * s2 + 1.0 / (double)k;
    double lnm = (2.0 * sv) * t;
    return (double)e + lnm * VHS_INV_LN2;
}
static double vhs_exp2(double y)
{
    /* Taylor coefficients 1/k!, k = 0..18: each the rounded quotient of two
     * exactly representable integers */
    static const double c[19] = {
        1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
        1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
        1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0,
        1.0 / 355687428096000.0, 1.0 / 6402373705728000.0};
    double n = floor(y);
    double f = (y - n) * VHS_LN2;
    double t = c[18];
    for (int k = 17; k >= 0; --k) t = t * f + c[k];
    return ldexp(t, (int)n);
}
static double vhs_pow(double x, double a)
{
    if (a == 0.0) return 1.0;
    if (!(x > 0.0)) return 0.0;
    if (x == 1.0) return 1.0;
    double y = a * vhs_log2(x);
    if (y < -1000.0) return 0.0;
    return vhs_exp2(y);
}
#ifdef ORC_PRIMARY
double orc_vhs_pow(double x, double a) { return vhs_pow(x, a); }
#endif

/* ------------------------------------------------- VSS scattering */
/* Variable soft spheres (Koura & Matsumoto 1991; Bird 1994): the relative velocity g keeps its length and is deflected by chi with
 * cos chi = 2 B^(1/alpha) - 1, B uniform on (0, 1), about g at a uniform
 * azimuth eps; the centre-of-mass velocity is kept.  alpha = 1 is isotropic
 * scattering.  Both random numbers come from the collision's isotropic unit
 * vector n (the same one hard spheres use): B = (1 + n_z) / 2 is uniform
 * because n_z is, and (cos eps, sin eps) = (n_x, n_y) / |(n_x, n_y)|.  The
 * deflected vector is written in the frame of g with the two unit normals
 *   A = (h, -g_x g_y / h, -g_x g_z / h) / g  and  C = (0, g_z, -g_y) / h,
 *   h = sqrt(g_y^2 + g_z^2):  g' = g (cos chi g/g + sin chi (sin eps A + cos eps C))
 * (Bird's component formulas); when h = 0 the normals are the y and z axes.
 * Everything in double, in this order; the results are rounded to REAL. */
void FN(orc_scatter_vss)(REAL ci[3], REAL cj[3], const REAL n[3], double inv_alpha)
{
    double gx = (double)ci[0] - (double)cj[0];
    double gy = (double)ci[1] - (double)cj[1];
    double gz = (double)ci[2] - (double)cj[2];
    double g = sqrt((gx * gx + gy * gy) + gz * gz);
    /* deflection */
    double B = 0.5 * (1.0 + (double)n[2]);
    double cchi = 2.0 * vhs_pow(B, inv_alpha) - 1.0;
    double schi2 = 1.0 - cchi * cchi;
    double schi = schi2 > 0.0 ? sqrt(schi2) : 0.0;
    /* azimuth */
    double nx = (double)n[0], ny = (double)n[1];
    double rho2 = nx * nx + ny * ny;
    double ce = 1.0, se = 0.0;
    if (rho2 > 0.0) {
        double rho = sqrt(rho2);
        ce = nx / rho;
        se = ny / rho;
    }
    double h2 = gy * gy + gz * gz;
    double px, py, pz;
    if (h2 > 0.0) {
        double h = sqrt(h2);
        px = cchi * gx + (schi * se) * h;
        py = cchi * gy + schi * (((ce * g) * gz - (se * gx) * gy) / h);
        pz = cchi * gz - schi * (((ce * g) * gy + (se * gx) * gz) / h);
    } else {
        px = cchi * gx;
        py = (schi * ce) * g;
        pz = (schi * se) * g;
    }
    double pv[3] = {px, py, pz};
    for (int d = 0; d < 3; ++d) {
        double cm = 0.5 * ((double)ci[d] + (double)cj[d]);
        double t = 0.5 * pv[d];
        ci[d] = (REAL)(cm + t);
        cj[d] = (REAL)(cm - t);
    }
}

/* NTC collisions in one cell (Bird 1994), with the cell's particles listed in
 * canonical order (list[0..n-1]).  Candidate count
 * M = floor(1/2 N (N-1) F_N sigma g_max dt / V + U0); candidate k draws the
 * ordered pair (i, j) from block 0 of its PAIR stream and is accepted iff
 * (U g_max)^2 < g^2 (hard spheres; Maxwell molecules accept every candidate,
 * with sigma * g_max replaced by the constant sigma g = K; variable hard and
 * soft spheres accept with probability (g / g_max)^(2 - 2 omega)).  Candidates
 * are processed strictly in order k = 0, 1, ... */
static int collide_cell(const orc_cfg *cfg, soa_t *s, const int64_t *list, int64_t n,
                        uint32_t cell, uint32_t step, double V, uint64_t *cnt, orc_diag *diag,
                        int32_t *learned_flag)
{
    *learned_flag = 0;
    if (n < 2) return 0;
    double gmax;
    if (cfg->molecule == 1) {
        gmax = 1.0; /* unused by the Maxwell acceptance */
    } else if (cfg->majorant == 1 && cfg->mlp) {
        int used = 0;
        gmax = FN(orc_learned_majorant)(cfg, s->cx, s->cy, s->cz, list, n, V, &used);
        *learned_flag = used;
        if (used == 1) diag->learned_used++;
        else if (used == -1) diag->fallback++;
        else diag->learned_skip++;
    } else if (cfg->majorant == 2) {
        /* the true largest pair speed of the cell (brute force), with the same
         * rounding margin as the bound */
        double eps = IS_F32 ? 9.5367431640625e-07 : 8.8817841970012523e-16;
        gmax = FN(orc_diameter)(s->cx, s->cy, s->cz, list, n) * (1.0 + eps);
    } else {
        gmax = FN(orc_exact_bound)(s->cx, s->cy, s->cz, list, n);
    }
    if (cfg->vr && cfg->vr_kappa > 1.0 && cfg->molecule != 1) gmax = gmax * cfg->vr_kappa;
    double Mreal;
    if (cfg->molecule == 1)
        Mreal = (((((0.5 * (double)n) * (double)(n - 1)) * cfg->FN) * cfg->sigma) * cfg->dt) / V;
    else if (cfg->molecule >= 2)
        /* VHS and VSS: (sigma_T g)_max = sigma g_max^(2 - 2 omega) */
        Mreal = ((((((0.5 * (double)n) * (double)(n - 1)) * cfg->FN) * cfg->sigma) *
                  vhs_pow(gmax * gmax, 1.0 - cfg->omega)) * cfg->dt) / V;
    else
        Mreal = ((((((0.5 * (double)n) * (double)(n - 1)) * cfg->FN) * cfg->sigma) * gmax) * cfg->dt) / V;
    uint32_t r[4];
    draw(cfg->key, 0, TAG_NCAND, 0, cell, step, r);
    double U0 = u53(r[0], r[1]);
    double Mf = floor(Mreal + U0);
    if (!(Mf >= 0.0)) Mf = 0.0;
    if (Mf > 16777216.0) return ERR_CAPACITY; /* at most 2^24 candidates per cell and step */
    int64_t M = (int64_t)Mf;
    REAL gm = (REAL)gmax;
    uint64_t acc_count = 0;
    for (int64_t k = 0; k < M; ++k) {
        draw(cfg->key, (uint32_t)k, TAG_PAIR, 0, cell, step, r);
        uint32_t i = mulhi32(r[0], (uint32_t)n);
        uint32_t j = mulhi32(r[1], (uint32_t)(n - 1));
        if (j >= i) j++;
        int64_t pi = list[i], pj = list[j];
        REAL ci[3] = {s->cx[pi], s->cy[pi], s->cz[pi]};
        REAL cj[3] = {s->cx[pj], s->cy[pj], s->cz[pj]};
        REAL dx = ci[0] - cj[0], dy = ci[1] - cj[1], dz = ci[2] - cj[2];
        REAL g2 = (dx * dx + dy * dy) + dz * dz;
        int accept;
        double p;
        if (cfg->molecule == 1) {
            accept = 1;
            p = 1.0;
        } else if (cfg->molecule >= 2) {
            /* VHS, VSS: accept with probability (g / g_max)^(2 - 2 omega),
             * i.e. iff U < (g^2 / g_max^2)^(1 - omega), in double */
            double U = IS_F32 ? (double)u24(r[2]) : u53(r[2], r[3]);
            p = vhs_pow((double)g2 / (gmax * gmax), 1.0 - cfg->omega);
            accept = U < p;
            if (g2 > gm * gm) diag->overshoot++;
        } else {
            REAL U = IS_F32 ? (REAL)u24(r[2]) : (REAL)u53(r[2], r[3]);
            REAL a = U * gm;
            accept = (a * a) < g2;
            if (g2 > gm * gm) diag->overshoot++;
            p = sqrt((double)g2) / gmax;
        }
        if (cfg->vr) FN(orc_vr_update)(accept, p, &s->w[pi], &s->w[pj]);
        if (accept) {
            REAL nn[3];
            FN(orc_direction)(cfg->key, (uint32_t)k, cell, step, nn);
            if (cfg->molecule == 3)
                FN(orc_scatter_vss)(ci, cj, nn, 1.0 / cfg->alpha);
            else
                FN(orc_scatter)(ci, cj, g2, nn);
            s->cx[pi] = ci[0]; s->cy[pi] = ci[1]; s->cz[pi] = ci[2];
            s->cx[pj] = cj[0]; s->cy[pj] = cj[1]; s->cz[pj] = cj[2];
            acc_count++;
        }
    }
    cnt[0] += (uint64_t)M;
    cnt[1] += acc_count;
    return 0;
}

/* ------------------------------------------------ weight re-estimation */
/* Re-estimation of the importance weights of one cell (project reading of the
 * reconstruction step of Al-Mohssen & Hadjiconstantinou 2010; the weights
 * W ~ f_eq / f carry, besides that smooth ratio, a per-particle noise that
 * the collision update amplifies).  The deviations d_i = W_i - 1 are replaced
 * by their least-squares projection onto the 13 functions of the velocity
 * whose sums the cell samples, taken of v = c / sqrt(T0):
 *   phi(v) = (1, v_x, v_y, v_z, v_x^2, v_y^2, v_z^2, v_x v_y, v_x v_z, v_y v_z,
 *             v_x |v|^2, v_y |v|^2, v_z |v|^2),
 * i.e. d'_i = phi(v_i) . a with G a = b, G = sum_i phi(v_i) phi(v_i)^T and
 * b = sum_i d_i phi(v_i).  Then sum_i d'_i phi_k(v_i) = b_k: every sampled
 * weighted moment of the cell is unchanged, and d = 0 gives d' = 0 exactly
 * (unit weights stay exactly 1).  G is factorised by Cholesky (G = L L^T) and
 * the two triangular systems are solved in order; a cell with fewer than 26
 * particles, or with a pivot not above 1e-12 times its diagonal entry of G,
 * keeps its weights.  All in double; W'_i = 1 + d'_i rounded to REAL.
 * Returns 1 if the weights were replaced. */
#define NRB 13
static void recon_basis(double vx, double vy, double vz, double phi[NRB])
{
    double v2 = (vx * vx + vy * vy) + vz * vz;
    phi[0] = 1.0; phi[1] = vx; phi[2] = vy; phi[3] = vz;
    phi[4] = vx * vx; phi[5] = vy * vy; phi[6] = vz * vz;
    phi[7] = vx * vy; phi[8] = vx * vz; phi[9] = vy * vz;
    phi[10] = vx * v2; phi[11] = vy * v2; phi[12] = vz * v2;
}

int FN(orc_vr_reconstruct)(const REAL *cx, const REAL *cy, const REAL *cz, REAL *w, const int64_t *list,
                           int64_t n, double T0)
{
    if (n < 2 * NRB) return 0;
    double G[NRB][NRB], b[NRB], L[NRB][NRB], a[NRB], y[NRB], phi[NRB];
    memset(G, 0, sizeof(G));
    memset(b, 0, sizeof(b));
    memset(L, 0, sizeof(L));
    double sc = 1.0 / sqrt(T0);
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = list ? list[q] : q;
        recon_basis((double)cx[p] * sc, (double)cy[p] * sc, (double)cz[p] * sc, phi);
        double d = (double)w[p] - 1.0;
        for (int k = 0; k < NRB; ++k) {
            b[k] += d * phi[k];
            for (int l = 0; l <= k; ++l) G[k][l] += phi[k] * phi[l];
        }
    }
    /* Cholesky, column by column */
    for (int k = 0; k < NRB; ++k) {
        double piv = G[k][k];
        for (int j = 0; j < k; ++j) piv -= L[k][j] * L[k][j];
        if (!(piv > 1e-12 * G[k][k])) return 0;
        L[k][k] = sqrt(piv);
        for (int i = k + 1; i < NRB; ++i) {
            double t = G[i][k];
            for (int j = 0; j < k; ++j) t -= L[i][j] * L[k][j];
            L[i][k] = t / L[k][k];
        }
    }
    /* L y = b, then L^T a = y */
    for (int k = 0; k < NRB; ++k) {
        double t = b[k];
        for (int j = 0; j < k; ++j) t -= L[k][j] * y[j];
        y[k] = t / L[k][k];
    }
    for (int k = NRB - 1; k >= 0; --k) {
        double t = y[k];
        for (int j = k + 1; j < NRB; ++j) t -= L[j][k] * a[j];
        a[k] = t / L[k][k];
    }
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = list ? list[q] : q;
        recon_basis((double)cx[p] * sc, (double)cy[p] * sc, (double)cz[p] * sc, phi);
        double d = 0.0;
        for (int k = 0; k < NRB; ++k) d += a[k] * phi[k];
        w[p] = (REAL)(1.0 + d);
    }
    return 1;
}

/* Cell sampling (Bird 1994): raw FP64 sums S0 = N, S1 = sum c (3),
 * S2 = sum c_d c_e (xx, yy, zz, xy, xz, yz), S3 = sum c_d |c|^2 (3); with
 * variance reduction the same 13 sums weighted by (1 - W) follow. */
static int sample_cell(const orc_cfg *cfg, const soa_t *s, const int64_t *list, int64_t n, double *out)
{
    double L[NSUM];
    memset(L, 0, sizeof(L));
    for (int64_t a = 0; a < n; ++a) {
        int64_t p = list[a];
        double vx = (double)s->cx[p], vy = (double)s->cy[p], vz = (double)s->cz[p];
        double c2 = (vx * vx + vy * vy) + vz * vz;
        double q[13] = {1.0, vx, vy, vz, vx * vx, vy * vy, vz * vz, vx * vy, vx * vz, vy * vz,
                        vx * c2, vy * c2, vz * c2};
        for (int k = 0; k < 13; ++k) L[k] += q[k];
        if (cfg->vr) {
            double f = 1.0 - (double)s->w[p];
            for (int k = 0; k < 13; ++k) L[13 + k] += f * q[k];
        }
    }
    /* Non-finite plain sums mean the dynamics broke: an error.  The weighted
     * sums only carry the variance-reduced estimator, and weights never feed
     * back into the motion, so their divergence (the known growth of the
     * weight variance without reconstruction) is reported as a diagnostic. */
    int vr_bad = 0;
    for (int k = 0; k < NSUM; ++k) {
        if (!isfinite(L[k])) {
            if (k < 13) return ERR_NONFINITE;
            vr_bad = 1;
        }
        out[k] += L[k];
    }
    return vr_bad;
}

/* Group particles by cell in counting-sort fashion: the particles are taken
 * in the order of seq[0..np-1] (seq NULL: storage order) and each cell's
 * particles keep that relative order (a stable sort by cell).  Fills
 * start[0..ncell] and list[0..np-1]; cellp and count are scratch. */
static void stable_group(const orc_cfg *cfg, int64_t np, const REAL *x, const REAL *y, const int64_t *seq,
                         int64_t ncell, int64_t *cellp, int64_t *count, int64_t *start, int64_t *list)
{
    memset(count, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t p = 0; p < np; ++p) { cellp[p] = cell_of(cfg, x[p], cfg->dims == 2 ? y[p] : 0); count[cellp[p]]++; }
    start[0] = 0;
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] = start[c] + count[c];
    memset(count, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t k = 0; k < np; ++k) {
        int64_t p = seq ? seq[k] : k;
        int64_t c = cellp[p];
        list[start[c] + count[c]++] = p;
    }
}

/* The particle sequence before the first step (reading of the canonical
 * in-cell order): grouped by the cell of the initial position, cells in
 * ascending index, ascending particle id inside each cell. */
void FN(orc_initial_layout)(const orc_cfg *cfg, int64_t np, const REAL *x, const REAL *y, const uint32_t *id,
                            int64_t *layout)
{
    int64_t ncell = (int64_t)cfg->nx * (cfg->dims == 2 ? cfg->ny : 1);
    int64_t *count = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cellp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    stable_group(cfg, np, x, y, NULL, ncell, cellp, count, start, layout);
    g_sort_ids = id;
    for (int64_t c = 0; c < ncell; ++c)
        qsort(layout + start[c], (size_t)(start[c + 1] - start[c]), sizeof(int64_t), cmp_by_id);
    free(count); free(start); free(cellp);
}

/* Run nsteps time steps starting at step index step0.  Particle arrays are
 * modified in place (storage order is never changed).  sums[n_cells][26] and
 * counters[n_cells][2] (candidates, accepted) are accumulated.  Per step:
 * stream -> group -> collide -> (re-estimate the weights) -> sample.
 *
 * Walled runs (dims 1, 2) carry the particle sequence layout[0..np-1]
 * (indices into the arrays) from step to step: after streaming, the new
 * sequence is the stable grouping of the old one by new cell, and each
 * cell's particles are collided in that order (the canonical in-cell order).
 * The caller starts from orc_initial_layout. */
int FN(orc_run)(const orc_cfg *cfg, int64_t np, REAL *x, REAL *y, REAL *cx, REAL *cy, REAL *cz,
                REAL *w, const uint32_t *id, int64_t *layout, int64_t step0, int32_t nsteps, double *sums,
                uint64_t *counters, orc_diag *diag, int32_t *learned_log /* [nsteps][ncell] or NULL */)
{
    soa_t s = {x, y, cx, cy, cz, w, id};
    int64_t ncell = cfg->dims == 0 ? cfg->n_inst : (int64_t)cfg->nx * (cfg->dims == 2 ? cfg->ny : 1);
    int64_t *count = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int64_t *cellp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int rc = 0;
    double Vuni = cfg->dims == 2 ? (cfg->Lx / cfg->nx) * (cfg->Ly / cfg->ny)
                                 : (cfg->dims == 1 ? cfg->Lx / cfg->nx : 1.0);
    for (int32_t si = 0; si < nsteps && rc == 0; ++si) {
        uint32_t step = (uint32_t)(step0 + si);
        if (cfg->dims >= 1) {
            /* stream: each particle independently */
            for (int64_t p = 0; p < np && rc == 0; ++p) rc = stream_one(cfg, &s, p, step, diag);
            if (rc) break;
            /* group: stable counting sort of the current sequence by new cell */
            stable_group(cfg, np, x, y, layout, ncell, cellp, count, start, list);
            memcpy(layout, list, sizeof(int64_t) * (size_t)np);
        } else {
            /* homogeneous instances: contiguous ranges, storage order is canonical */
            for (int64_t c = 0; c <= ncell; ++c) start[c] = cfg->inst_offset[c];
            for (int64_t p = 0; p < np; ++p) list[p] = p;
        }
        int64_t next_only = 0;
        for (int64_t c = 0; c < ncell && rc == 0; ++c) {
            if (cfg->only_cells) {
                /* sampled-output mode: every particle streams, only the listed cells collide */
                if (next_only >= cfg->n_only || cfg->only_cells[next_only] != c) continue;
                next_only++;
            }
            int64_t n = start[c + 1] - start[c];
            double V = cfg->cell_volume ? cfg->cell_volume[c] : Vuni;
            int32_t lf = 0;
            uint32_t key_id = (cfg->dims == 0 && cfg->cell_ids) ? (uint32_t)cfg->cell_ids[c] : (uint32_t)c;
            rc = collide_cell(cfg, &s, list + start[c], n, key_id, step, V, &counters[2 * c], diag, &lf);
            if (learned_log) learned_log[(int64_t)si * ncell + c] = lf;
            if (rc == 0 && cfg->vr && cfg->vr_reconstruct > 0 && step % (uint32_t)cfg->vr_reconstruct == 0)
                FN(orc_vr_reconstruct)(cx, cy, cz, w, list + start[c], n, cfg->vr_T0);
            if (rc == 0) {
                rc = sample_cell(cfg, &s, list + start[c], n, &sums[NSUM * c]);
                if (rc == 1) { diag->vr_nonfinite++; rc = 0; }
            }
        }
    }
    free(count); free(start); free(list); free(cellp);
    if (rc) diag->error = rc;
    return rc;
}

/* Exported helpers for the pins: one candidate's pair draw. */
void FN(orc_pair)(const uint32_t key[2], uint32_t k, uint32_t cell, uint32_t step, uint32_t n,
                  uint32_t *i, uint32_t *j, REAL *U)
{
    uint32_t r[4];
    draw(key, k, TAG_PAIR, 0, cell, step, r);
    *i = mulhi32(r[0], n);
    uint32_t jj = mulhi32(r[1], n - 1);
    if (jj >= *i) jj++;
    *j = jj;
    *U = IS_F32 ? (REAL)u24(r[2]) : (REAL)u53(r[2], r[3]);
}

/* Exported helper: cell index of a position (pins of the grouping rule). */
int64_t FN(orc_cell_of)(const orc_cfg *cfg, REAL x, REAL y) { return cell_of(cfg, x, y); }
