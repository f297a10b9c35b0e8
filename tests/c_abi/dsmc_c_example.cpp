// A caller of the library that uses only its C ABI (include/dsmc.h) and the
// HIP runtime: no Python, no torch.  It allocates every buffer itself, runs a
// small weighted lid-driven cavity and writes what it used and what it got,
// so that a test can check the run against the CPU oracle.
//
// Usage: dsmc_c_example OUTDIR
//   writes OUTDIR/init_{x,y,cx,cy,cz,w}.f64 and init_id.u32 (the initial
//   state), final_*.f64 / final_id.u32 (the state after the run, in the
//   library's particle sequence), sums.f64 [64][26], counters.u64 [64][2],
//   est.f64 [64][14] (dsmc_estimators, weighted) and meta.txt.
// Exit status 0 on success; the failing call is printed otherwise.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dsmc.h"

namespace {

constexpr int kNx = 8, kNy = 8, kPerCell = 24;
constexpr int kSteps = 12;
constexpr double kLid = 0.2;

// splitmix64 (Steele, Lea & Flood 2014): the example's own input generator
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
    double normal() {  // Box-Muller
        const double u1 = 1.0 - uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

bool write_file(const std::string &path, const void *data, size_t bytes) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(data, 1, bytes, f) == bytes;
    return std::fclose(f) == 0 && ok;
}

#define HIP_OK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));       \
            return 3;                                                                    \
        }                                                                                \
    } while (0)
#define DSMC_OK(call)                                                                    \
    do {                                                                                 \
        dsmc_status s_ = (call);                                                         \
        if (s_ != DSMC_OK) {                                                             \
            std::fprintf(stderr, "%s failed: %s\n", #call, dsmc_status_string(s_));      \
            return 4;                                                                    \
        }                                                                                \
    } while (0)

}  // namespace

int main(int argc, char **argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s OUTDIR\n", argv[0]);
        return 2;
    }
    const std::string out = argv[1];
    const int ncell = kNx * kNy;
    const int64_t n = (int64_t)ncell * kPerCell;

    // initial state: uniform positions, Maxwellian velocities at T = 1, unit weights
    std::vector<double> h[6];
    for (auto &v : h) v.resize((size_t)n);
    std::vector<uint32_t> id((size_t)n);
    SplitMix rng{20240601ull};
    for (int64_t p = 0; p < n; ++p) {
        h[0][p] = rng.uniform();
        h[1][p] = rng.uniform();
        h[2][p] = rng.normal();
        h[3][p] = rng.normal();
        h[4][p] = rng.normal();
        h[5][p] = 1.0;
        id[p] = (uint32_t)p;
    }
    const char *names[6] = {"x", "y", "cx", "cy", "cz", "w"};
    for (int k = 0; k < 6; ++k)
        if (!write_file(out + "/init_" + names[k] + ".f64", h[k].data(), h[k].size() * 8)) return 5;
    if (!write_file(out + "/init_id.u32", id.data(), id.size() * 4)) return 5;

    // configuration: unit square, diffuse walls at T = 1, lid (y+) moving along +x,
    // hard spheres at Kn 0.05, weights re-estimated every second step
    dsmc_config cfg;
    std::memset(&cfg, 0, sizeof cfg);
    cfg.abi_version = DSMC_ABI_VERSION;
    cfg.dims = 2;
    cfg.real_bytes = 8;
    cfg.molecule = DSMC_HARD_SPHERE;
    cfg.n_cells[0] = kNx;
    cfg.n_cells[1] = kNy;
    cfg.majorant = DSMC_MAJORANT_EXACT;
    cfg.vr = 1;
    cfg.length[0] = cfg.length[1] = 1.0;
    cfg.dt = 2e-3;
    cfg.sigma = 1.0 / (std::sqrt(2.0) * (double)n * 0.05);
    cfg.FN = 1.0;
    cfg.vr_T0 = 1.0;
    for (int k = 0; k < 4; ++k) {
        cfg.wall_kind[k] = DSMC_WALL_DIFFUSE;
        cfg.wall_T[k] = 1.0;
    }
    cfg.wall_u[3][0] = kLid;
    cfg.seed = 7;
    cfg.n_particles = n;
    cfg.vr_reconstruct = 2;
    cfg.vr_kappa = 1.5;

    size_t ws_bytes = 0;
    DSMC_OK(dsmc_workspace_size(&cfg, &ws_bytes));
    void *d[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    uint32_t *d_id = nullptr;
    void *ws = nullptr;
    for (int k = 0; k < 6; ++k) {
        HIP_OK(hipMalloc(&d[k], (size_t)n * 8));
        HIP_OK(hipMemcpy(d[k], h[k].data(), (size_t)n * 8, hipMemcpyHostToDevice));
    }
    HIP_OK(hipMalloc((void **)&d_id, (size_t)n * 4));
    HIP_OK(hipMemcpy(d_id, id.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMalloc(&ws, ws_bytes));
    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));

    dsmc_soa soa = {d[0], d[1], d[2], d[3], d[4], d[5], d_id};
    dsmc_ctx *ctx = nullptr;
    DSMC_OK(dsmc_init(&cfg, &soa, ws, ws_bytes, (void *)stream, &ctx));
    DSMC_OK(dsmc_step(ctx, kSteps));
    std::vector<double> sums((size_t)ncell * DSMC_NSUM);
    std::vector<uint64_t> counters((size_t)ncell * 2);
    uint64_t n_samples = 0;
    DSMC_OK(dsmc_sample(ctx, sums.data(), counters.data(), &n_samples, 0));
    std::vector<double> est((size_t)ncell * DSMC_NEST);
    DSMC_OK(dsmc_estimators(sums.data(), ncell, n_samples, cfg.FN, nullptr, 1.0 / ncell, 1, (double)n,
                            cfg.vr_T0, est.data()));
    dsmc_diag diag;
    DSMC_OK(dsmc_diagnostics(ctx, &diag));

    // the current state (the library alternates between buffers: ask where it is)
    dsmc_soa cur;
    DSMC_OK(dsmc_particles(ctx, &cur));
    void *src[6] = {cur.x, cur.y, cur.cx, cur.cy, cur.cz, cur.w};
    for (int k = 0; k < 6; ++k) {
        HIP_OK(hipMemcpy(h[k].data(), src[k], (size_t)n * 8, hipMemcpyDeviceToHost));
        if (!write_file(out + "/final_" + names[k] + ".f64", h[k].data(), h[k].size() * 8)) return 5;
    }
    HIP_OK(hipMemcpy(id.data(), cur.id, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (!write_file(out + "/final_id.u32", id.data(), id.size() * 4)) return 5;
    if (!write_file(out + "/sums.f64", sums.data(), sums.size() * 8)) return 5;
    if (!write_file(out + "/counters.u64", counters.data(), counters.size() * 8)) return 5;
    if (!write_file(out + "/est.f64", est.data(), est.size() * 8)) return 5;
    FILE *m = std::fopen((out + "/meta.txt").c_str(), "w");
    if (!m) return 5;
    std::fprintf(m, "n %lld steps %d samples %llu seed %llu dt %.17g sigma %.17g lid %.17g reest %d kappa %.17g "
                 "accepted %llu wall_hits %llu vr_nonfinite %llu\n",
                 (long long)n, kSteps, (unsigned long long)n_samples, (unsigned long long)cfg.seed, cfg.dt,
                 cfg.sigma, kLid, cfg.vr_reconstruct, cfg.vr_kappa, (unsigned long long)diag.accepted,
                 (unsigned long long)diag.wall_hits, (unsigned long long)diag.vr_nonfinite);
    std::fclose(m);

    DSMC_OK(dsmc_destroy(ctx));
    HIP_OK(hipStreamDestroy(stream));
    for (int k = 0; k < 6; ++k) HIP_OK(hipFree(d[k]));
    HIP_OK(hipFree(d_id));
    HIP_OK(hipFree(ws));
    return 0;
}
