/* Test driver: runs the CPU oracle on inputs written by a test, so that the
 * oracle can be built with AddressSanitizer and UndefinedBehaviorSanitizer
 * into a stand-alone executable (no instrumented Python needed).
 *
 * Test infrastructure only.  Compiled with -DREAL=double -DSFX=_f64 or
 * -DREAL=float -DSFX=_f32; includes the oracle source itself.
 *
 * Usage: oracle_driver DIR
 *   DIR/meta.txt   np nsteps step0 n_off has_volume has_mlp
 *   DIR/cfg.bin    the orc_cfg struct (its pointer fields are ignored)
 *   DIR/{x,y,cx,cy,cz,w}.bin  REAL[np];  DIR/id.bin  uint32[np]
 *   DIR/offset.bin int64[n_off] (homogeneous instances), DIR/volume.bin
 *   double[n_cells], DIR/mlp.bin float[4673]
 * Writes DIR/out_{x,y,cx,cy,cz,w}.bin, out_sums.bin (double[n_cells][26]),
 * out_counters.bin (uint64[n_cells][2]), out_diag.bin (orc_diag) and returns
 * the run's status (0 on success). */
#include "../../oracle/dsmc_oracle.c"

#include <stdio.h>

static void *read_file(const char *dir, const char *name, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void *buf = malloc(bytes > 0 ? bytes : 1);
    if (bytes > 0 && fread(buf, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return buf;
}

static void write_file(const char *dir, const char *name, const void *buf, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || (bytes > 0 && fwrite(buf, 1, bytes, f) != bytes)) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
    fclose(f);
}

int main(int argc, char **argv)
{
    if (argc != 2) { fprintf(stderr, "usage: %s DIR\n", argv[0]); return 2; }
    const char *dir = argv[1];
    long long np, step0, n_off;
    int nsteps, has_volume, has_mlp;
    {
        char path[4096];
        snprintf(path, sizeof path, "%s/meta.txt", dir);
        FILE *f = fopen(path, "r");
        if (!f || fscanf(f, "%lld %d %lld %lld %d %d", &np, &nsteps, &step0, &n_off, &has_volume, &has_mlp) != 6) {
            fprintf(stderr, "bad meta.txt\n");
            return 2;
        }
        fclose(f);
    }
    orc_cfg cfg;
    {
        orc_cfg *c = (orc_cfg *)read_file(dir, "cfg.bin", sizeof(orc_cfg));
        cfg = *c;
        free(c);
    }
    cfg.cell_volume = NULL;
    cfg.inst_offset = NULL;
    cfg.mlp = NULL;
    cfg.cell_ids = NULL;
    cfg.only_cells = NULL;
    cfg.n_only = 0;
    const size_t rb = sizeof(REAL) * (size_t)np;
    REAL *x = (REAL *)read_file(dir, "x.bin", rb), *y = (REAL *)read_file(dir, "y.bin", rb);
    REAL *cx = (REAL *)read_file(dir, "cx.bin", rb), *cy = (REAL *)read_file(dir, "cy.bin", rb);
    REAL *cz = (REAL *)read_file(dir, "cz.bin", rb), *w = (REAL *)read_file(dir, "w.bin", rb);
    uint32_t *id = (uint32_t *)read_file(dir, "id.bin", sizeof(uint32_t) * (size_t)np);
    int64_t *off = NULL;
    double *vol = NULL;
    float *mlp = NULL;
    if (cfg.dims == 0) {
        off = (int64_t *)read_file(dir, "offset.bin", sizeof(int64_t) * (size_t)n_off);
        cfg.inst_offset = off;
    }
    int64_t ncell = cfg.dims == 0 ? cfg.n_inst : (int64_t)cfg.nx * (cfg.dims == 2 ? cfg.ny : 1);
    if (has_volume) {
        vol = (double *)read_file(dir, "volume.bin", sizeof(double) * (size_t)ncell);
        cfg.cell_volume = vol;
    }
    if (has_mlp) {
        mlp = (float *)read_file(dir, "mlp.bin", sizeof(float) * MLP_NPARAM);
        cfg.mlp = mlp;
    }
    int64_t *layout = NULL;
    if (cfg.dims >= 1) {
        layout = (int64_t *)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
        FN(orc_initial_layout)(&cfg, np, x, y, id, layout);
    }
    double *sums = (double *)calloc((size_t)ncell * NSUM, sizeof(double));
    uint64_t *counters = (uint64_t *)calloc((size_t)ncell * 2, sizeof(uint64_t));
    orc_diag diag;
    memset(&diag, 0, sizeof diag);
    int rc = FN(orc_run)(&cfg, np, x, y, cx, cy, cz, w, id, layout, step0, nsteps, sums, counters, &diag, NULL);
    write_file(dir, "out_x.bin", x, rb);
    write_file(dir, "out_y.bin", y, rb);
    write_file(dir, "out_cx.bin", cx, rb);
    write_file(dir, "out_cy.bin", cy, rb);
    write_file(dir, "out_cz.bin", cz, rb);
    write_file(dir, "out_w.bin", w, rb);
    write_file(dir, "out_sums.bin", sums, sizeof(double) * (size_t)ncell * NSUM);
    write_file(dir, "out_counters.bin", counters, sizeof(uint64_t) * (size_t)ncell * 2);
    write_file(dir, "out_diag.bin", &diag, sizeof diag);
    free(x); free(y); free(cx); free(cy); free(cz); free(w); free(id);
    free(off); free(vol); free(mlp); free(layout); free(sums); free(counters);
    return rc == 0 ? 0 : 3;
}
