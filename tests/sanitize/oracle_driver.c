/* AddressSanitizer / UndefinedBehaviorSanitizer run of the FP64 oracle (test
 * tooling): the oracle's two sources are compiled into this one translation
 * unit with the sanitizers on, and every entry point the tests use is driven
 * over small cases that reach each code path (water and CT grids, the block
 * with a concave opening, the range shifter, divergence and a virtual source,
 * batches, the LET numerator, traces, start-move allowances, slab and block
 * experiments, the network).  Exit status 0 with no sanitizer report; the energy balance of
 * every run is checked so the cases really transport. */
#include "../../oracle/vpmc_oracle.c"
#include "../../oracle/vpmc_mlp.c"

#include <stdio.h>

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            fails++;                                                       \
        }                                                                  \
    } while (0)


static void run_case(const orc_geom *g, orc_field *f, const orc_scen *sc, int physics, int batches)
{
    orc_spot sp[2] = {{0.0, 0.0, 150.0, 3.0, 0.5, 1.0, 600}, {6.0, -2.0, 120.0, 4.0, 0.0, 2.0, 400}};
    const int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    int64_t *q = calloc((size_t)nvox, sizeof *q), *qL = calloc((size_t)nvox, sizeof *qL);
    int64_t led[NLEDGER] = {0};
    orc_opts o = {12345u, 3, physics, 36, 0, batches};
    for (int b = 0; b < (batches > 1 ? batches : 1); b++) {
        o.batch = b;
        orc_run(g, f, sp, 0, 2, sc, &o, q, led, 2, qL);
    }
    /* the ledgers ([0] = the grid) hold the weighted energy put in, 1 x 150 +
     * 2 x 120 MeV (the first spot's 0.5 MeV spread averages out), and the
     * grid's ledger is the sum of its voxels */
    int64_t grid_sum = 0;
    double e = 0.0;
    for (int64_t i = 0; i < nvox; i++) grid_sum += q[i];
    for (int j = 0; j < NLEDGER; j++) e += ldexp((double)led[j], -o.k);
    CHECK(grid_sum == led[0]);
    CHECK(fabs(e - 390.0) < 0.5);
    double *grid = calloc((size_t)nvox, sizeof *grid), *glet = calloc((size_t)nvox, sizeof *glet), ledg[NLEDGER];
    int64_t info[4];
    const double mv[3] = {1e-3, -2e-3, 1e-4};
    orc_trace_history(g, f, &sp[0], 0, 7, sc, &o, ledg, grid, info, glet, mv);
    free(glet);
    /* start-move allowance: two histories, one and two moves, with LET */
    {
        const int32_t ms[2] = {0, 1};
        const int64_t mh[2] = {3, 11}, moff[3] = {0, 1, 3};
        const double moves[9] = {0.25, 0.0, 0.0, 0.0, -0.25, 0.0, 0.25, 0.25, 0.5};
        double *al = calloc((size_t)nvox, sizeof *al), *all = calloc((size_t)nvox, sizeof *all);
        orc_move_allowance(g, f, sp, sc, &o, 2, ms, mh, moff, moves, al, all, 2);
        double tot = 0.0;
        for (int64_t i = 0; i < nvox; i++) {
            CHECK(al[i] >= 0.0 && all[i] >= 0.0);
            tot += al[i];
        }
        CHECK(tot <= 2.0 * (150.0 / 600 + 2.0 * 120.0 / 400));
        free(al);
        free(all);
    }
    double *ex = malloc(8 * 50 * sizeof *ex);
    orc_patient_exit(g, f, &sp[1], 1, 50, sc, &o, ex, 2);
    free(ex);
    free(grid);
    free(q);
    free(qL);
}

int main(void)
{
    orc_init();
    /* water 40 x 36 x 90 at 1.5 mm, beam along +z, concave opening */
    orc_geom w = {0, 40, 36, 90, {1.5, 1.5, 1.5}, {-30.0, -27.0, 0.0}, NULL};
    double poly[2 * 6] = {-10, -10, 10, -10, 10, 10, 2, 10, 0, 2, -10, 10};
    orc_field f = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, 1, 6, poly, 30.0, 8.5, 50.0,
                   1, 38.85, 61.0, 90.0, 0.0, 0.0};
    orc_scen sc = {{0.5, -1.0, 2.0}, 1.035};
    run_case(&w, &f, &sc, 7, 4);
    run_case(&w, &f, &sc, 0, 1);
    f.vsad = 2000.0;
    f.focus = 1800.0;
    run_case(&w, &f, &sc, 7, 1);
    /* CT 32 x 30 x 40 at 2 mm: air, tissue, bone, beam along -x */
    orc_geom ct = {1, 32, 30, 40, {2.0, 2.0, 2.0}, {-32.0, -30.0, -40.0}, NULL};
    int16_t *hu = malloc(32 * 30 * 40 * sizeof *hu);
    for (int i = 0; i < 32 * 30 * 40; i++) hu[i] = (int16_t)((i * 7919) % 4000 - 1024);
    ct.hu = hu;
    orc_field g90 = {{0, 0, 0}, {0, -1, 0}, {0, 0, 1}, {-1, 0, 0}, 1, 6, poly, 30.0, 8.5, 150.0,
                     1, 38.85, 61.0, 190.0, 0.0, 0.0};
    orc_scen nom = {{0, 0, 0}, 1.0};
    run_case(&ct, &g90, &nom, 7, 2);
    g90.nv = 0;   /* closed block */
    run_case(&ct, &g90, &nom, 7, 1);

    /* thin slabs, block traversals, one traced block crossing */
    double *out = malloc(8 * 200 * sizeof *out);
    orc_slab_exit(3, 8.5, 3.0, 180.0, 7, 99u, 200, out, 2);
    free(out);
    double entries[5 * 20];
    for (int i = 0; i < 20; i++) {
        entries[5 * i + 0] = -12.0 + 1.2 * i;
        entries[5 * i + 1] = 0.3 * i - 3.0;
        entries[5 * i + 2] = 0.01 * (i % 3);
        entries[5 * i + 3] = -0.01 * (i % 2);
        entries[5 * i + 4] = 80.0 + 7.0 * i;
    }
    double *bt = malloc(20 * 16 * sizeof *bt);
    f.vsad = 0.0;
    f.focus = 0.0;
    orc_block_traverse(&f, entries, 20, 5u, 0, 7, bt, 2);
    free(bt);
    double p[3] = {9.9, 0.0, -80.0}, d[3] = {0.01, 0.0, 0.99995};
    double tr[64];
    orc_block_trace(&f, p, d, 170.0, 7, 3u, tr);
    CHECK(orc_in_polygon(poly, 6, 0.0, -5.0) == 1);
    CHECK(orc_in_polygon(poly, 6, 0.0, 8.0) == 0);

    /* network: forward, loss and gradient, Adam */
    const int np = mlp_num_params();
    double *prm = malloc((size_t)np * sizeof *prm), *grad = malloc((size_t)np * sizeof *grad);
    double *m = calloc((size_t)np, sizeof *m), *v = calloc((size_t)np, sizeof *v);
    for (int i = 0; i < np; i++) prm[i] = 0.01 * sin(0.1 * i);
    double x[4 * 8], y[4 * 3], tt[4] = {1, 0, 1, 1}, o29[4 * 29];
    for (int i = 0; i < 32; i++) x[i] = 0.1 * (i % 7) - 0.3;
    for (int i = 0; i < 12; i++) y[i] = 0.2 * (i % 5) - 0.4;
    mlp_forward(prm, x, 4, o29);
    double loss = mlp_loss_grad(prm, x, y, tt, 4, grad);
    CHECK(isfinite(loss));
    mlp_adam_step(prm, grad, m, v, np, 1, 1e-3, 0.9, 0.999, 1e-8);
    free(prm);
    free(grad);
    free(m);
    free(v);
    free(hu);
    if (fails) return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
