// AddressSanitizer / UndefinedBehaviorSanitizer run of the host runtime of
// libvpmc (test tooling): linked against a build of the library whose host
// code carries the sanitizers, it drives every entry point on a
// validation-only context (device -1: no GPU is touched), through the
// argument checks, the polygon validation and distance raster, the
// fixed-point and memory-cap checks, the CSR and cell-map scans, the
// optimiser's checks and the weights-file parser, and compares each return
// code with the documented one.  Exit status 0 with no sanitizer report.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../../include/vpmc.h"

static int fails = 0;
#define EXPECT(call, code)                                                                      \
    do {                                                                                        \
        const int rc_ = (call);                                                                 \
        if (rc_ != (code)) {                                                                    \
            fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, rc_, \
                    (code), vpmc_last_error(nullptr));                                          \
            fails++;                                                                            \
        }                                                                                       \
    } while (0)

static std::vector<float> circle(int n, float r) {
    std::vector<float> p(2 * n);
    for (int i = 0; i < n; ++i) {
        p[2 * i] = r * cosf(6.2831853f * (i + 0.5f) / n);
        p[2 * i + 1] = r * sinf(6.2831853f * (i + 0.5f) / n);
    }
    return p;
}

int main() {
    vpmc_ctx *c = nullptr;
    EXPECT(vpmc_create(&c, -1), VPMC_OK);
    EXPECT(vpmc_create(nullptr, 0), VPMC_E_ARG);
    double tab[256];
    for (int m = 0; m < 5; ++m)
        for (int w = 0; w < 5; ++w) EXPECT(vpmc_table_host(m, w, tab, 256), 256);

    // geometry: water and CT (shape kept on a validation-only context)
    const float sp[3] = {1.0f, 1.0f, 2.0f}, org[3] = {-32.0f, -32.0f, -40.0f};
    std::vector<int16_t> hu(64 * 64 * 40);
    for (size_t i = 0; i < hu.size(); ++i) hu[i] = (int16_t)((i * 7919) % 4000 - 1024);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_HU, hu.data(), 64, 64, 40, sp, org, 0), VPMC_OK);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_HU, nullptr, 64, 64, 40, sp, org, 0), VPMC_E_ARG);
    EXPECT(vpmc_load_geometry(c, 5, nullptr, 64, 64, 40, sp, org, 0), VPMC_E_ARG);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_WATER, nullptr, 2048, 1024, 1024, sp, org, 0), VPMC_E_ARG);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_WATER, nullptr, 100, 100, 100, sp, org, 0), VPMC_OK);

    // fields: circle with range shifter, concave opening, closed block, errors
    vpmc_beam beam = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    vpmc_block blk = {30.0f, 8.5f, 50.0f};
    vpmc_rs rs = {45.0f, 61.0f, 90.0f};
    std::vector<float> circ = circle(256, 10.0f);
    EXPECT(vpmc_set_aperture(c, 0, &beam, circ.data(), 256, &blk, &rs), VPMC_OK);
    const float concave[12] = {-10, -10, 10, -10, 10, 10, 2, 10, 0, 2, -10, 10};
    EXPECT(vpmc_set_aperture(c, 1, &beam, concave, 6, &blk, nullptr), VPMC_OK);
    EXPECT(vpmc_set_aperture(c, 2, &beam, nullptr, 0, &blk, nullptr), VPMC_OK);
    EXPECT(vpmc_set_aperture(c, 3, &beam, nullptr, 0, nullptr, nullptr), VPMC_OK);
    const float bowtie[8] = {0, 0, 1, 1, 1, 0, 0, 1};
    EXPECT(vpmc_set_aperture(c, 4, &beam, bowtie, 4, &blk, nullptr), VPMC_E_POLYGON);
    std::vector<float> big = circle(1025, 10.0f);
    EXPECT(vpmc_set_aperture(c, 4, &beam, big.data(), 1025, &blk, nullptr), VPMC_E_POLYGON);
    EXPECT(vpmc_set_aperture(c, 64, &beam, circ.data(), 256, &blk, nullptr), VPMC_E_ARG);
    EXPECT(vpmc_set_divergence(c, 0, 2000.0f, 1800.0f), VPMC_OK);
    EXPECT(vpmc_set_divergence(c, 0, 100.0f, 0.0f), VPMC_E_ARG);
    EXPECT(vpmc_set_divergence(c, 3, 0.0f, 500.0f), VPMC_E_ARG);
    EXPECT(vpmc_set_divergence(c, 9, 0.0f, 0.0f), VPMC_E_STATE);

    // runs: every check before the device, then the missing device
    vpmc_spot spots[3] = {{0, 0, 150.0f, 3.0f, 0.0f, 1.0f, 1000},
                          {2.5f, 0, 140.0f, 3.2f, 0.5f, 2.0f, 500},
                          {0, 2.5f, 130.0f, 3.4f, 0.0f, 1.0f, 800}};
    vpmc_scenario scen[2] = {{{0, 0, 0}, 1.0f}, {{3.0f, 0, 0}, 1.035f}};
    vpmc_opts o{};
    o.physics = VPMC_PHYS_ALL;
    std::vector<float> dose(1);
    std::vector<int64_t> rp(7);
    EXPECT(vpmc_run_spots(c, 0, spots, 3, scen, 2, &o, dose.data(), nullptr, nullptr, nullptr), VPMC_E_STATE);
    o.n_batches = 16;
    o.max_device_bytes = 4u << 20;
    EXPECT(vpmc_run_spots(c, 0, spots, 3, scen, 2, &o, dose.data(), dose.data(), nullptr, nullptr), VPMC_E_OOM);
    o.max_device_bytes = 0;
    o.fixed_point_bits = 62;
    EXPECT(vpmc_run_spots(c, 0, spots, 3, scen, 2, &o, dose.data(), nullptr, nullptr, nullptr), VPMC_E_RANGE);
    o.fixed_point_bits = 0;
    vpmc_spot hot = spots[0];
    hot.energy_mev = 300.0f;
    EXPECT(vpmc_run_spots(c, 0, &hot, 1, scen, 1, &o, dose.data(), nullptr, nullptr, nullptr), VPMC_E_RANGE);
    o.output = VPMC_OUT_CSR;
    o.n_batches = 0;
    EXPECT(vpmc_run_spots(c, 1, spots, 3, scen, 2, &o, nullptr, nullptr, nullptr, rp.data()), VPMC_E_STATE);
    const int ids[2] = {0, 1};
    const vpmc_spot *sps[2] = {spots, spots};
    const int ns[2] = {3, 3};
    std::vector<int64_t> rpb(13);
    EXPECT(vpmc_run_batched(c, ids, sps, ns, 2, scen, 2, &o, nullptr, nullptr, rpb.data()), VPMC_E_STATE);
    const int dup[2] = {1, 1};
    EXPECT(vpmc_run_batched(c, dup, sps, ns, 2, scen, 2, &o, nullptr, nullptr, rpb.data()), VPMC_E_ARG);
    o.max_device_bytes = 1u << 20;
    EXPECT(vpmc_run_batched(c, ids, sps, ns, 2, scen, 2, &o, nullptr, nullptr, rpb.data()), VPMC_E_OOM);
    o.max_device_bytes = 0;
    vpmc_opts best{};
    EXPECT(vpmc_autotune(c, 0, spots, 3, scen, &o, 100000, &best), VPMC_E_STATE);
    o.output = VPMC_OUT_DOSE;
    o.flags = VPMC_DEVICE_PTRS;
    EXPECT(vpmc_run_spots_noalloc(c, 0, spots, 3, scen, 2, &o, dose.data(), nullptr, nullptr), VPMC_E_STATE);
    o.n_batches = 16;   // 1e6 voxels x 24 B fit in the 32 MiB scratch
    EXPECT(vpmc_run_spots_noalloc(c, 0, spots, 3, scen, 2, &o, dose.data(), dose.data(), nullptr), VPMC_E_STATE);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_WATER, nullptr, 128, 128, 100, sp, org, 0), VPMC_OK);
    EXPECT(vpmc_run_spots_noalloc(c, 0, spots, 3, scen, 2, &o, dose.data(), dose.data(), nullptr), VPMC_E_OOM);
    EXPECT(vpmc_load_geometry(c, VPMC_GEOM_WATER, nullptr, 100, 100, 100, sp, org, 0), VPMC_OK);
    o.flags = 0;
    EXPECT(vpmc_run_spots_noalloc(c, 0, spots, 3, scen, 2, &o, dose.data(), nullptr, nullptr), VPMC_E_ARG);

    // influence-matrix consumers: the optimiser's and the cell merge's scans
    const int nvox = 100 * 100 * 100;
    std::vector<int64_t> orp = {0, 3, 5, 9};
    std::vector<int32_t> col = {1, 5, 9, 2, 7, 0, 3, 4, 999999};
    std::vector<float> val = {1, 2, 3, 4, 5, 6, 7, 8, 9};
    std::vector<uint8_t> roi(nvox, 0);
    roi[5] = 1;
    roi[7] = 2;
    std::vector<double> x(3, 1.0);
    vpmc_opt_params p{};
    p.d_presc = 2.0;
    p.w_target = 1.0;
    p.d_max = 1.0;
    p.w_oar = 1.0;
    p.iters = 10;
    p.n_power = 5;
    EXPECT(vpmc_optimize(c, orp.data(), col.data(), val.data(), 1, 3, nvox, roi.data(), &p, x.data(), nullptr, nullptr,
                         nullptr), VPMC_E_STATE);
    col[8] = nvox;   // out of range
    EXPECT(vpmc_optimize(c, orp.data(), col.data(), val.data(), 1, 3, nvox, roi.data(), &p, x.data(), nullptr, nullptr,
                         nullptr), VPMC_E_ARG);
    col[8] = 4;
    orp[2] = 2;   // decreasing
    EXPECT(vpmc_optimize(c, orp.data(), col.data(), val.data(), 1, 3, nvox, roi.data(), &p, x.data(), nullptr, nullptr,
                         nullptr), VPMC_E_ARG);
    orp[2] = 5;
    std::vector<int32_t> cells(nvox);
    for (int v = 0; v < nvox; ++v) cells[v] = v / 4;
    std::vector<int64_t> q(9, 1), rpo(4);
    std::vector<int32_t> ccol = {1, 5, 9, 2, 7, 0, 3, 4, 8};
    EXPECT(vpmc_csr_cells(c, orp.data(), 3, ccol.data(), q.data(), 30, cells.data(), nvox / 4, rpo.data(), nullptr,
                          nullptr, nullptr, 0), VPMC_E_STATE);
    cells[17] = 9;   // jumps by more than one
    EXPECT(vpmc_csr_cells(c, orp.data(), 3, ccol.data(), q.data(), 30, cells.data(), nvox / 4, rpo.data(), nullptr,
                          nullptr, nullptr, 0), VPMC_E_ARG);

    // the surrogate's configuration and weights file
    EXPECT(vpmc_surrogate_config(c, 3.0f, 0.02f, 0.98f), VPMC_OK);
    EXPECT(vpmc_surrogate_config(c, -1.0f, 0.02f, 0.98f), VPMC_E_ARG);
    EXPECT(vpmc_surrogate_load(c, nullptr), VPMC_OK);
    EXPECT(vpmc_surrogate_load(c, "/nonexistent/dir/w.bin"), VPMC_E_ARG);
    const char *tmp = getenv("VPMC_SANITIZE_TMP");
    if (tmp) {
        char path[1024];
        snprintf(path, sizeof path, "%s/w.bin", tmp);
        FILE *fp = fopen(path, "wb");
        const int np = vpmc_surrogate_param_count();
        const uint32_t n = (uint32_t)np;
        std::vector<float> w(np, 0.0f);
        fwrite("VPMCMLP1", 1, 8, fp);
        fwrite(&n, 4, 1, fp);
        fwrite(w.data(), 4, np - 1, fp);   // one parameter short
        fclose(fp);
        EXPECT(vpmc_surrogate_load(c, path), VPMC_E_ARG);
        fp = fopen(path, "ab");
        fwrite(w.data(), 4, 1, fp);
        fclose(fp);
        EXPECT(vpmc_surrogate_load(c, path), VPMC_E_STATE);   // well formed; no device to hold it
    }
    std::vector<float> xin(8 * 4, 0.0f), out(29 * 4);
    EXPECT(vpmc_surrogate_forward(c, xin.data(), 4, out.data()), VPMC_E_STATE);
    vpmc_destroy(c);
    if (fails) return 1;
    printf("host runtime sanitizer run: ok\n");
    return 0;
}
