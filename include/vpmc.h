/*
 * vpmc.h -- C ABI of the MI355X (gfx950) virtual-particle Monte Carlo
 * transport of proton pencil beams through an optional range shifter and a
 * patient-specific brass aperture block into a voxelised water or CT
 * geometry, with int64 fixed-point dose tallies and per-spot sparse
 * influence matrices.
 *
 * Paper: Feng et al., "Modelling small block aperture in an in-house
 * developed GPU-accelerated Monte Carlo-based dose engine for pencil beam
 * scanning proton therapy", arXiv 2307.01416.  Section references below are
 * to that paper.
 *
 * Conventions
 *  - Every function returns int: VPMC_OK (0) or a negative error code.  On
 *    error the outputs are left untouched and the context stays usable;
 *    vpmc_last_error() returns a thread-local message owned by the library.
 *  - Units: mm, MeV, g/cm^3.  Voxel (i,j,k) covers [origin + i*d,
 *    origin + (i+1)*d) per axis; x is fastest in memory (index
 *    i + nx*(j + ny*k)).
 *  - Inputs are borrowed for the duration of the call; host inputs are copied
 *    before the call returns.
 *  - Outputs are caller-owned.  With VPMC_DEVICE_PTRS in the flags they are
 *    device pointers on the context's GPU (for instance torch tensors) and
 *    all work is ordered on opts->hip_stream; otherwise they are host
 *    pointers and the call returns after the copy.
 *  - Argument validation is done on the host before any HIP call.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef VPMC_H
#define VPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VPMC_OK 0
#define VPMC_E_ARG -1      /* invalid argument */
#define VPMC_E_STATE -2    /* call out of order (no geometry, no field, no device) */
#define VPMC_E_POLYGON -3  /* aperture polygon degenerate or self-intersecting */
#define VPMC_E_OOM -4      /* device memory (or opts.max_device_bytes) exhausted */
#define VPMC_E_DEVICE -5   /* HIP runtime error */
#define VPMC_E_RANGE -6    /* energy outside the tables or fixed-point overflow bound */
#define VPMC_E_ABORTED -7  /* work-queue iteration cap (vpmc_opts.queue_cap) reached */

/* physics switches (0 = straight CSDA transport) */
#define VPMC_STRAGGLE 1u
#define VPMC_MCS 2u
#define VPMC_NUCLEAR 4u
#define VPMC_PHYS_ALL 7u

#define VPMC_GEOM_WATER 0  /* homogeneous water, density 1 */
#define VPMC_GEOM_HU 1     /* int16 CT numbers, calibrated to material and density */

#define VPMC_OUT_DOSE 0    /* dense dose grid per scenario */
#define VPMC_OUT_CSR 1     /* per-(scenario, spot) sparse influence-matrix rows */

#define VPMC_DEVICE_PTRS 1u /* pointers are device pointers; work on opts.hip_stream */
#define VPMC_GRAPH 2u       /* CSR: capture all epochs of the run in one hipGraph */
#define VPMC_SURROGATE 4u   /* VPs entering the brass far from the opening's edge cross it
                               by the learned surrogate (weights must be set; dense and
                               eager CSR runs, not with VPMC_GRAPH) */
#define VPMC_LET 8u         /* dense dose: also tally the numerator of the dose-averaged LET
                               (vpmc_last_let); rejected with CSR output */

#define VPMC_MAX_FIELDS 64
#define VPMC_MAX_VERTICES 1024
#define VPMC_NLEDGER 6     /* [0] patient grid [1] range shifter [2] aperture block
                              [3] escaped / missed the grid [4] nuclear, carried away [5] spare */

typedef struct vpmc_ctx vpmc_ctx;

/* Create a context on HIP device `hip_device`.  hip_device == -1 creates a
 * validation-only context (no GPU is touched; run calls return
 * VPMC_E_STATE after validating their arguments).  The physics tables
 * (Methods A: per-material tables X(E) of energy loss, straggling,
 * deflection and interaction probability) are generated in FP64 on the host
 * and staged to the device in FP32. */
int vpmc_create(vpmc_ctx **out, int hip_device);
void vpmc_destroy(vpmc_ctx *ctx);
const char *vpmc_last_error(const vpmc_ctx *ctx);
int vpmc_version(void);

/* Load the patient or phantom voxel grid (Methods D.2 water phantoms, D.3
 * CT geometries).  kind VPMC_GEOM_WATER ignores hu (may be NULL);
 * VPMC_GEOM_HU copies nx*ny*nz int16 CT numbers (host pointer, or device
 * pointer with VPMC_DEVICE_PTRS).  nx*ny*nz must be < 2^31.  On a
 * validation-only context only the grid's shape is kept (for the checks of
 * later calls) and hu is not read. */
int vpmc_load_geometry(vpmc_ctx *ctx, int kind, const int16_t *hu, int nx, int ny, int nz,
                       const float spacing_mm[3], const float origin_mm[3], unsigned flags);

/* Beam frame of a field: origin `iso_mm` in CT coordinates; ex, ey, ez are
 * the beam-frame axes as CT-frame unit vectors (right-handed, orthonormal);
 * the beam travels along +ez and beam-line components sit at negative z. */
typedef struct {
    float iso_mm[3];
    float ex[3], ey[3], ez[3];
} vpmc_beam;

/* Aperture block (Methods B): brass slab of the given thickness and
 * density whose downstream face lies downstream_mm upstream of the
 * beam-frame origin plane; non-divergent opening (Methods D) unless
 * vpmc_set_divergence gives a focus. */
typedef struct {
    float thickness_mm, density_gcc, downstream_mm;
} vpmc_block;

/* Range shifter (Methods B): PMMA disc of the given water-equivalent
 * thickness and diameter, downstream face downstream_mm upstream of the
 * beam-frame origin plane.  Must lie upstream of the block. */
typedef struct {
    float wet_mm, diameter_mm, downstream_mm;
} vpmc_rs;

/* Define field `field_id`: its beam frame, its aperture and its range
 * shifter (Methods B).  xy_mm holds n_vertices (x, y) pairs of the opening
 * in the beam's-eye view (implicitly closed, either orientation, must not
 * self-intersect); the crossing-number test decides opening vs brass.
 * block == NULL: no aperture block.  block != NULL and n_vertices == 0:
 * closed block (no opening).  rs == NULL: no range shifter.
 * Errors: VPMC_E_ARG (bad numbers, field id), VPMC_E_POLYGON (fewer than 3
 * vertices but not 0, zero area, self-intersection, > VPMC_MAX_VERTICES). */
int vpmc_set_aperture(vpmc_ctx *ctx, int field_id, const vpmc_beam *beam, const float *xy_mm,
                      int n_vertices, const vpmc_block *block, const vpmc_rs *rs);

/* Divergence of field `field_id` (the divergent block is the paper's next
 * step, Discussion; this library's addition, not the paper's validated
 * geometry).  vsad_mm > 0: every VP's ray passes through a virtual source
 * vsad_mm upstream of the beam-frame origin plane (a spot's position is then
 * its central ray's crossing of that plane); 0: parallel beam.
 * focus_mm > 0: divergent block, every wall is the plane through the point
 * focus_mm upstream of the origin plane and an edge of the polygon, which
 * then describes the opening on the block's downstream face (at depth z the
 * opening is the polygon scaled by (z + focus) / (focus - downstream_mm)); 0:
 * non-divergent block.  VPs entering a divergent block are never handed to
 * the learned surrogate.  vpmc_set_aperture resets both to 0.  Errors:
 * VPMC_E_STATE (field not set), VPMC_E_ARG (negative or non-finite values,
 * a virtual source not upstream of every beam-line component, a focus without
 * a block or not upstream of the block). */
int vpmc_set_divergence(vpmc_ctx *ctx, int field_id, float vsad_mm, float focus_mm);

/* One pencil-beam spot (Methods D.1/D.2): position at the beam-frame origin
 * plane, energy, Gaussian in-air sigma, optional Gaussian energy spread,
 * weight and number of virtual particles (histories). */
typedef struct {
    float x_mm, y_mm, energy_mev, sigma_mm, energy_sigma_mev, weight;
    uint32_t n_histories;
} vpmc_spot;

/* Robust scenario (Methods E): the patient is displaced by shift_mm and
 * every stopping power in the patient is multiplied by range_scale. */
typedef struct {
    float shift_mm[3];
    float range_scale;
} vpmc_scenario;

typedef struct {
    uint64_t seed;          /* Philox key; one stream per (field, spot, history) */
    unsigned physics;       /* VPMC_STRAGGLE | VPMC_MCS | VPMC_NUCLEAR, 0 = straight */
    int n_batches;          /* 0/1: no variance; 2..1024: history h goes to batch h mod B */
    int output;             /* VPMC_OUT_DOSE or VPMC_OUT_CSR */
    int fixed_point_bits;   /* 0: automatic; else k in [1, 62] */
    unsigned flags;         /* VPMC_DEVICE_PTRS */
    void *hip_stream;       /* hipStream_t or NULL (default stream) */
    size_t max_device_bytes;/* 0 = no cap; scratch above the cap -> VPMC_E_OOM */
    int block_threads;      /* 0 = tuned default; else 256 or 512, for CSR output also 768 or 1024
                               (the CSR queue runs at most 1024 threads in physics mode, 768 in
                               straight mode, and its LDS tile shrinks with the workgroup) */
    int grid_blocks;        /* 0 = tuned default */
    int hist_per_lane;      /* CSR work-queue chunk = 64 * hist_per_lane histories; 0 = default 4 */
    int max_slots;          /* CSR rows resident at once (<= 1024); 0 = sized from memory */
    uint64_t queue_cap;     /* CSR work queue: iterations (chunks drawn, row picks, waits) a
                               wavefront may make before it gives up and the run returns
                               VPMC_E_ABORTED with no rows written; 0 = 2^40 (no practical cap) */
} vpmc_opts;

/* Transport all histories of n_spots spots of field `field_id` for each of
 * n_scen scenarios.  Energy deposits are tallied as q = rne(dE * w_s/N_s *
 * 2^k) in int64 (order-independent, so reruns are bit-identical).
 * Dense mode (opts->output == VPMC_OUT_DOSE):
 *   dose_gy   [n_scen][nvox] FP32 dose to medium, Gy per unit spot weight
 *   sigma_gy  [n_scen][nvox] FP32 standard error (needs n_batches >= 2) or NULL
 *   ledger_mev[n_scen][6]    FP64 energy balance (weighted MeV) or NULL; always
 *                            host memory
 * CSR mode: row_ptr [n_scen*n_spots + 1] (row = scen*n_spots + spot) is
 *   filled; the total number of non-zeros is row_ptr[n_scen*n_spots]; then
 *   call vpmc_copy_csr.  dose_gy/sigma_gy may be NULL.
 * Errors: VPMC_E_STATE (no geometry/field), VPMC_E_ARG, VPMC_E_RANGE
 * (energy outside (1, 256] MeV or k too small), VPMC_E_OOM (the run's device
 * scratch exceeds opts->max_device_bytes: checked before any HIP call for the
 * dense grids and one CSR row slot, then by the allocator), VPMC_E_DEVICE,
 * VPMC_E_ABORTED (CSR: opts->queue_cap reached). */
int vpmc_run_spots(vpmc_ctx *ctx, int field_id, const vpmc_spot *spots, int n_spots,
                   const vpmc_scenario *scen, int n_scen, const vpmc_opts *opts, float *dose_gy,
                   float *sigma_gy, double *ledger_mev, int64_t *row_ptr);

/* Allocation-free dense run, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same transport, batches and dose conversion as a dense
 * vpmc_run_spots with the same arguments, with the same bits out; every
 * intermediate (ledgers, counters, spot records, batch offsets, the int64
 * tally and, with n_batches >= 2, the batch tally and the FP64 sum of
 * squares) lives in one static device array of 32 MiB per GPU, which the
 * library holds until the process ends.  It calls no hipMalloc or hipFree.
 *   opts->output must be VPMC_OUT_DOSE and opts->flags exactly
 *   VPMC_DEVICE_PTRS: dose_gy [n_scen][nvox] and sigma_gy (needs
 *   n_batches >= 2) are device pointers, either may be NULL; ledger_mev
 *   [n_scen][6] is host memory or NULL.  With ledger_mev the call returns
 *   after the work is done; without it the work is left queued on
 *   opts->hip_stream.  opts->max_device_bytes is ignored.
 *   Size limit: 8 B per voxel (24 B with batches) + 28 B per spot + 8 B per
 *   spot and batch + 48 B per scenario, each piece rounded up to 256 B,
 *   must fit in 32 MiB: about 4.1e6 voxels without batches, 1.39e6 with.
 * The array keeps the last call's contents (each call clears what it needs);
 * calls that overlap on one GPU, from any context or stream, race on it.
 * vpmc_last_tally, vpmc_last_let and vpmc_last_stats keep describing the
 * last vpmc_run_spots / vpmc_run_batched call.
 * Errors: as vpmc_run_spots; VPMC_E_ARG for CSR output or any flag other
 * than VPMC_DEVICE_PTRS; VPMC_E_OOM if the run does not fit in the scratch
 * (outputs untouched). */
int vpmc_run_spots_noalloc(vpmc_ctx *ctx, int field_id, const vpmc_spot *spots, int n_spots,
                           const vpmc_scenario *scen, int n_scen, const vpmc_opts *opts, float *dose_gy,
                           float *sigma_gy, double *ledger_mev);

/* All robust scenarios x fields x spots in one work-queue pass (Methods C
 * and E: influence matrices of every scenario for robust optimisation).
 * Rows are ordered (scenario, field in the order given, spot); spots[f] holds
 * n_spots[f] spots of field field_ids[f] (set by vpmc_set_aperture).  The
 * output is always CSR: row_ptr [n_scen * sum(n_spots) + 1] (pointer kind per
 * flags), then vpmc_copy_csr.  dose_gy [n_scen][nvox] (optional) receives the
 * plan dose of each scenario (sum of its rows); ledger_mev [n_scen][6] host.
 * Each row equals, bitwise, the tally of the same spot run alone with the
 * same seed and fixed_point_bits (streams are keyed by field, spot, history).
 * Errors: as vpmc_run_spots; VPMC_E_ARG if the fields' vertices exceed
 * VPMC_MAX_VERTICES in total. */
int vpmc_run_batched(vpmc_ctx *ctx, const int *field_ids, const vpmc_spot *const *spots,
                     const int *n_spots, int n_fields, const vpmc_scenario *scen, int n_scen,
                     const vpmc_opts *opts, float *dose_gy, double *ledger_mev, int64_t *row_ptr);

/* Autotuner: for the launch shape only (never for results: tallies are
 * integers and streams are keyed by history, so every shape gives the same
 * bits).  Runs a bounded sample of the given spots (every s-th spot with its
 * own history count, s chosen so that the sample holds about
 * sample_histories VPs) in the output mode of *base for each candidate
 * shape (each timed twice, the faster time counting), keeps the one with
 * the shortest transport time per history, writes it into *best (a copy of
 * *base with hist_per_lane, grid_blocks and block_threads filled) and
 * remembers it for later runs on this context whose opts leave them at 0;
 * in CSR mode hist_per_lane is also remembered for field_id, and each epoch
 * of a batched run takes the value of the field that holds most of its rows
 * (the best chunk size depends on the beam direction).
 * Candidates (CSR): hist_per_lane in {1,2,3,4,6,8} x workgroups of 1024 or
 * 512 threads (768 or 512
 * in straight mode), as many as fill every CU at its full wave occupancy;
 * (dense): {4,8,16,32} x CUs x 256 threads of work per launch in workgroups of
 * 256 or 512 threads. */
int vpmc_autotune(vpmc_ctx *ctx, int field_id, const vpmc_spot *spots, int n_spots,
                  const vpmc_scenario *scen, const vpmc_opts *base, uint64_t sample_histories,
                  vpmc_opts *best);

/* ---------------------------------------------------------------------------
 * Learned aperture surrogate: a multilayer perceptron 8 -> 4 x 256 (SiLU) ->
 * 29 run by BF16 matrix-core kernels with FP32 accumulation.  Inputs (one row
 * per VP entering the block): normalised entry x, y, direction cosines u, v,
 * energy, distance to the opening's edge, block thickness, material id.
 * Outputs: [0] transmission logit, [1..4] mixture-weight logits, [5..16]
 * means and [17..28] log standard deviations (3 per component) of the
 * normalised outgoing energy loss, deflection angle and lateral offset.  It is
 * trained on traversals produced by the plain brass transport (Methods B),
 * which stays the fallback near the opening's edge.  Parameters are FP32,
 * layer by layer as W[out][in] then b[out].  All pointers are host memory.
 * ------------------------------------------------------------------------- */
int vpmc_surrogate_param_count(void);
/* Training data from the plain transport: entries [n][5] = (x, y) on the
 * upstream face of field_id's block (BEV, mm), direction cosines (u, v),
 * energy (MeV); each crosses the block with the plain brass transport
 * (seeded streams, `physics` as in vpmc_opts).  Writes the network inputs
 * x [n][8] = (x/20, y/20, u/0.05, v/0.05, (E-150)/50, min(d_edge,100)/10,
 * thickness/30, material 0), targets y [n][3] = ((dE/E - 0.5)/0.25,
 * angle/0.05 rad, offset/2 mm) and trans[n] = 1 transmitted, 0 stopped or
 * lost, -1 entered through the opening (no brass traversal). */
int vpmc_surrogate_sample(vpmc_ctx *ctx, int field_id, const float *entries, int n, uint64_t seed,
                          unsigned physics, float *x, float *y, float *trans);
int vpmc_surrogate_set_weights(vpmc_ctx *ctx, const float *params, int n_params);
int vpmc_surrogate_get_weights(vpmc_ctx *ctx, float *params, int n_params);
/* Weights by file (little-endian): the 8 bytes "VPMCMLP1", a uint32
 * parameter count, then the FP32 parameters in the layout above.
 * vpmc_surrogate_load(ctx, NULL) disables the network (runs with
 * VPMC_SURROGATE then fail with VPMC_E_STATE until weights are set again).
 * Errors: VPMC_E_ARG (unreadable or malformed file, wrong count, a value not
 * finite, unwritable path), VPMC_E_STATE (validation-only context; save
 * without weights), VPMC_E_DEVICE. */
int vpmc_surrogate_load(vpmc_ctx *ctx, const char *weights_path);
int vpmc_surrogate_save(vpmc_ctx *ctx, const char *weights_path);
/* Use of the network in runs with VPMC_SURROGATE (Methods B; the
 * paper's block model is the plain transport, the network is this library's
 * replacement for the deep brass part of it).  A VP whose block entry point
 * lies in the brass at least d_fallback_mm from the opening's polygon is
 * queued; the network then gives its transmission probability p.  With
 * p_lo <= p <= p_hi the plain brass transport crosses it from its unchanged
 * state (so p_lo = 0, p_hi = 1 reproduces the run without the flag bit for
 * bit); otherwise the outcome is sampled (stopped: its energy goes to the block ledger;
 * transmitted: a mixture component, then energy loss, deflection and offset
 * with a uniform azimuth) and the patient transport follows.  Defaults
 * 3 mm, 0.02, 0.98.  Errors: VPMC_E_ARG unless d_fallback_mm >= 0 and
 * 0 <= p_lo <= p_hi <= 1. */
int vpmc_surrogate_config(vpmc_ctx *ctx, float d_fallback_mm, float p_lo, float p_hi);
/* outputs [n][29] for inputs [n][8] */
int vpmc_surrogate_forward(vpmc_ctx *ctx, const float *x, int n, float *out);
/* mean loss over n <= 16384 samples (transmission cross-entropy + mixture
 * negative log likelihood of y [n][3] for transmitted samples, trans[n] in
 * {0,1}) and its gradient with respect to the parameters, without update */
int vpmc_surrogate_loss_grad(vpmc_ctx *ctx, const float *x, const float *y, const float *trans, int n,
                             float *grad, double *loss);
/* Adam (lr, beta 0.9/0.999) on FP32 master weights over `epochs` shuffled
 * passes of mini-batches of `batch` samples; mean loss per epoch written to
 * loss_per_epoch[epochs] (optional). */
int vpmc_surrogate_train(vpmc_ctx *ctx, const float *x, const float *y, const float *trans, int n, int epochs,
                         int batch, float lr, uint64_t seed, float *loss_per_epoch);

/* After a CSR run: column (voxel) indices in ascending order per row and FP32
 * values (Gy per unit spot weight, converted from the int64 tally); q_raw
 * (optional) receives the int64 tallies themselves.  Buffers must hold
 * row_ptr[last] entries; pointer kind follows the run's flags. */
int vpmc_copy_csr(vpmc_ctx *ctx, int32_t *col_voxel, float *val_gy, int64_t *q_raw);

/* After a dense run: copy the int64 tally of scenario `scen_index` and the
 * fixed-point exponent k (dose = q * 2^-k MeV converted per voxel mass).
 * scen_index == -1 with q_out == NULL returns only k (also after a CSR run). */
int vpmc_last_tally(vpmc_ctx *ctx, int scen_index, int64_t *q_out, int *k_out, unsigned flags);

/* Measurements of the last run: transport_ms is the sum of the transport
 * kernels' durations (HIP events recorded on the run's stream around each
 * launch; with VPMC_SURROGATE each interval also holds the network and
 * resume kernels of that batch), total_ms the whole call; steps counts
 * condensed-history steps (every region), histories the VPs transported. */
typedef struct {
    double transport_ms, total_ms;
    uint64_t histories, steps, launches;
    uint64_t deferred;      /* VPs handed to the aperture surrogate (VPMC_SURROGATE) */
} vpmc_stats;
int vpmc_last_stats(const vpmc_ctx *ctx, vpmc_stats *out);

/* Host-only view of the library's own FP64 physics tables (no device
 * needed): material 0 water, 1 air, 2 PMMA, 3 brass, 4 bone; which 0 energy
 * nodes, 1 CSDA range, 2 straggling variance, 3 scattering power, 4 nuclear
 * removal.  Writes n <= 256 values; returns the node count. */
int vpmc_table_host(int material, int which, double *out, int n);

/* Dose-averaged LET (an addition to the paper's dose engine, whose TPS uses
 * LET clinically, Discussion): after a dense vpmc_run_spots with VPMC_LET,
 * copies scenario scen_index's int64 numerator sum(dep * LET) * w/N *
 * 2^(k - shift) into ql_out[nvox] (host, or device with VPMC_DEVICE_PTRS)
 * and writes shift (8).  Each step's LET is its mean CSDA stopping power in
 * keV/um (dE_csda over the step length; a VP that stops: E rho / R over its
 * residual range), so LET_d = ql * 2^shift / q with q from vpmc_last_tally.
 * Errors: VPMC_E_ARG (no output, bad index or flags), VPMC_E_STATE (the last
 * dense run did not tally LET), VPMC_E_DEVICE. */
int vpmc_last_let(vpmc_ctx *ctx, int scen_index, int64_t *ql_out, int *shift_out, unsigned flags);

/* Measurement support for the roofline of the transport (the atomic-rate
 * bound of the deposit tally): times n_atomics non-returning int64 atomic
 * adds into a zeroed nx*ny*nz grid on the context's device, issued as tracks
 * of 100 consecutive voxels along x at Gaussian lateral offsets (sigma 4
 * voxels) around 64 spot axes, the deposit pattern of a lateral pencil beam,
 * after one untimed warm-up pass; writes atomics per second.  Allocates and
 * frees its grid (8 bytes per voxel).  Errors: VPMC_E_ARG (grid below 16^3 or
 * >= 2^31 voxels, n_atomics outside [1024, 2^40], NULL pointers),
 * VPMC_E_STATE (validation-only context), VPMC_E_DEVICE (HIP failure). */
int vpmc_atomic_rate(vpmc_ctx *ctx, int nx, int ny, int nz, uint64_t n_atomics, double *atomics_per_s);

/* ---------------------------------------------------------------------------
 * Robust spot-weight optimisation on influence matrices (the plan optimiser
 * that consumes the matrices of the 13 robust scenarios, Methods E; the
 * paper's own optimiser belongs to its planning system, this one is the
 * library's).  Objective, averaged over the n_scen scenarios s:
 *   F(x) = 1/S sum_s [ w_target sum_{v in T} (D_s(v) - d_presc)^2
 *                      + w_oar sum_{v in O} max(0, D_s(v) - d_max)^2 ],
 *   D_s = A_s^T x, x >= 0: one weight per spot shared by all scenarios,
 * A_s[j, v] = the CSR row of (scenario s, spot j) = dose in voxel v per unit
 * weight.  Solver: projected FISTA with the fixed step 1/L, L = 1.05 x the
 * largest eigenvalue of 2/S sum_s A_s M A_s^T (M = w_target on T plus w_oar
 * on O) from n_power power iterations started at the all-ones vector; if
 * that eigenvalue is 0 the step is the projection alone.  Each dose sweep
 * sums in int64 fixed point and each gradient in FP64 in a fixed order, so
 * reruns give identical bits.  The objective and its gradient involve only
 * voxels with a structure bit, so the iterations use only the rows' entries
 * in those voxels (restricted once per index build) and read each of them
 * twice (a copy bucketed by voxel chunk for the dose, a compacted CSR for the
 * gradient): HBM-bound.  The optional dose output sweeps the whole rows.
 * ------------------------------------------------------------------------- */
#define VPMC_OPT_REUSE 16u  /* keep the segment index of the previous call: row_ptr, col and val
                               must be unchanged (same dims, same row_ptr contents checked) */

typedef struct {
    double d_presc;     /* target prescription, Gy (finite) */
    double w_target;    /* weight of the target term (>= 0) */
    double d_max;       /* organ-at-risk maximum dose, Gy (finite) */
    double w_oar;       /* weight of the organ term (>= 0) */
    int iters;          /* FISTA iterations, 0 .. 100000 */
    int n_power;        /* power iterations for L, 1 .. 1000 */
    int row_stride;     /* CSR row of (s, j) = s*row_stride + row_offset + j; 0 = n_spots.  A field's */
    int row_offset;     /*   spots inside rows of vpmc_run_batched: stride = all spots, offset = field's */
    unsigned flags;     /* VPMC_DEVICE_PTRS, VPMC_OPT_REUSE */
    void *hip_stream;   /* hipStream_t or NULL */
} vpmc_opt_params;

/* row_ptr [n_scen*row_stride + 1] non-decreasing int64 offsets (the whole
 * layout, as vpmc_run_batched writes it), col [row_ptr[n_scen*row_stride]]
 * voxel indices in [0, nvox), val [same] finite FP32, roi [nvox] bit 0 target,
 * bit 1 organ at risk (both allowed), x [n_spots] starting weights in, final
 * weights out (FP64), obj_hist [iters + 1] (optional) F at each FISTA
 * extrapolation point y_0 .. y_{iters-1} then F at the final x, step_L
 * (optional, always host) the L used, dose_gy [n_scen][nvox] (optional) D_s at
 * the final x.  Pointer kind of every array per p->flags.  n_spots <= 2^20.
 * Scratch, kept for VPMC_OPT_REUSE: 16 B per entry in a structure voxel,
 * with dose_gy also 8 B per entry of the used rows (a bucketed copy of the
 * whole rows), plus about 4 B x n_scen x nvox and 32 B per spot and scenario.
 * VPMC_OPT_REUSE also requires identical structure masks (checked).  Errors:
 * VPMC_E_ARG (dims, parameters, flags, row_ptr decreasing, a column out of
 * range or a value not finite), VPMC_E_STATE (validation-only context;
 * VPMC_OPT_REUSE without a matching index), VPMC_E_OOM, VPMC_E_DEVICE. */
int vpmc_optimize(vpmc_ctx *ctx, const int64_t *row_ptr, const int32_t *col, const float *val, int n_scen,
                  int n_spots, int nvox, const uint8_t *roi, const vpmc_opt_params *p, double *x, double *obj_hist,
                  double *step_L, float *dose_gy);

/* Dynamic voxel spacing of influence matrices (the planning system keeps
 * organs at risk on coarser voxels to save IM memory, Methods C): merges the
 * entries of every row into cells.  A cell is a run of consecutive voxels
 * (linear index, x fastest): cell_of_voxel [nvox of the loaded geometry] must
 * start at 0, grow by 0 or 1 from voxel to voxel and end at n_cells - 1.
 * Input rows: row_ptr [n_rows + 1] non-decreasing, col ascending within a
 * row, q the int64 fixed-point energies of exponent k (as vpmc_copy_csr's
 * q_raw and vpmc_last_tally's k).  Output: row_ptr_out [n_rows + 1] (always
 * written; rows start at 0), then, if any is given, cell_out (ascending cell
 * ids), q_out (exact int64 sums of the cell's entries) and val_out (FP32 Gy
 * per unit weight = the cell's energy over its mass, the mass-weighted mean
 * of its voxels' doses; masses from the loaded geometry), each
 * row_ptr_out[n_rows] long.  Pointer kind of every array per flags
 * (VPMC_DEVICE_PTRS).  Errors: VPMC_E_ARG (dims, k outside [0, 62], a bad
 * map, row_ptr decreasing, a column out of range or not ascending),
 * VPMC_E_STATE (no geometry; validation-only context), VPMC_E_OOM,
 * VPMC_E_DEVICE. */
int vpmc_csr_cells(vpmc_ctx *ctx, const int64_t *row_ptr, int n_rows, const int32_t *col, const int64_t *q, int k,
                   const int32_t *cell_of_voxel, int n_cells, int64_t *row_ptr_out, int32_t *cell_out,
                   int64_t *q_out, float *val_out, unsigned flags);

#ifdef __cplusplus
}
#endif
#endif /* VPMC_H */
