// Internal definitions shared by the host runtime and the gfx950 kernels of
// libvpmc.  Nothing here is part of the public C ABI (include/vpmc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vpmc {

// ---------------------------------------------------------------- tables
// Per-material tables X(E) (Methods A): NE nodes log-spaced on [1, 256] MeV.
constexpr int NE = 256;
constexpr int NMAT = 5;
constexpr double E_LO = 1.0;
constexpr double E_HI = 256.0;
enum Material { MAT_WATER = 0, MAT_AIR = 1, MAT_PMMA = 2, MAT_BRASS = 3, MAT_BONE = 4 };

// FP32 device blob, high parts first.  Shared: energy nodes, segment energy
// widths E_i+1 - E_i.  Per material: R, dE/dR per segment, R_i+1 - R_i,
// omega^2, T, Sigma_nuc; NE floats each, all per unit of density x path
// length in mm (10 x g/cm^2).  Then the low parts that make the node, width,
// slope and range-width tables (high, low) FP32 pairs of the FP64 values, for
// the double-float bookkeeping of the deterministic mode; the physics-mode
// kernels stage only the high block (32 KiB) in LDS.
enum { TAB_E = 0, TAB_DWH = NE, TAB_MAT0 = 2 * NE, TAB_PER_MAT = 6 * NE };
enum { T_R = 0, T_SH = 1, T_DH = 2, T_W2 = 3, T_T = 4, T_SN = 5 };
constexpr int TAB_HI_FLOATS = 2 * NE + NMAT * 6 * NE;    // 8192 floats = 32 KiB
enum { TAB_EL = TAB_HI_FLOATS, TAB_DWL = TAB_HI_FLOATS + NE, TAB_LMAT0 = TAB_HI_FLOATS + 2 * NE,
       TAB_PER_LMAT = 2 * NE };
enum { L_SL = 0, L_DL = 1 };
constexpr int TAB_FLOATS = TAB_HI_FLOATS + 2 * NE + NMAT * 2 * NE;   // 11264 floats = 44 KiB

struct MaterialDef {
    double z_over_a, mean_exc_ev, rad_len_gcm2, nuc_coeff, density;
};
extern const MaterialDef kMaterials[NMAT];

// FP64 host tables (generated once per process)
struct HostTables {
    double E[NE];
    double R[NMAT][NE], W2[NMAT][NE], T[NMAT][NE], SN[NMAT][NE];
};
const HostTables &host_tables();
void pack_device_tables(float *blob /* TAB_FLOATS */);
double range_host(int m, double E);           // piecewise-linear CSDA range (g/cm^2)
double rs_thickness_mm(double wet_mm);        // PMMA slab thickness for a given WET

// model constants (readings of the paper's unstated physics)
constexpr float STEP_FRACTION = 0.25f;     // step <= 1/4 residual range
constexpr float NUC_F_LOCAL = 0.10f;       // nuclear event: share deposited locally
constexpr float NUC_F_ESCAPE = 0.30f;      // share carried off by neutral secondaries
constexpr float NUC_SIGMA_RAD = 0.15f;     // deflection of the leading secondary
constexpr float EDGE_PUSH_MM = 1e-4f;      // push across an aperture edge in the BEV plane (FP32)
constexpr int MAX_STEPS = 1000000;         // safety bound on steps per VP
constexpr int MAX_BLOCK_ITER = 10000;      // bound on crossing-number tests per block traversal
constexpr double kSdfMargin = 8.0;         // mm of aperture distance raster beyond the polygon's box
constexpr double kListRadius = 1.9;        // mm: edges listed per raster cell around its reference point
constexpr double MEV_TO_J = 1.602176634e-13;

enum { L_GRID = 0, L_RS = 1, L_BLOCK = 2, L_ESCAPED = 3, L_NUC = 4, NLEDGER = 6 };
enum { PH_STRAGGLE = 1, PH_MCS = 2, PH_NUCLEAR = 4 };

// ------------------------------------------------------- kernel arguments
struct GeomDev {
    int kind, nx, ny, nz;
    float sp[3], lo[3];
    const int16_t *hu;
};

struct FieldDev {
    float iso[3], ex[3], ey[3], ez[3];
    int has_block, nv;
    const float2 *poly;
    // signed distance raster of the polygon (+ inside the opening), cell size
    // 1/sdf_ih, for conservative bounds that skip the exact edge loops
    const float *sdf;
    float sdf_x0, sdf_y0, sdf_ih, sdf_r, sdf_far;
    int sdf_nx, sdf_ny;
    // per raster cell near the boundary: edge lists around a reference point
    // whose side is known (bit 31 of cell_off), for exact tests on a handful
    // of edges; valid for BEV paths up to list_reach from the point
    const uint32_t *cell_off;
    const uint16_t *cell_edge;
    const float2 *cell_ref;
    float list_reach;
    float blk_zu, blk_zd, blk_rho, blk_t, blk_tl;
    int has_rs;
    float rs_zu, rs_zd, rs_r2, rs_rho, rs_rhol, rs_t, rs_tl;   // *_l: low parts of the FP64 values
    // virtual source vsad upstream of the origin plane (0: parallel beam);
    // divergent block (div): the opening at block depth pz is the polygon
    // scaled by pz * fs + fc0 (walls through the focus)
    float vsad;
    int div;
    float fs, fc0;
};

struct SpotDev {
    float x, y, e0, sigma, esig, emax, scale;   // scale = w/N * 2^k
    uint32_t nh;
};

// VP deferred at the block entry for the surrogate: its whole state on the
// block's upstream face (E + Elo is the compensated energy, pzlo the low part
// of the depth), so the plain transport can resume it unchanged
struct DeferRec {
    uint32_t spot, hist, nblk, tag;   // tag: the row within the epoch (influence-matrix runs)
    float x, y, u, v, w, E, Elo, pzlo, d_edge, thick, pad[2];
};
static_assert(sizeof(DeferRec) == 64, "DeferRec is 64 bytes");

struct SurDev {
    int enabled;
    float d_fallback;                 // VPs nearer the opening's edge stay on the plain transport
    unsigned long long *count;        // records written (may exceed capacity: the rest ran plain)
    unsigned long long capacity;
    DeferRec *rec;
};

struct LaunchDev {
    const SpotDev *spots;
    const unsigned long long *item_off;   // [n_spots + 1] prefix of items per spot
    int n_spots;
    unsigned long long n_items;
    int batch, n_batches;
    uint32_t key0, key1;
    unsigned physics;
    float shift[3];
    float range_scale;
    unsigned long long *tally;            // int64 fixed point, two's complement
    unsigned long long *let_tally;        // dose-averaged LET numerator (same layout) or null
    unsigned long long *ledger;           // [NLEDGER]
    unsigned long long *stats;            // [2]: steps, histories
    const float *tables;                  // TAB_FLOATS
    SurDev sur;
};

constexpr int POLY_LDS = 1024;  // == VPMC_MAX_VERTICES
constexpr int kLetShift = 8;    // LET numerator scale 2^(k - 8): LET <= 256 keV/um keeps it within the dose bound

// ------------------------------------------- influence-matrix (CSR) mode
// One row = (scenario, field, spot).  Rows are processed in epochs of at
// most kMaxSlots rows; row (row_begin + i) of an epoch owns slot i: a dense
// int64 grid plus one byte per block of 32 voxels that is set when the block
// receives a deposit.  Compaction counts and emits per chunk of 256 blocks.
constexpr int kMaxSlots = 1024;

struct RowDev {
    int field;            // index into the field table of the launch
    uint32_t field_id;    // caller's field id (part of the Philox key)
    uint32_t spot;        // spot index within its field (Philox counter)
    uint32_t spot_global; // index into the flattened spot table
    int scen;
    uint32_t n_hist;
    int tlo[3], tn[3];    // LDS tile box of the row in voxel indices (tn = 0: none)
};

struct ScenDev {
    float shift[3];
    float range_scale;
};

struct QueueDev {
    const RowDev *rows;
    const unsigned long long *chunk_off;  // [n_rows + 1] chunk prefix of this epoch's rows
    int row_begin, n_rows;
    unsigned long long n_chunks;
    unsigned long long *head;             // fresh-row counter of this epoch
    unsigned long long *row_next;         // [n_rows] chunk counter per row of this epoch
    int tile_cap;                         // int64 entries of the workgroup's LDS tile
    int hist_per_lane;                    // one chunk = 64 * hist_per_lane histories
    int refill_min;                       // idle lanes that trigger a refill in the patient loop
    float *stage;                         // [waves of the launch][64 * min(hist_per_lane, kStageHpl)] staged VPs (64 B)
    const FieldDev *fields;
    const int *poly_off;                  // per field: offset into polys
    const float2 *polys;
    int n_poly_total;
    const SpotDev *spots;
    const ScenDev *scen;
    uint32_t key0, seed_hi;
    unsigned physics;
    int div;                              // some field is divergent (virtual source or divergent block)
    unsigned long long *grid;             // [slots][gstride] int64 tallies
    uint8_t *mark;                        // [slots][mstride] touched-block bytes (32 voxels each)
    size_t nvox, nblk, nchunk;            // blocks = ceil(nvox/32), chunks = ceil(blocks/256)
    size_t gstride, mstride;              // gstride = 32 * nblk voxels, mstride >= nblk bytes
    unsigned long long *ledger;           // [n_scen][NLEDGER]
    unsigned long long *stats;            // [2]
    const float *tables;
    SurDev sur;                           // surrogate queue (enabled = 0: off)
    unsigned long long iter_cap;          // work-queue iterations a wavefront may make
    unsigned int *flags;                  // bit 2 (value 4) set when a wavefront reached iter_cap
};
constexpr unsigned long long kDefaultQueueCap = 1ull << 40;   // far above any run's chunk count
constexpr unsigned int kFlagAborted = 4u;

// staging floats the queue kernel needs for a launch shape (per wave up to
// 64 * kStageHpl VPs of 16 words)
constexpr size_t kStageFields = 16;
constexpr int kStageHpl = 32;
constexpr int kRefillMin = 8;   // idle lanes that trigger a refill of the patient loop
inline size_t queue_stage_floats(int blocks, int threads, int hist_per_lane) {
    const size_t hps = (size_t)(hist_per_lane < kStageHpl ? hist_per_lane : kStageHpl);
    return (size_t)blocks * (size_t)((threads + 63) / 64) * kStageFields * 64 * hps;
}
hipError_t launch_queue(const GeomDev &g, const QueueDev &Q, int blocks, int threads, hipStream_t s);
// workgroup size the queue kernel runs with for a requested size, and the
// LDS tile entries that leave the CU its full wave occupancy
int queue_threads(unsigned physics, int threads);
int queue_tile_cap(unsigned physics, int threads);

// ------------------------------------------------------- aperture surrogate
// MLP 8 -> 256 -> 256 -> 256 -> 256 -> 29, parameters layer by layer as
// W[out][in] then b[out] (FP32 master, BF16 copy in the same layout).
constexpr int MLP_LAYERS = 5;
constexpr int MLP_IN = 8;
constexpr int MLP_OUT = 29;
constexpr int MLP_HIDDEN = 256;
constexpr int MLP_OUT_LD = 32;   // row pitch of the BF16 output gradient
constexpr int kMlpSplit = 16;    // K split of the weight-gradient products
constexpr int MLP_MAX_BATCH = 16384;
constexpr unsigned long long kSurMaxRecords = 1ull << 22;   // surrogate queue (64 B each)

struct MlpBuffers {
    float *w;            // FP32 master parameters
    __bf16 *wb;          // BF16 parameters
    __bf16 *x;           // [n][8] inputs
    __bf16 *h[4];        // [n][256] hidden activations
    float *z[4];         // [n][256] hidden pre-activations
    float *out;          // [n][29]
    float *dout;         // [n][29] d loss / d out (batch mean)
    __bf16 *dout_b;      // [n][MLP_OUT_LD], zero padded
    __bf16 *dzb_a, *dzb_b;  // [n][256] d loss / d Z of a hidden layer
    float *wpart;        // [kMlpSplit][256 * 256] split-K partial weight gradients
    float *bpart;        // [(n + 31) / 32][256] 32-row partial bias gradients
    float *loss;         // [n] per-sample loss
};

hipError_t launch_sur_resume(const GeomDev &g, const FieldDev &f, const LaunchDev &L, const DeferRec *rec,
                             const float *out, unsigned long long n, float p_lo, float p_hi, hipStream_t s);
hipError_t launch_sur_resume_csr(const GeomDev &g, const QueueDev &Q, const DeferRec *rec, const float *out,
                                 unsigned long long n, float p_lo, float p_hi, hipStream_t s);
hipError_t launch_surrogate_sample(const FieldDev &f, const float *entries, int n, uint32_t key0, uint32_t key1,
                                   unsigned physics, const float *tables, float *x, float *y, float *t, hipStream_t s);
int mlp_param_count();
int mlp_param_offset(int layer);
int mlp_dim(int i);
hipError_t mlp_forward(const MlpBuffers &b, int n, hipStream_t s);
// fused inference of n samples: inputs x [n][8] FP32, or (rec != NULL) the
// features of deferred-VP records; outputs out [n][29] FP32
hipError_t mlp_infer(const float *x, const DeferRec *rec, int n, const __bf16 *wb, const float *wf, float *out,
                     hipStream_t s);
// forward + backward of n samples: gradient of the batch-mean loss into
// grad; *loss_acc += the batch-mean loss
hipError_t mlp_loss_grad(const MlpBuffers &b, const float *y, const float *trans, int n, float *grad,
                         double *loss_acc, hipStream_t s);
hipError_t mlp_gather(const float *x, const int *idx, int n, int cols, __bf16 *xb, float *xf, hipStream_t s);
hipError_t mlp_to_bf16(const float *x, __bf16 *y, size_t n, hipStream_t s);
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, __bf16 *pb, int np, float lr, int step,
                    hipStream_t s);
hipError_t launch_csr_count(const QueueDev &Q, unsigned int *cnt, hipStream_t s);
hipError_t launch_csr_chunk_scan(const unsigned int *cnt, unsigned int *coff, unsigned int *rowcnt, int n_rows,
                                 size_t nchunk, hipStream_t s);
hipError_t launch_csr_offsets(const unsigned int *nnz, int n_rows, int row_begin, unsigned long long *row_off,
                              unsigned long long *row_nnz, unsigned long long *used, unsigned long long capacity,
                              unsigned int *flags, hipStream_t s);
hipError_t launch_csr_emit(const QueueDev &Q, const unsigned int *cnt, const unsigned int *coff,
                           const unsigned long long *row_off, const unsigned long long *row_nnz, int32_t *col,
                           long long *qv, unsigned long long capacity, unsigned int *flags, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s);
hipError_t launch_atomic_rate(unsigned long long *grid, int nx, int ny, int nz, unsigned long long n_tracks, int len,
                              float sigma, uint32_t seed, hipStream_t s);
hipError_t launch_csr_scatter(const int32_t *col, const long long *qv, unsigned long long begin,
                              unsigned long long end, unsigned long long *dense, hipStream_t s);
hipError_t launch_csr_values(const int32_t *col, const long long *qv, size_t n, const GeomDev &g,
                             double mev_scale, float *val, hipStream_t s);
// dynamic voxel spacing: merge influence-matrix rows into cells (runs of
// consecutive voxels of a non-decreasing voxel -> cell map), a wavefront per
// piece of at most kCellPiece entries of one row
constexpr int kCellPiece = 4096;
struct CellPiece {
    long long begin;   // first entry (CSR index)
    int len;
    int row;
};
hipError_t launch_cell_mass(const GeomDev &g, const int32_t *cstart, int n_cells, double *mass, hipStream_t s);
hipError_t launch_cell_count(const long long *rp, const CellPiece *pcs, long long n_pieces, const int32_t *col,
                             const int32_t *cmap, int nvox, unsigned long long *cnt, unsigned *err, hipStream_t s);
hipError_t launch_cell_emit(const long long *rp, const CellPiece *pcs, long long n_pieces, const int32_t *col,
                            const long long *q, const int32_t *cmap, const long long *pout, const double *mass,
                            double mev_scale, int32_t *ocell, long long *oq, float *oval, hipStream_t s);

// ------------------------------------------------- spot-weight optimiser
#ifndef VPMC_OPT_CHUNK_BITS
#define VPMC_OPT_CHUNK_BITS 9
#endif
constexpr int kOptChunkBits = VPMC_OPT_CHUNK_BITS;
constexpr int kOptChunk = 1 << kOptChunkBits;   // voxels per forward workgroup (int64 LDS sums)
enum { kOptPowerInit = 0, kOptPower = 1, kOptFistaInit = 2, kOptFista = 3, kOptFinalPrep = 4, kOptFinal = 5 };
enum { kOptLam = 0, kOptL = 1 };   // device scalars

constexpr int kOptPiece = 4096;   // entries per gradient wavefront

// at most kOptPiece consecutive entries of one row
struct OptPiece {
    long long begin;   // first entry (CSR index)
    int len;
    int row;           // compact row s * n_spots + j
};

struct OptDev {
    const long long *row_ptr;       // CSR row pointer, row of (s, j) = s*row_stride + row_offset + j
    const int32_t *col;             // voxel indices per row
    const float *val;               // Gy per unit spot weight
    const uint8_t *roi;             // [nvox] bit 0 target, bit 1 organ at risk
    int n_scen, n_spots, row_stride, row_offset, nvox, nchunks;
    double d_presc, w_target, d_max, w_oar;
    // chunk-bucketed copy of the entries: list (s, chunk) holds entries
    // boff[list] .. boff[list + 1], key = spot << kOptChunkBits | voxel - chunk base
    const unsigned long long *boff; // [n_scen * nchunks + 1]
    const uint32_t *bkey;
    const float *bval;
    const uint32_t *work;           // [n_work] lists to sweep, in decreasing entry count
    long long n_work;
    const OptPiece *piece;          // gradient pieces, row-major
    long long n_pieces;
    const long long *piece_off;     // [n_scen * n_spots + 1] first piece of each compact row
    float *amax;                    // [n_scen * n_spots] largest |a| of each row
    float *resid;                   // [n_scen][nvox] residual of the last forward sweep
    float *rstruct;                 // [n_scen][nstruct] the same on the structure voxels only (or NULL)
    const int32_t *sidx;            // [nvox] index among the structure voxels, -1 elsewhere
    int nstruct;                    // structure voxels
    double *fpart;                  // [n_work] objective partials
    double *gpart;                  // [n_pieces] piece products with the residual
    double *x, *y, *z, *gvec;       // [n_spots]
    double *scale;                  // [2 * n_scen] 2^m, 2^-m of the next forward sweep
    double *scal;                   // device scalars (kOptLam, kOptL)
};

hipError_t opt_build_count(const OptDev &O, unsigned long long *cnt, unsigned *err, hipStream_t st);
hipError_t opt_roi_count(const OptDev &O, unsigned long long *rcnt, unsigned *err, hipStream_t st);
hipError_t opt_roi_copy(const OptDev &O, const long long *rptr, int32_t *ccol, float *cval, hipStream_t st);
hipError_t opt_renumber(int32_t *ccol, long long n, const int32_t *sidx, int nvox, hipStream_t st);
hipError_t opt_build_scan(unsigned long long *cnt, unsigned long long *off, size_t n, hipStream_t st);
hipError_t opt_build_emit(const OptDev &O, const unsigned long long *off, unsigned long long *cur, uint32_t *bkey,
                          float *bval, hipStream_t st);
hipError_t opt_forward(const OptDev &O, const double *w, int mode, float *dose_out, hipStream_t st);
hipError_t opt_gradient(const OptDev &O, hipStream_t st);
hipError_t opt_update(const OptDev &O, int mode, double beta, int it, double *hist, hipStream_t st);

// launchers (vpmc_kernels.hip)
hipError_t launch_transport(const GeomDev &g, const FieldDev &f, const LaunchDev &L, int blocks,
                            int threads, hipStream_t s);
hipError_t launch_fold_batch(unsigned long long *q_batch, long long *q_total, double *s2, size_t n,
                             hipStream_t s);
hipError_t launch_dose(const long long *q, const double *s2, int n_batches, const GeomDev &g,
                       double mev_scale, float *dose, float *sigma, size_t n, hipStream_t s);

// Static device scratch of the allocation-free dense run
// (vpmc_run_spots_noalloc): a file-scope __device__ array in
// vpmc_kernels.hip, one copy per GPU, held until the process ends.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxScratchDevices = 64;
// Device address of the scratch on `device`, which must be the current
// device: looked up once per device with hipGetSymbolAddress and kept.
hipError_t scratch_device_ptr(int device, void **out);

}  // namespace vpmc
