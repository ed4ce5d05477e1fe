/*
 * vpmc_oracle.c -- plain FP64 CPU oracle of the aperture-block virtual-particle
 * (VP) transport.  TEST INFRASTRUCTURE ONLY: the product path never links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.
 *
 * It is written for readability, not speed: one VP at a time, FP64
 * everywhere, binary searches for table lookups, OpenMP only over
 * histories.  It shares no code with the HIP library (no headers, no table
 * generator, no constants file); both follow the same written specification,
 * which is restated in the comments below with the passage of the paper it
 * reads.
 *
 * Paper: "Modelling small block aperture in an in-house developed
 * GPU-accelerated Monte Carlo-based dose engine for pencil beam scanning
 * proton therapy" (arXiv 2307.01416).
 *   Methods A   - VP concept: one proton-like VP per proton (primary or
 *                 secondary), all VPs created at the start, one model for
 *                 every VP; physics from pre-computed tables X(E) of
 *                 deposited energy, straggling, deflection and interaction
 *                 probability.
 *   Methods B   - 30 mm brass block, range shifter (RS) 45 mm WET, 61 mm
 *                 diameter, 10 mm gap; RS tables depend on energy only;
 *                 crossing-number test between the block's entrance and exit
 *                 planes at every step; open -> straight transport, brass ->
 *                 state updated from the brass tables.
 *   Methods D   - non-divergent apertures; dose grids; <0.5 % uncertainty.
 *   Methods E   - robust scenarios: range (stopping-power) scaling and
 *                 isocentre shifts.
 * Where the paper is silent the readings used here are the ones listed in
 * the design notes (R1-R28); each is named at the point of use.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------
 * Physical constants (CODATA 2018 / PDG) and model constants
 * ---------------------------------------------------------------------- */
#define N_AVOGADRO 6.02214076e23
#define R_ELECTRON_CM 2.8179403262e-13
#define ME_C2 0.51099895000      /* MeV */
#define MP_C2 938.27208816       /* MeV */
#define MEV_TO_J 1.602176634e-13
#define ES_MCS 13.6              /* MeV, scattering-power constant (R7) */
#define E_LO 1.0                 /* MeV, lowest table energy = cut-off (R6) */
#define E_HI 256.0               /* MeV */
#define NE 256                   /* table nodes, log-spaced on [E_LO, E_HI] */
#define STEP_FRACTION 0.25       /* step <= 1/4 of the residual range (R6) */
#define NUC_E_ZERO 7.0           /* nuclear removal ramps from 0 at 7 MeV ... */
#define NUC_E_FULL 20.0          /* ... to its full value at 20 MeV (R2) */
#define NUC_F_LOCAL 0.10         /* share of E deposited on a nuclear event (R2) */
#define NUC_F_ESCAPE 0.30        /* share carried away by neutral secondaries (R2) */
#define NUC_SIGMA_RAD 0.15       /* deflection of the leading secondary (R2) */
#define EDGE_PUSH_MM 1e-4        /* push across an aperture edge, in the aperture plane (R5) */
#define MAX_ITER 1000000         /* safety bound on steps per VP */
#define MAX_BLOCK_ITER 10000     /* safety bound on crossing-number tests per block traversal */
#define LET_SHIFT 8              /* LET numerator in units of 2^(8-k) MeV keV/um (LET <= 256 keV/um) */

enum { M_WATER = 0, M_AIR = 1, M_PMMA = 2, M_BRASS = 3, M_BONE = 4, NMAT = 5 };
enum { L_GRID = 0, L_RS = 1, L_BLOCK = 2, L_ESCAPED = 3, L_NUC = 4, L_SPARE = 5, NLEDGER = 6 };
enum { PH_STRAGGLE = 1, PH_MCS = 2, PH_NUCLEAR = 4 };

/* Materials (reading R1): Z/A, mean excitation energy I (eV), radiation
 * length X0 (g/cm^2), nuclear removal coefficient (cm^2/g) above 20 MeV,
 * nominal density (g/cm^3).  Brass = Cu/Zn 63/37 by mass, I from Bragg
 * additivity of Cu 322 eV and Zn 330 eV, 1/X0 = sum w_i / X0_i. */
typedef struct {
    double za, I_ev, x0, sig_nuc, rho;
} material_t;

static const material_t MATS[NMAT] = {
    {0.55508, 75.0, 36.08, 0.0115, 1.0},          /* water */
    {0.49919, 85.7, 36.62, 0.0110, 0.00120479},   /* air */
    {0.53937, 74.0, 40.55, 0.0112, 1.19},         /* PMMA (range shifter) */
    {0.457285, 324.947, 12.6975, 0.0075, 8.5},    /* brass (aperture block) */
    {0.52130, 106.4, 16.71, 0.0107, 1.85},        /* cortical bone */
};

/* ------------------------------------------------------------------------
 * Physics tables X(E): the paper's PDF database (Methods A) read as
 * analytic per-material tables on a log energy grid (reading R1).
 * ---------------------------------------------------------------------- */
static double g_E[NE];
static double g_R[NMAT][NE];   /* CSDA range from E_LO, g/cm^2 */
static double g_W2[NMAT][NE];  /* Bohr straggling variance per areal density, MeV^2 cm^2/g */
static double g_T[NMAT][NE];   /* projected-angle scattering power, rad^2 cm^2/g */
static double g_SN[NMAT][NE];  /* nuclear removal coefficient, cm^2/g */
static int g_ready = 0;

static double beta2_of(double E)
{
    double g = 1.0 + E / MP_C2;
    return 1.0 - 1.0 / (g * g);
}

/* Bethe mass stopping power for a proton, no shell or density corrections
 * (MeV cm^2/g).  K = 4 pi N_A r_e^2 m_e c^2; T_max in the PDG form. */
double orc_stopping_power(int m, double E)
{
    const double K = 4.0 * M_PI * N_AVOGADRO * R_ELECTRON_CM * R_ELECTRON_CM * ME_C2;
    double g = 1.0 + E / MP_C2;
    double b2 = 1.0 - 1.0 / (g * g);
    double r = ME_C2 / MP_C2;
    double tmax = 2.0 * ME_C2 * b2 * g * g / (1.0 + 2.0 * g * r + r * r);
    double I = MATS[m].I_ev * 1e-6;
    double L = 0.5 * log(2.0 * ME_C2 * b2 * g * g * tmax / (I * I)) - b2;
    return K * MATS[m].za / b2 * L;
}

/* Bohr energy-straggling variance per unit areal density with the
 * relativistic factor (1 - b^2/2)/(1 - b^2):  4 pi N_A r_e^2 (m_e c^2)^2 Z/A. */
double orc_omega2(int m, double E)
{
    const double C = 4.0 * M_PI * N_AVOGADRO * R_ELECTRON_CM * R_ELECTRON_CM * ME_C2 * ME_C2;
    double b2 = beta2_of(E);
    return C * MATS[m].za * (1.0 - 0.5 * b2) / (1.0 - b2);
}

/* Scattering power (E_s / pv)^2 / X0 for the projected angle (reading R7). */
double orc_scatter_power(int m, double E)
{
    double pv = E * (E + 2.0 * MP_C2) / (E + MP_C2);
    double a = ES_MCS / pv;
    return a * a / MATS[m].x0;
}

/* Nuclear removal coefficient: the material constant above 20 MeV, a linear
 * ramp to zero at 7 MeV (reading R2). */
double orc_nuclear_coeff(int m, double E)
{
    double f;
    if (E <= NUC_E_ZERO) f = 0.0;
    else if (E >= NUC_E_FULL) f = 1.0;
    else f = (E - NUC_E_ZERO) / (NUC_E_FULL - NUC_E_ZERO);
    return MATS[m].sig_nuc * f;
}

static double inv_stopping(int m, double E) { return 1.0 / orc_stopping_power(m, E); }

/* adaptive Simpson quadrature of 1/S on [a, b] */
static double simpson_rec(int m, double a, double b, double fa, double fm, double fb,
                          double whole, double tol, int depth)
{
    double c = 0.5 * (a + b);
    double l = 0.5 * (a + c), r = 0.5 * (c + b);
    double fl = inv_stopping(m, l), fr = inv_stopping(m, r);
    double left = (c - a) / 6.0 * (fa + 4.0 * fl + fm);
    double right = (b - c) / 6.0 * (fm + 4.0 * fr + fb);
    double diff = left + right - whole;
    if (depth <= 0 || fabs(diff) <= 15.0 * tol)
        return left + right + diff / 15.0;
    return simpson_rec(m, a, c, fa, fl, fm, left, 0.5 * tol, depth - 1) +
           simpson_rec(m, c, b, fm, fr, fb, right, 0.5 * tol, depth - 1);
}

static double range_integral(int m, double a, double b)
{
    double fa = inv_stopping(m, a), fb = inv_stopping(m, b), fm = inv_stopping(m, 0.5 * (a + b));
    double whole = (b - a) / 6.0 * (fa + 4.0 * fm + fb);
    return simpson_rec(m, a, b, fa, fm, fb, whole, 1e-14 * fabs(whole), 24);
}

void orc_init(void)
{
    if (g_ready) return;
    for (int i = 0; i < NE; i++)
        g_E[i] = E_LO * pow(E_HI / E_LO, (double)i / (double)(NE - 1));
    for (int m = 0; m < NMAT; m++) {
        g_R[m][0] = 0.0;
        for (int i = 1; i < NE; i++)
            g_R[m][i] = g_R[m][i - 1] + range_integral(m, g_E[i - 1], g_E[i]);
        for (int i = 0; i < NE; i++) {
            g_W2[m][i] = orc_omega2(m, g_E[i]);
            g_T[m][i] = orc_scatter_power(m, g_E[i]);
            g_SN[m][i] = orc_nuclear_coeff(m, g_E[i]);
        }
    }
    g_ready = 1;
}

/* segment index: the largest i in [0, NE-2] with E_i <= E */
static int seg_of_energy(double E)
{
    if (E <= g_E[0]) return 0;
    if (E >= g_E[NE - 1]) return NE - 2;
    int lo = 0, hi = NE - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (g_E[mid] <= E) lo = mid; else hi = mid;
    }
    return lo;
}

/* CSDA relation: E(R) is the piecewise-linear curve through the nodes
 * (R_i, E_i); R(E) is its inverse. */
double orc_range(int m, double E)
{
    if (E <= E_LO) return 0.0;
    int i = seg_of_energy(E);
    return g_R[m][i] + (E - g_E[i]) * (g_R[m][i + 1] - g_R[m][i]) / (g_E[i + 1] - g_E[i]);
}

double orc_energy_of_range(int m, double R)
{
    if (R <= 0.0) return E_LO;
    const double *r = g_R[m];
    int lo = 0, hi = NE - 1;
    if (R >= r[NE - 1]) lo = NE - 2;
    else {
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (r[mid] <= R) lo = mid; else hi = mid;
        }
    }
    return g_E[lo] + (R - r[lo]) * (g_E[lo + 1] - g_E[lo]) / (r[lo + 1] - r[lo]);
}

/* other tables: linear in E between nodes, clamped at the ends */
static double interp_node(const double *tab, double E)
{
    if (E <= g_E[0]) return tab[0];
    if (E >= g_E[NE - 1]) return tab[NE - 1];
    int i = seg_of_energy(E);
    double f = (E - g_E[i]) / (g_E[i + 1] - g_E[i]);
    return tab[i] + f * (tab[i + 1] - tab[i]);
}

/* table export for tests: which = 0 E, 1 R, 2 omega^2, 3 T, 4 Sigma_nuc */
int orc_table(int m, int which, double *out)
{
    orc_init();
    if (m < 0 || m >= NMAT) return -1;
    const double *src = which == 0 ? g_E : which == 1 ? g_R[m] : which == 2 ? g_W2[m]
                      : which == 3 ? g_T[m] : which == 4 ? g_SN[m] : NULL;
    if (!src) return -1;
    memcpy(out, src, sizeof(double) * NE);
    return NE;
}

double orc_material_density(int m) { return (m >= 0 && m < NMAT) ? MATS[m].rho : -1.0; }

/* ------------------------------------------------------------------------
 * HU -> (material, density) (reading R12): density piecewise linear through
 * (-1000, 0.00121) (0, 1.0) (1000, 1.6) (1500, 1.85) (3071, 2.8), HU clamped
 * to [-1000, 3071]; class air below -900, soft tissue (water) below 150,
 * bone above.
 * ---------------------------------------------------------------------- */
static void hu_material(int hu, int *m, double *rho)
{
    static const double H[5] = {-1000.0, 0.0, 1000.0, 1500.0, 3071.0};
    static const double D[5] = {0.00121, 1.0, 1.6, 1.85, 2.8};
    double h = hu < -1000 ? -1000.0 : hu > 3071 ? 3071.0 : (double)hu;
    int s = 0;
    while (s < 3 && h > H[s + 1]) s++;
    *rho = D[s] + (h - H[s]) * (D[s + 1] - D[s]) / (H[s + 1] - H[s]);
    *m = hu < -900 ? M_AIR : hu < 150 ? M_WATER : M_BONE;
}

void orc_hu_lookup(const int16_t *hu, int64_t n, int32_t *mat, double *rho)
{
    for (int64_t i = 0; i < n; i++) {
        int m; double r;
        hu_material(hu[i], &m, &r);
        mat[i] = m; rho[i] = r;
    }
}

/* ------------------------------------------------------------------------
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), one
 * counter-based stream per (spot, history).  Counter = (block n, history,
 * spot, 0); key = (seed low word, seed high word XOR field id).
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 32-bit word -> uniform on the open interval (0,1): top 23 bits + 1/2,
 * scaled by 2^-23; exactly representable in FP32 and FP64. */
double orc_uniform(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

/* standard-normal quantile by Newton iteration on erfc (no table) */
double orc_normal_quantile(double u)
{
    double p = u < 0.5 ? u : 1.0 - u;           /* exact: u is on a 2^-24 grid */
    double c = 2.0 * p;                          /* solve erfc(t) = c, t >= 0 */
    double lc = log(c * (2.0 - c));              /* ln(1 - y^2) with y = 1 - c */
    double a = 0.147, k = 2.0 / (M_PI * a) + 0.5 * lc;
    double t = sqrt(sqrt(k * k - lc / a) - k);   /* Winitzki's starting value */
    for (int it = 0; it < 50; it++) {
        double f = erfc(t) - c;
        double dfdt = -2.0 / sqrt(M_PI) * exp(-t * t);
        double dt = f / dfdt;
        t -= dt;
        if (fabs(dt) <= 1e-16 * fabs(t) + 1e-300) break;
    }
    double z = -M_SQRT2 * t;
    return u < 0.5 ? z : -z;
}

static void box_muller(double ua, double ub, double *z1, double *z2)
{
    double r = sqrt(-2.0 * log(ua));
    *z1 = r * cos(2.0 * M_PI * ub);
    *z2 = r * sin(2.0 * M_PI * ub);
}

/* ------------------------------------------------------------------------
 * Run description (host structs filled by the Python test harness)
 * ---------------------------------------------------------------------- */
typedef struct {
    int kind;                 /* 0 water (rho = 1), 1 HU */
    int nx, ny, nz;
    double sp[3], org[3];
    const int16_t *hu;        /* [nz][ny][nx] or NULL */
} orc_geom;

typedef struct {
    double iso[3], ex[3], ey[3], ez[3];   /* beam frame in CT coordinates */
    int has_block, nv;                    /* nv == 0 with a block: closed */
    const double *poly;                   /* nv (x,y) pairs, BEV, mm */
    double blk_t, blk_rho, blk_d;         /* thickness, density, downstream face to origin */
    int has_rs;
    double rs_t, rs_diam, rs_d;           /* physical thickness, diameter, downstream face */
    double vsad;                          /* virtual source upstream of the origin plane (0: parallel beam) */
    double focus;                         /* focus of the block's walls upstream of the origin plane
                                             (0: non-divergent block) */
} orc_field;

typedef struct {
    double x, y, e0, sigma, esig, weight;
    int64_t nh;
} orc_spot;

typedef struct {
    double shift[3];
    double range_scale;
} orc_scen;

typedef struct {
    uint64_t seed;
    int field_id;
    int physics;
    int k;                    /* fixed-point exponent */
    int batch, n_batches;     /* histories h with h mod n_batches == batch */
} orc_opts;

/* per-VP state */
typedef struct {
    double p[3], d[3], E;
    uint32_t key[2];
    uint32_t spot, hist, nblk;
    int physics;
    int n_nuc, n_steps;
    double brass_path;        /* path length inside brass (test support) */
} vp_t;

/* tally sink: either fixed-point atomics (run) or FP64 sums (trace) */
typedef struct {
    int64_t *q;                 /* [nvox] or NULL */
    double scale;               /* w_s / N_s * 2^k */
    int64_t *qL;                /* [nvox] LET numerator or NULL */
    int64_t led_q[NLEDGER];     /* per-thread fixed-point ledgers */
    double *grid_fp;            /* trace: FP64 per-voxel deposits or NULL */
    double *grid_let_fp;        /* trace: FP64 per-voxel LET numerator (deposit x LET) or NULL */
    double led_fp[NLEDGER];     /* trace: FP64 ledgers */
    int track_touch;            /* trace: list the voxels given their first deposit */
    int64_t *touch, n_touch, cap_touch;
} sink_t;

/* deposit e (MeV) in voxel v by a step of LET `let` (MeV/mm = keV/um): the
 * dose tally and, when asked for, the numerator of the dose-averaged LET,
 * rne(e * let * w/N * 2^(k - LET_SHIFT)) */
static void sink_grid(sink_t *s, int64_t v, double e, double let)
{
    if (e == 0.0) return;
    s->led_fp[L_GRID] += e;
    if (s->track_touch && s->grid_fp[v] == 0.0) {
        if (s->n_touch == s->cap_touch) {
            s->cap_touch = s->cap_touch ? 2 * s->cap_touch : 1024;
            s->touch = (int64_t *)realloc(s->touch, (size_t)s->cap_touch * sizeof(int64_t));
            if (!s->touch) abort();
        }
        s->touch[s->n_touch++] = v;
    }
    if (s->grid_fp) s->grid_fp[v] += e;
    if (s->grid_let_fp) s->grid_let_fp[v] += e * let;
    int64_t q = llrint(e * s->scale);
    s->led_q[L_GRID] += q;
    if (s->q && q) __atomic_fetch_add(&s->q[v], q, __ATOMIC_RELAXED);
    if (s->qL) {
        int64_t qL = llrint(e * let * ldexp(s->scale, -LET_SHIFT));
        if (qL) __atomic_fetch_add(&s->qL[v], qL, __ATOMIC_RELAXED);
    }
}

static void sink_ledger(sink_t *s, int j, double e)
{
    if (e == 0.0) return;
    s->led_fp[j] += e;
    s->led_q[j] += llrint(e * s->scale);
}

static void draw_block(vp_t *vp, double u[4])
{
    uint32_t ctr[4] = {vp->nblk, vp->hist, vp->spot, 0u}, w[4];
    orc_philox4x32_10(ctr, vp->key, w);
    vp->nblk++;
    for (int j = 0; j < 4; j++) u[j] = orc_uniform(w[j]);
}

/* Rotate a unit direction by small projected angles (ax, ay) about two axes
 * perpendicular to it.  The perpendicular basis is the branch-free one of
 * Duff et al. (JCGT 2017); cos/sin of the polar angle are exact. */
static void rotate_dir(double d[3], double ax, double ay)
{
    double th = sqrt(ax * ax + ay * ay);
    if (th == 0.0) return;
    double sg = copysign(1.0, d[2]);
    double a = -1.0 / (sg + d[2]);
    double b = d[0] * d[1] * a;
    double e1[3] = {1.0 + sg * d[0] * d[0] * a, sg * b, -sg * d[0]};
    double e2[3] = {b, sg + d[1] * d[1] * a, -d[1]};
    double c = cos(th), s = sin(th) / th, n[3], nn = 0.0;
    for (int k = 0; k < 3; k++) { n[k] = c * d[k] + s * (ax * e1[k] + ay * e2[k]); nn += n[k] * n[k]; }
    nn = 1.0 / sqrt(nn);
    for (int k = 0; k < 3; k++) d[k] = n[k] * nn;
}

enum { ST_STOP = 0, ST_GEO = 1, ST_INNER = 2 };

/* One condensed-history step in a homogeneous region (Methods A: the VP's
 * state is updated from the tables X(E)).
 *   rho_loss: density for energy loss and straggling (range-scaled in the
 *             patient, R13); rho: density for scattering and nuclear removal
 *   dg:       distance (mm) to the region's geometric limit along d
 * On return *dep is the energy left in this region, *esc the nuclear-escaped
 * energy; the VP has moved (hinge scheme) and E is updated. */
/* One condensed-history step.  *let: the step's linear energy transfer
 * (MeV/mm = keV/um), the mean CSDA stopping power over the step, dE_csda / s;
 * for a VP that stops, its energy over its residual path, E / (R / rho); at
 * the cut-off, the CSDA relation's slope on its first segment (LET
 * tally: dose-averaged LET = sum(dep * let) / sum(dep) per voxel). */
static int phys_step(vp_t *vp, int m, double rho_loss, double rho, double dg,
                     double *dep, double *esc, double *let)
{
    *dep = 0.0; *esc = 0.0; *let = 0.0;
    vp->n_steps++;
    if (vp->E <= E_LO) {
        *let = rho_loss / 10.0 * (g_E[1] - g_E[0]) / (g_R[m][1] - g_R[m][0]);
        *dep = vp->E; vp->E = 0.0; return ST_STOP;
    }
    double R = orc_range(m, vp->E);
    if (rho_loss * dg / 10.0 >= R) {           /* stops inside: range-out */
        *let = vp->E * rho_loss / (10.0 * R);
        *dep = vp->E; vp->E = 0.0; return ST_STOP;
    }
    double smax = 10.0 * STEP_FRACTION * R / rho_loss;   /* mm */
    int geo = dg <= smax;
    double s = geo ? dg : smax;
    double E = vp->E;
    double E1 = orc_energy_of_range(m, R - rho_loss * s / 10.0);   /* CSDA */
    double Ebar = 0.5 * (E + E1);
    if (s > 0.0) *let = (E - E1) / s;
    double u[4] = {0.5, 0.5, 0.5, 1.0};
    if (vp->physics) draw_block(vp, u);
    if (vp->physics & PH_STRAGGLE) {
        double var = rho_loss * s / 10.0 * interp_node(g_W2[m], Ebar);
        E1 += sqrt(var) * orc_normal_quantile(u[2]);
        if (E1 < 0.0) E1 = 0.0;
        if (E1 > E) E1 = E;
    }
    *dep = E - E1;
    if (vp->physics & PH_MCS) {
        double th0 = sqrt(rho * s / 10.0 * interp_node(g_T[m], Ebar));
        double z1, z2;
        box_muller(u[0], u[1], &z1, &z2);
        for (int k = 0; k < 3; k++) vp->p[k] += 0.5 * s * vp->d[k];
        rotate_dir(vp->d, th0 * z1, th0 * z2);
        for (int k = 0; k < 3; k++) vp->p[k] += 0.5 * s * vp->d[k];
    } else {
        for (int k = 0; k < 3; k++) vp->p[k] += s * vp->d[k];
    }
    if (vp->physics & PH_NUCLEAR) {
        double P = -expm1(-rho * s / 10.0 * interp_node(g_SN[m], Ebar));
        if (u[3] < P) {
            /* the VP becomes its leading secondary proton (R2) */
            double v[4], n1, n2;
            draw_block(vp, v);
            double loc = NUC_F_LOCAL * E1, out = NUC_F_ESCAPE * E1;
            E1 = E1 - loc - out;
            *dep += loc;
            *esc = out;
            box_muller(v[0], v[1], &n1, &n2);
            rotate_dir(vp->d, NUC_SIGMA_RAD * n1, NUC_SIGMA_RAD * n2);
            vp->n_nuc++;
        }
    }
    vp->E = E1;
    return geo ? ST_GEO : ST_INNER;
}

/* ------------------------------------------------------------------------
 * Aperture opening: crossing-number (ray-casting) point-in-polygon test
 * (Methods B) with the half-open rule for ties (R5).
 * ---------------------------------------------------------------------- */
int orc_in_polygon(const double *poly, int nv, double x, double y)
{
    int c = 0;
    for (int i = 0, j = nv - 1; i < nv; j = i++) {
        double xi = poly[2 * i], yi = poly[2 * i + 1], xj = poly[2 * j], yj = poly[2 * j + 1];
        if ((yi > y) != (yj > y)) {
            double xc = xi + (y - yi) * (xj - xi) / (yj - yi);
            if (x < xc) c = !c;
        }
    }
    return c;
}

/* Divergent block (the paper's next step, Discussion): every wall is the
 * plane through the focus and an edge of the polygon, which is given on the
 * downstream face; at depth z the opening is the polygon scaled by
 * s(z) = (z + focus) / (focus - blk_d).  A non-divergent block has s = 1. */
static double blk_scale(const orc_field *f, double z)
{
    return f->focus > 0.0 ? (z + f->focus) / (f->focus - f->blk_d) : 1.0;
}

static double blk_kw(const orc_field *f, double w)
{
    return f->focus > 0.0 ? w / (f->focus - f->blk_d) : 0.0;
}

/* path length along d until the ray from p meets a wall: for the edge (a, b)
 * the point p + t d lies on the wall when p_xy + t d_xy = s(t) (a + lam (b - a))
 * with s(t) = s0 + t kw and 0 <= lam <= 1, which is linear in t (INFINITY if
 * it never does).  s0 = 1, kw = 0 is the non-divergent block, where this is
 * the ray-segment intersection of the beam's-eye-view projection. */
double orc_edge_distance_div(const double *poly, int nv, const double p[3], const double d[3], double s0, double kw)
{
    double best = INFINITY;
    for (int i = 0, j = nv - 1; i < nv; j = i++) {
        double ax = poly[2 * j], ay = poly[2 * j + 1];
        double ex = poly[2 * i] - ax, ey = poly[2 * i + 1] - ay;
        double ux = d[0] - kw * ax, uy = d[1] - kw * ay;
        double den = ux * ey - uy * ex;
        if (den == 0.0) continue;
        double wx = s0 * ax - p[0], wy = s0 * ay - p[1];
        double t = (wx * ey - wy * ex) / den;
        double mu = (wx * uy - wy * ux) / den;
        double st = s0 + t * kw;
        if (t > 0.0 && st > 0.0 && mu >= 0.0 && mu <= st && t < best) best = t;
    }
    return best;
}

/* path length along the 3D direction d until the BEV projection of the ray
 * from (x, y) meets an edge of the polygon (INFINITY if never) */
double orc_edge_distance(const double *poly, int nv, double x, double y, double u, double v)
{
    double best = INFINITY;
    for (int i = 0, j = nv - 1; i < nv; j = i++) {
        double ax = poly[2 * j], ay = poly[2 * j + 1];
        double ex = poly[2 * i] - ax, ey = poly[2 * i + 1] - ay;
        double den = u * ey - v * ex;
        if (den == 0.0) continue;
        double wx = ax - x, wy = ay - y;
        double t = (wx * ey - wy * ex) / den;
        double lam = (wx * v - wy * u) / den;
        if (t > 0.0 && lam >= 0.0 && lam <= 1.0 && t < best) best = t;
    }
    return best;
}

static double plane_distance(const vp_t *vp, double zu, double zd, int *down)
{
    double w = vp->d[2];
    if (w > 0.0) { *down = 1; return (zd - vp->p[2]) / w; }
    if (w < 0.0) { *down = 0; return (zu - vp->p[2]) / w; }
    *down = 1;
    return INFINITY;
}

enum { EX_DOWN = 0, EX_GONE = 1 };

/* Move the VP's projected (BEV) position EDGE_PUSH_MM further along its
 * projected direction, so that the next crossing-number test sees it on the
 * far side of the edge it has just reached; its depth is unchanged (R5). */
static void edge_push(vp_t *vp, const orc_field *f)
{
    /* in a divergent block the crossing direction is that of the scaled
     * position p_xy / s(z): d_xy - kw p_xy / s */
    double s = blk_scale(f, vp->p[2]), kw = blk_kw(f, vp->d[2]);
    double u = vp->d[0] - kw * (vp->p[0] / s), v = vp->d[1] - kw * (vp->p[1] / s), n = sqrt(u * u + v * v);
    if (n > 0.0) {
        vp->p[0] += EDGE_PUSH_MM * u / n;
        vp->p[1] += EDGE_PUSH_MM * v / n;
    }
}

/* homogeneous slab (range shifter): material m, density rho, z in [zu, zd] */
static int slab_transport(vp_t *vp, sink_t *sk, int m, double rho, double zu, double zd, int ledger)
{
    for (int it = 0; it < MAX_ITER; it++) {
        int down;
        double tp = plane_distance(vp, zu, zd, &down);
        if (tp < 0.0) tp = 0.0;
        double dep, esc;
        double let;
        int st = phys_step(vp, m, rho, rho, tp, &dep, &esc, &let);
        sink_ledger(sk, ledger, dep);
        sink_ledger(sk, L_NUC, esc);
        if (st == ST_STOP) return EX_GONE;
        if (st == ST_GEO || vp->p[2] >= zd || vp->p[2] <= zu) {
            int out_down = (st == ST_GEO) ? down : (vp->p[2] >= zd);
            vp->p[2] = out_down ? zd : zu;
            if (out_down) return EX_DOWN;
            sink_ledger(sk, L_ESCAPED, vp->E);
            return EX_GONE;
        }
    }
    sink_ledger(sk, L_ESCAPED, vp->E);
    return EX_GONE;
}

/* aperture block: z in [zu, zd]; at every step the crossing number at the
 * VP's projected position decides opening (straight transport, no random
 * numbers) or brass (a condensed-history step with the brass tables) */
static int block_transport(vp_t *vp, sink_t *sk, const orc_field *f, double zu, double zd)
{
    for (int it = 0; it < MAX_BLOCK_ITER; it++) {
        int down;
        double tp = plane_distance(vp, zu, zd, &down);
        if (tp < 0.0) tp = 0.0;
        double s0 = blk_scale(f, vp->p[2]), kw = blk_kw(f, vp->d[2]);
        int open = f->nv >= 3 && orc_in_polygon(f->poly, f->nv, vp->p[0] / s0, vp->p[1] / s0);
        double te = f->nv >= 3 ? orc_edge_distance_div(f->poly, f->nv, vp->p, vp->d, s0, kw) : INFINITY;
        if (open) {
            if (tp <= te) {
                for (int k = 0; k < 3; k++) vp->p[k] += tp * vp->d[k];
                vp->p[2] = down ? zd : zu;
                if (down) return EX_DOWN;
                sink_ledger(sk, L_ESCAPED, vp->E);
                return EX_GONE;
            }
            for (int k = 0; k < 3; k++) vp->p[k] += te * vp->d[k];
            edge_push(vp, f);
            continue;
        }
        double dg = te < tp ? te : tp;
        double dep, esc;
        double let;
        double p0[3] = {vp->p[0], vp->p[1], vp->p[2]};
        int st = phys_step(vp, M_BRASS, f->blk_rho, f->blk_rho, dg, &dep, &esc, &let);
        vp->brass_path += sqrt((vp->p[0] - p0[0]) * (vp->p[0] - p0[0]) + (vp->p[1] - p0[1]) * (vp->p[1] - p0[1]) +
                               (vp->p[2] - p0[2]) * (vp->p[2] - p0[2]));
        sink_ledger(sk, L_BLOCK, dep);
        sink_ledger(sk, L_NUC, esc);
        if (st == ST_STOP) return EX_GONE;
        if (st == ST_GEO && tp <= te) {
            vp->p[2] = down ? zd : zu;
            if (down) return EX_DOWN;
            sink_ledger(sk, L_ESCAPED, vp->E);
            return EX_GONE;
        }
        if (st == ST_GEO) edge_push(vp, f);
        if (vp->p[2] >= zd) { vp->p[2] = zd; return EX_DOWN; }
        if (vp->p[2] <= zu) { vp->p[2] = zu; sink_ledger(sk, L_ESCAPED, vp->E); return EX_GONE; }
    }
    sink_ledger(sk, L_ESCAPED, vp->E);
    return EX_GONE;
}

/* Beam line in the beam frame: source ray -> range shifter -> aperture block.
 * On return 1, (p, d) describe the VP's ray and *tmin the ray parameter
 * before which it may not enter the patient (the last component's exit). */
static int beamline(vp_t *vp, sink_t *sk, const orc_field *f, double *tmin)
{
    *tmin = -INFINITY;
    if (f->has_rs) {
        double zu = -(f->rs_d + f->rs_t), zd = -f->rs_d;
        double t = (zu - vp->p[2]) / vp->d[2];
        double q[3];
        for (int k = 0; k < 3; k++) q[k] = vp->p[k] + t * vp->d[k];
        q[2] = zu;
        double r = 0.5 * f->rs_diam;
        if (q[0] * q[0] + q[1] * q[1] <= r * r) {     /* membership at entry (R11) */
            memcpy(vp->p, q, sizeof q);
            if (slab_transport(vp, sk, M_PMMA, MATS[M_PMMA].rho, zu, zd, L_RS) != EX_DOWN) return 0;
            *tmin = 0.0;
        }
    }
    if (f->has_block) {
        double zu = -(f->blk_d + f->blk_t), zd = -f->blk_d;
        if (vp->d[2] <= 0.0) { sink_ledger(sk, L_ESCAPED, vp->E); return 0; }
        double t = (zu - vp->p[2]) / vp->d[2];
        double q[3];
        for (int k = 0; k < 3; k++) q[k] = vp->p[k] + t * vp->d[k];
        q[2] = zu;
        double su = blk_scale(f, zu);
        int open = f->nv >= 3 && orc_in_polygon(f->poly, f->nv, q[0] / su, q[1] / su);
        if (open) {
            double te = orc_edge_distance_div(f->poly, f->nv, q, vp->d, su, blk_kw(f, vp->d[2]));
            double tx = (zd - zu) / vp->d[2];
            if (te >= tx) {                      /* straight through the opening */
                *tmin = (zd - vp->p[2]) / vp->d[2];
                return 1;
            }
        }
        memcpy(vp->p, q, sizeof q);
        if (block_transport(vp, sk, f, zu, zd) != EX_DOWN) return 0;
        *tmin = 0.0;
    }
    return 1;
}

static void voxel_material(const orc_geom *g, int64_t v, int *m, double *rho)
{
    if (g->kind == 0) { *m = M_WATER; *rho = 1.0; return; }
    hu_material(g->hu[v], m, rho);
}

/* Patient: beam frame -> CT frame (isocentre, axes, scenario shift: the
 * patient moves by +shift so the VP's CT coordinates move by -shift), ray-box
 * entry, then voxel-by-voxel condensed-history steps with dose tallies. */
static void patient(vp_t *vp, sink_t *sk, const orc_geom *g, const orc_field *f,
                    const orc_scen *sc, double tmin)
{
    double p[3], d[3];
    for (int k = 0; k < 3; k++) {
        p[k] = (f->iso[k] + (vp->p[0] * f->ex[k] + vp->p[1] * f->ey[k] + vp->p[2] * f->ez[k])) - sc->shift[k];
        d[k] = vp->d[0] * f->ex[k] + vp->d[1] * f->ey[k] + vp->d[2] * f->ez[k];
    }
    const int n[3] = {g->nx, g->ny, g->nz};
    double lo[3], hi[3];
    for (int k = 0; k < 3; k++) { lo[k] = g->org[k]; hi[k] = g->org[k] + n[k] * g->sp[k]; }
    double tnear = -INFINITY, tfar = INFINITY;
    int ax_near = -1;
    for (int k = 0; k < 3; k++) {
        if (d[k] == 0.0) {
            if (p[k] < lo[k] || p[k] >= hi[k]) { sink_ledger(sk, L_ESCAPED, vp->E); return; }
            continue;
        }
        double t1 = (lo[k] - p[k]) / d[k], t2 = (hi[k] - p[k]) / d[k];
        double a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
        if (a > tnear) { tnear = a; ax_near = k; }
        if (b < tfar) tfar = b;
    }
    double t0 = tnear > tmin ? tnear : tmin;
    if (!(tfar > t0)) { sink_ledger(sk, L_ESCAPED, vp->E); return; }
    for (int k = 0; k < 3; k++) p[k] += t0 * d[k];
    if (t0 == tnear && ax_near >= 0) p[ax_near] = d[ax_near] > 0.0 ? lo[ax_near] : hi[ax_near];
    int idx[3];
    for (int k = 0; k < 3; k++) {
        double c = floor((p[k] - lo[k]) / g->sp[k]);
        idx[k] = !(c >= 0) ? 0 : c > n[k] - 1 ? n[k] - 1 : (int)c;   /* NaN -> 0 */
    }
    memcpy(vp->p, p, sizeof p);
    memcpy(vp->d, d, sizeof d);
    for (int it = 0; it < MAX_ITER; it++) {
        int64_t v = idx[0] + (int64_t)g->nx * (idx[1] + (int64_t)g->ny * idx[2]);
        int m; double rho;
        voxel_material(g, v, &m, &rho);
        double rho_loss = rho * sc->range_scale;
        /* distance to the voxel exit; ties go to the lower axis */
        double dg = INFINITY, bnd = 0.0;
        int ax = -1, sgn = 0;
        for (int k = 0; k < 3; k++) {
            if (vp->d[k] == 0.0) continue;
            int up = vp->d[k] > 0.0;
            double b = lo[k] + (idx[k] + up) * g->sp[k];
            double t = (b - vp->p[k]) / vp->d[k];
            if (t < 0.0) t = 0.0;
            if (t < dg) { dg = t; ax = k; sgn = up ? 1 : -1; bnd = b; }
        }
        double dep, esc, let;
        int st = phys_step(vp, m, rho_loss, rho, dg, &dep, &esc, &let);
        sink_grid(sk, v, dep, let);
        sink_ledger(sk, L_NUC, esc);
        if (st == ST_STOP) return;
        if (st == ST_GEO) {
            idx[ax] += sgn;
            vp->p[ax] = bnd;
            if (idx[ax] < 0 || idx[ax] >= n[ax]) { sink_ledger(sk, L_ESCAPED, vp->E); return; }
        }
        /* Keep the hinge end point in its voxel (reading: the paper's step
         * loop is voxel by voxel; the deflected second half of a step may end
         * up to s/2 * theta beyond a face of the voxel the step began in, and
         * is moved back onto that face; the face crossed by a boundary-limited
         * step is set exactly).  Its effect on the lateral spread is below
         * the Fermi-Eyges pins' resolution (0.3 %). */
        for (int k = 0; k < 3; k++) {
            double a = lo[k] + idx[k] * g->sp[k], b = lo[k] + (idx[k] + 1) * g->sp[k];
            if (vp->p[k] < a) vp->p[k] = a;
            if (vp->p[k] > b) vp->p[k] = b;
        }
    }
    sink_ledger(sk, L_ESCAPED, vp->E);
}

/* Source (Methods A, Introduction): Gaussian pencil beam, spot sigma from
 * the spot list, monoenergetic unless an energy spread is given.  The VP
 * starts on its ray at the beam-frame origin plane, direction +z, or with a
 * virtual source vsad upstream of that plane (scanned beams diverge from it)
 * along the line from the virtual source through its start point. */
static void source(vp_t *vp, const orc_spot *sp, const orc_field *f, const double *move)
{
    double u[4], z1, z2;
    draw_block(vp, u);
    box_muller(u[0], u[1], &z1, &z2);
    vp->p[0] = sp->x + sp->sigma * z1;
    vp->p[1] = sp->y + sp->sigma * z2;
    if (move) {                 /* test support: start moved in the source plane (mm) */
        vp->p[0] += move[0];
        vp->p[1] += move[1];
    }
    vp->p[2] = 0.0;
    vp->d[0] = 0.0; vp->d[1] = 0.0; vp->d[2] = 1.0;
    if (f->vsad > 0.0) {
        double n = sqrt(vp->p[0] * vp->p[0] + vp->p[1] * vp->p[1] + f->vsad * f->vsad);
        vp->d[0] = vp->p[0] / n;
        vp->d[1] = vp->p[1] / n;
        vp->d[2] = f->vsad / n;
    }
    vp->E = sp->e0;
    if (sp->esig > 0.0) {
        double e = sp->e0 + sp->esig * orc_normal_quantile(u[2]);
        double emax = sp->e0 + 6.0 * sp->esig;
        if (emax > E_HI) emax = E_HI;
        if (e > emax) e = emax;
        if (e < E_LO) e = E_LO;
        vp->E = e;
    }
    if (move) vp->E += move[2];   /* test support: start energy offset (MeV) */
}

static void one_history_moved(const orc_geom *g, const orc_field *f, const orc_spot *sp, int spot_index,
                              int64_t h, const orc_scen *sc, const orc_opts *o, sink_t *sk, vp_t *vp,
                              const double *move)
{
    memset(vp, 0, sizeof *vp);
    vp->key[0] = (uint32_t)(o->seed & 0xffffffffu);
    vp->key[1] = (uint32_t)(o->seed >> 32) ^ (uint32_t)o->field_id;
    vp->spot = (uint32_t)spot_index;
    vp->hist = (uint32_t)h;
    vp->physics = o->physics;
    source(vp, sp, f, move);
    double tmin;
    if (!beamline(vp, sk, f, &tmin)) return;
    patient(vp, sk, g, f, sc, tmin);
}

static void one_history(const orc_geom *g, const orc_field *f, const orc_spot *sp, int spot_index,
                        int64_t h, const orc_scen *sc, const orc_opts *o, sink_t *sk, vp_t *vp)
{
    one_history_moved(g, f, sp, spot_index, h, sc, o, sk, vp, NULL);
}

/* Run all histories h of spots [s_begin, s_end) in the requested batch.
 * q[nvox] receives int64 fixed-point deposits rne(dE * w_s/N_s * 2^k);
 * led[6] the same for the ledgers; qL[nvox] (optional) the LET numerator
 * rne(dE * LET * w_s/N_s * 2^(k - LET_SHIFT)).  Returns the number of
 * histories run. */
int64_t orc_run(const orc_geom *g, const orc_field *f, const orc_spot *spots, int s_begin, int s_end,
                const orc_scen *sc, const orc_opts *o, int64_t *q, int64_t *led, int nthreads, int64_t *qL)
{
    orc_init();
    int B = o->n_batches > 1 ? o->n_batches : 1;
    int b = o->n_batches > 1 ? o->batch : 0;
    int64_t total = 0;
    for (int s = s_begin; s < s_end; s++) {
        const orc_spot *sp = &spots[s];
        double scale = ldexp(sp->weight / (double)sp->nh, o->k);
        int64_t nb = sp->nh > b ? (sp->nh - b + B - 1) / B : 0;
        int64_t led_tot[NLEDGER] = {0};
#ifdef _OPENMP
        if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
        {
            sink_t sk;
            memset(&sk, 0, sizeof sk);
            sk.q = q;
            sk.qL = qL;
            sk.scale = scale;
            vp_t vp;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t j = 0; j < nb; j++) {
                int64_t h = b + j * B;
                one_history(g, f, sp, s, h, sc, o, &sk, &vp);
            }
            for (int l = 0; l < NLEDGER; l++)
                __atomic_fetch_add(&led_tot[l], sk.led_q[l], __ATOMIC_RELAXED);
        }
        for (int l = 0; l < NLEDGER; l++) led[l] += led_tot[l];
        total += nb;
    }
    return total;
}

/* One history with FP64 bookkeeping for invariant tests: ledgers[6] in MeV
 * (index 0 = patient grid), grid_fp[nvox] (optional) FP64 deposits,
 * grid_let_fp[nvox] (optional) the FP64 sum of deposit x LET (MeV x keV/um)
 * per voxel, info[4] = {steps, nuclear events, random blocks used, 0};
 * move[3] (optional) moves the start in the source plane (move[0], move[1]
 * in mm, before a virtual source's direction is taken from it) and adds
 * move[2] MeV to its energy. */
void orc_trace_history(const orc_geom *g, const orc_field *f, const orc_spot *sp, int spot_index,
                       int64_t h, const orc_scen *sc, const orc_opts *o, double *ledgers,
                       double *grid_fp, int64_t *info, double *grid_let_fp, const double *move)
{
    orc_init();
    sink_t sk;
    memset(&sk, 0, sizeof sk);
    sk.grid_fp = grid_fp;
    sk.grid_let_fp = grid_let_fp;
    vp_t vp;
    one_history_moved(g, f, sp, spot_index, h, sc, o, &sk, &vp, move);
    for (int l = 0; l < NLEDGER; l++) ledgers[l] = sk.led_fp[l];
    info[0] = vp.n_steps; info[1] = vp.n_nuc; info[2] = vp.nblk; info[3] = 0;
}

/* Start-rounding allowance of the straight-mode comparisons (test support).
 * Entry j names history hist[j] of spot spot[j] and the start moves
 * moves[3*m .. 3*m+2] (mm in the source plane, then MeV of energy; see
 * orc_trace_history) for m in [move_off[j], move_off[j+1]).  The history is
 * transported once as drawn and
 * once per move; per voxel the largest |moved - as drawn| deposit, times the
 * spot's w/N, is added to allow[nvox] (MeV w/N), and likewise the deposit x
 * LET numerator to allow_let[nvox] when that is non-NULL.  In straight mode a
 * history draws no random numbers after its source, so a moved copy is the
 * same history started elsewhere. */
void orc_move_allowance(const orc_geom *g, const orc_field *f, const orc_spot *spots, const orc_scen *sc,
                        const orc_opts *o, int64_t n, const int32_t *spot, const int64_t *hist,
                        const int64_t *move_off, const double *moves, double *allow, double *allow_let,
                        int nthreads)
{
    orc_init();
    const int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    const int want_let = allow_let != NULL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *base = (double *)calloc((size_t)nvox, sizeof(double));
        double *var = (double *)calloc((size_t)nvox, sizeof(double));
        double *worst = (double *)calloc((size_t)nvox, sizeof(double));
        double *base_l = want_let ? (double *)calloc((size_t)nvox, sizeof(double)) : NULL;
        double *var_l = want_let ? (double *)calloc((size_t)nvox, sizeof(double)) : NULL;
        double *worst_l = want_let ? (double *)calloc((size_t)nvox, sizeof(double)) : NULL;
        int64_t *hit = NULL, n_hit = 0, cap_hit = 0;    /* voxels whose worst is set */
        sink_t sb, sv;
        memset(&sb, 0, sizeof sb);
        memset(&sv, 0, sizeof sv);
        sb.track_touch = sv.track_touch = 1;
        if (!base || !var || !worst || (want_let && (!base_l || !var_l || !worst_l))) abort();
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t j = 0; j < n; j++) {
            const orc_spot *sp = &spots[spot[j]];
            vp_t vp;
            sb.grid_fp = base;
            sb.grid_let_fp = base_l;
            sb.n_touch = 0;
            one_history_moved(g, f, sp, spot[j], hist[j], sc, o, &sb, &vp, NULL);
            for (int64_t m = move_off[j]; m < move_off[j + 1]; m++) {
                sv.grid_fp = var;
                sv.grid_let_fp = var_l;
                sv.n_touch = 0;
                one_history_moved(g, f, sp, spot[j], hist[j], sc, o, &sv, &vp, moves + 3 * m);
                /* voxels reached by either copy */
                for (int pass = 0; pass < 2; pass++) {
                    const int64_t *t = pass ? sv.touch : sb.touch;
                    const int64_t nt = pass ? sv.n_touch : sb.n_touch;
                    for (int64_t i = 0; i < nt; i++) {
                        const int64_t v = t[i];
                        const double d = fabs(var[v] - base[v]);
                        const double dl = want_let ? fabs(var_l[v] - base_l[v]) : 0.0;
                        if ((d > 0.0 || dl > 0.0) && worst[v] == 0.0 && (!want_let || worst_l[v] == 0.0)) {
                            if (n_hit == cap_hit) {
                                cap_hit = cap_hit ? 2 * cap_hit : 1024;
                                hit = (int64_t *)realloc(hit, (size_t)cap_hit * sizeof(int64_t));
                                if (!hit) abort();
                            }
                            hit[n_hit++] = v;
                        }
                        if (d > worst[v]) worst[v] = d;
                        if (want_let && dl > worst_l[v]) worst_l[v] = dl;
                    }
                }
                for (int64_t i = 0; i < sv.n_touch; i++) {
                    var[sv.touch[i]] = 0.0;
                    if (want_let) var_l[sv.touch[i]] = 0.0;
                }
            }
            const double w = sp->weight / (double)sp->nh;
            for (int64_t i = 0; i < n_hit; i++) {
                const int64_t v = hit[i];
                const double a = w * worst[v];
#ifdef _OPENMP
#pragma omp atomic
#endif
                allow[v] += a;
                if (want_let) {
                    const double al = w * worst_l[v];
#ifdef _OPENMP
#pragma omp atomic
#endif
                    allow_let[v] += al;
                    worst_l[v] = 0.0;
                }
                worst[v] = 0.0;
            }
            n_hit = 0;
            for (int64_t i = 0; i < sb.n_touch; i++) {
                base[sb.touch[i]] = 0.0;
                if (want_let) base_l[sb.touch[i]] = 0.0;
            }
        }
        free(sb.touch); free(sv.touch); free(hit);
        free(base); free(var); free(worst); free(base_l); free(var_l); free(worst_l);
    }
}

/* Exit states of histories 0 .. n-1 of one spot through the whole path
 * (source, beam line, voxel loop), for the lateral-spread pins of the voxel
 * transport: out[n][8] = {1 if the VP left the grid through a face (0 if it
 * stopped or missed it), E, x, y, z (CT frame, mm), u, v, w}.  With the
 * grid's downstream face at depth L, a pencil beam's exit moments are the
 * Fermi-Eyges moments of the scattering power along its path. */
void orc_patient_exit(const orc_geom *g, const orc_field *f, const orc_spot *sp, int spot_index, int64_t n,
                      const orc_scen *sc, const orc_opts *o, double *out, int nthreads)
{
    orc_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t h = 0; h < n; h++) {
        sink_t sk;
        vp_t vp;
        memset(&sk, 0, sizeof sk);
        one_history(g, f, sp, spot_index, h, sc, o, &sk, &vp);
        double *q = out + 8 * h;
        q[0] = (vp.E > 0.0 && sk.led_fp[L_ESCAPED] > 0.0) ? 1.0 : 0.0;
        q[1] = vp.E;
        for (int k = 0; k < 3; k++) { q[2 + k] = vp.p[k]; q[5 + k] = vp.d[k]; }
    }
}

/* Thin-slab experiment for the physics pins: n VPs of energy e0 enter a slab
 * of material m (density rho, thickness L mm) at normal incidence and are
 * transported by the range-shifter routine.  out[n][8] = {exited, E, x, y,
 * u, v, w, nuclear events}. */
void orc_slab_exit(int m, double rho, double L, double e0, int physics, uint64_t seed, int64_t n,
                   double *out, int nthreads)
{
    orc_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; i++) {
        vp_t vp;
        sink_t sk;
        memset(&vp, 0, sizeof vp);
        memset(&sk, 0, sizeof sk);
        vp.key[0] = (uint32_t)seed; vp.key[1] = (uint32_t)(seed >> 32);
        vp.hist = (uint32_t)i; vp.spot = 0; vp.nblk = 1; vp.physics = physics;
        vp.p[0] = vp.p[1] = 0.0; vp.p[2] = -L;
        vp.d[0] = vp.d[1] = 0.0; vp.d[2] = 1.0;
        vp.E = e0;
        int ex = slab_transport(&vp, &sk, m, rho, -L, 0.0, L_RS);
        double *o = out + 8 * i;
        o[0] = ex == EX_DOWN; o[1] = vp.E; o[2] = vp.p[0]; o[3] = vp.p[1];
        o[4] = vp.d[0]; o[5] = vp.d[1]; o[6] = vp.d[2]; o[7] = vp.n_nuc;
    }
}

/* distance from (x, y) to the polygon's boundary (point-to-segment minimum) */
double orc_polygon_distance(const double *poly, int nv, double x, double y)
{
    double best = INFINITY;
    for (int i = 0, j = nv - 1; i < nv; j = i++) {
        double ax = poly[2 * j], ay = poly[2 * j + 1];
        double ex = poly[2 * i] - ax, ey = poly[2 * i + 1] - ay;
        double wx = x - ax, wy = y - ay, l2 = ex * ex + ey * ey;
        double t = l2 > 0.0 ? (wx * ex + wy * ey) / l2 : 0.0;
        t = t < 0.0 ? 0.0 : t > 1.0 ? 1.0 : t;
        double dx = wx - t * ex, dy = wy - t * ey, d2 = dx * dx + dy * dy;
        if (d2 < best) best = d2;
    }
    return sqrt(best);
}

/* One plain traversal of the field's block per entry state (the surrogate's
 * training data): entries[n][5] = (x, y) on the block's upstream face, (u, v)
 * direction cosines, E.  Streams: key (seed, field id), counter (block, i,
 * 0, 0).  out[n][8] = {outcome: 1 transmitted, 0 stopped or lost, -1 entered
 * through the opening; E_out; u', v', w'; x', y' on the downstream face;
 * distance of the entry point to the opening's edge}. */
void orc_block_traverse(const orc_field *f, const double *entries, int64_t n, uint64_t seed, int field_id,
                        int physics, double *out, int nthreads)
{
    orc_init();
    double zu = -(f->blk_d + f->blk_t), zd = -f->blk_d;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; i++) {
        const double *e = entries + 5 * i;
        double *o = out + 8 * i;
        vp_t vp;
        sink_t sk;
        memset(&vp, 0, sizeof vp);
        memset(&sk, 0, sizeof sk);
        vp.key[0] = (uint32_t)(seed & 0xffffffffu);
        vp.key[1] = (uint32_t)(seed >> 32) ^ (uint32_t)field_id;
        vp.hist = (uint32_t)i;
        vp.physics = physics;
        vp.p[0] = e[0]; vp.p[1] = e[1]; vp.p[2] = zu;
        vp.d[0] = e[2]; vp.d[1] = e[3];
        vp.d[2] = sqrt(fmax(1.0 - e[2] * e[2] - e[3] * e[3], 0.0));
        vp.E = e[4];
        double su = blk_scale(f, zu);
        o[7] = f->nv >= 3 ? su * orc_polygon_distance(f->poly, f->nv, e[0] / su, e[1] / su) : 1000.0;
        if (f->nv >= 3 && orc_in_polygon(f->poly, f->nv, e[0] / su, e[1] / su)) {
            o[0] = -1.0;
            continue;
        }
        int ex = block_transport(&vp, &sk, f, zu, zd);
        o[0] = ex == EX_DOWN ? 1.0 : 0.0;
        o[1] = vp.E; o[2] = vp.d[0]; o[3] = vp.d[1]; o[4] = vp.d[2]; o[5] = vp.p[0]; o[6] = vp.p[1];
    }
}

/* Largest fixed-point exponent k <= 40 with T * 2^k <= 2^62, where T bounds
 * the weighted energy any voxel or ledger can receive. */
int orc_fixed_point_k(double T)
{
    int k = 40;
    while (k > 0 && T * ldexp(1.0, k) > ldexp(1.0, 62)) k--;
    return k;
}

/* physical thickness (mm) of a PMMA range shifter of the given water-
 * equivalent thickness, from the CSDA ranges at 150 MeV (reading R10) */
double orc_rs_thickness(double wet_mm)
{
    orc_init();
    double rw = orc_range(M_WATER, 150.0), rp = orc_range(M_PMMA, 150.0);
    return wet_mm * (rp / MATS[M_PMMA].rho) / (rw / MATS[M_WATER].rho);
}

double orc_mev_to_joule(void) { return MEV_TO_J; }

/* One VP through the block from p (on its upstream face) along d with energy
 * E: out = [1 if it left through the downstream face, E, x, y, z, path length
 * inside brass].  Test support for the geometry of the block's walls. */
void orc_block_trace(const orc_field *f, const double *p, const double *d, double E, int physics, uint64_t seed,
                     double *out)
{
    orc_init();
    double zu = -(f->blk_d + f->blk_t), zd = -f->blk_d;
    vp_t vp;
    sink_t sk;
    memset(&vp, 0, sizeof vp);
    memset(&sk, 0, sizeof sk);
    vp.key[0] = (uint32_t)(seed & 0xffffffffu);
    vp.key[1] = (uint32_t)(seed >> 32);
    vp.physics = physics;
    for (int k = 0; k < 3; k++) { vp.p[k] = p[k]; vp.d[k] = d[k]; }
    vp.p[2] = zu;
    vp.E = E;
    int ex = block_transport(&vp, &sk, f, zu, zd);
    out[0] = ex == EX_DOWN; out[1] = vp.E; out[2] = vp.p[0]; out[3] = vp.p[1]; out[4] = vp.p[2];
    out[5] = vp.brass_path;
}
