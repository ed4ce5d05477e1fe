// gfx950 kernels of the virtual-particle (VP) transport.
//
// One lane carries one VP history at a time (Methods A: every VP, primary or
// secondary, follows the same model, so lanes of a wavefront run the same
// code).  Per launch each workgroup stages the 32 KiB of physics tables and
// the aperture polygon in LDS.  The step loop is FP32; the VP energy is kept
// as an unevaluated FP32 pair so per-step losses telescope without drift;
// every deposit is converted to int64 fixed point and added with a 64-bit
// atomic, which makes the tally independent of execution order.
#include <math.h>

#include <mutex>

#include "vpmc_internal.hpp"

namespace vpmc {
namespace {

constexpr float kELo = 1.0f;
constexpr float kSegPerLog2 = (float)(NE - 1) / 8.0f;   // E_HI / E_LO = 2^8
constexpr int kThreads = 256;

// ------------------------------------------------------------ random numbers
// Philox4x32-10 (Salmon et al., SC'11); counter (block, history, spot, 0),
// key (seed_lo, seed_hi ^ field).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // full 64-bit products (one v_mad_u64_u32 each)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

// top 23 bits + 1/2, times 2^-23: exact in FP32, strictly inside (0, 1)
__device__ __forceinline__ float unit_open(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

struct Lane {
    float px, py, pz, dx, dy, dz;
    float pzlo;               // low part of the depth (slab depth, or voxel-local z)
    float pxlo, pylo;         // low parts of the voxel-local x, y (patient only)
    float E, Elo;             // energy as an unevaluated pair E + Elo
    uint32_t nblk, spot, hist, k0, k1;
    unsigned physics;
    uint32_t nsteps;
};

// ---------------------------------------------------- double-float values
// An unevaluated FP32 pair h + l with |l| <= ulp(h)/2, built from error-free
// transformations: Knuth's TwoSum, Dekker's Fast2Sum (|a| >= |b| or a = 0)
// and the FMA-based exact product.  The CSDA bookkeeping (energy, residual
// range, path lengths, densities) runs on pairs, so a track's energy does not
// drift by FP32 rounding step after step; the drift would otherwise reach the
// residual deposit at the end of range amplified by S(E_end)/S(E_start).
struct DF {
    float h, l;
};

__device__ __forceinline__ DF fast2(float a, float b) {
    const float s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ DF two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DF df_add(DF a, DF b) {
    const DF s = two_sum(a.h, b.h);
    return fast2(s.h, s.l + (a.l + b.l));
}

__device__ __forceinline__ DF df_sub(DF a, DF b) { return df_add(a, {-b.h, -b.l}); }

__device__ __forceinline__ DF df_mul(DF a, DF b) {
    const float p = a.h * b.h;
    const float e = fmaf(a.h, b.h, -p) + (a.h * b.l + a.l * b.h);
    return fast2(p, e);
}

__device__ __forceinline__ DF df_mul_f(DF a, float b) {
    const float p = a.h * b;
    return fast2(p, fmaf(a.l, b, fmaf(a.h, b, -p)));
}

// a / b: FP32 quotient, then one correction from the exact remainder
__device__ __forceinline__ DF df_div(DF a, DF b) {
    const float rb = __builtin_amdgcn_rcpf(b.h);
    const float q = a.h * rb;
    const DF r = df_sub(a, df_mul_f(b, q));
    return fast2(q, (r.h + r.l) * rb);
}

__device__ __forceinline__ bool df_le(DF a, DF b) { return a.h < b.h || (a.h == b.h && a.l <= b.l); }

__device__ __forceinline__ uint4 draw(Lane &v) {
    const uint4 w = philox4x32_10(make_uint4(v.nblk, v.hist, v.spot, 0u), v.k0, v.k1);
    v.nblk++;
    return w;
}

// Sampling arithmetic of the physics steps uses the hardware square root
// (about 1 ulp); the straight-mode bookkeeping never calls it.
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// step normals: hardware sin/cos take the angle in turns
__device__ __forceinline__ void box_muller_fast(uint32_t a, uint32_t b, float &z1, float &z2) {
    const float r = sqrt_hw(-2.0f * __logf(unit_open(a)));
    const float t = unit_open(b);
    z1 = r * __builtin_amdgcn_cosf(t);
    z2 = r * __builtin_amdgcn_sinf(t);
}

// ------------------------------------------------------------ table lookups
// segment i with E_i <= E < E_i+1, clamped to [0, NE-2]
__device__ __forceinline__ int seg_of(const float *tab, float E) {
    int i = (int)(__log2f(fmaxf(E, kELo)) * kSegPerLog2);
    i = min(max(i, 0), NE - 2);
    while (i > 0 && E < tab[TAB_E + i]) --i;
    while (i < NE - 2 && E >= tab[TAB_E + i + 1]) ++i;
    return i;
}

// position of E on the node grid: segment and clamped fraction, shared by
// every table interpolated at the same energy (linear in E between nodes)
struct NodePos {
    int i;
    float f;
};

// position of an energy E < E_i+1 known to lie at or below segment i (the
// search walks down from i to the unique segment with E_j <= E < E_j+1)
__device__ __forceinline__ NodePos node_pos_below(const float *tab, float E, int i) {
    while (i > 0 && E < tab[TAB_E + i]) --i;
    const float f = (E - tab[TAB_E + i]) * __builtin_amdgcn_rcpf(tab[TAB_DWH + i]);
    return {i, fminf(fmaxf(f, 0.0f), 1.0f)};
}

// Standard normal quantile of u in (0, 1), z = sqrt(2) erfinv(2u - 1), for
// the straggling draw.  The structure is M. Giles' single-precision erfinv
// ("Approximating the erfinv function", GPU Computing Gems Jade Edition,
// 2011): with w = -log(1 - t^2) = -log(4u(1 - u)), erfinv(t)/t is a
// polynomial in w - 2.5 for w < 5 and in sqrt(w) - 3 above.  The degree-8
// coefficients are this library's own weighted least-squares fits to the FP64
// function (gen_quantile.py), largest relative error 2.7e-7 over the uniform
// grid u = (k + 1/2) 2^-23.
__device__ __forceinline__ float normal_quantile(float u) {
    const float t = 2.0f * u - 1.0f;
    const float w = -__logf(4.0f * u * (1.0f - u));
    float p;
    if (w < 5.0f) {   // central part (all but 0.34 % of the draws)
        const float s1 = w - 2.5f;
        float a = 2.798955610e-08f;
        a = fmaf(a, s1, 3.430734327e-07f);
        a = fmaf(a, s1, -3.522236486e-06f);
        a = fmaf(a, s1, -4.389634286e-06f);
        a = fmaf(a, s1, 2.185773789e-04f);
        a = fmaf(a, s1, -1.253729840e-03f);
        a = fmaf(a, s1, -4.177678720e-03f);
        a = fmaf(a, s1, 2.466407436e-01f);
        p = fmaf(a, s1, 1.501409417e+00f);
    } else {
        const float s2 = sqrt_hw(w) - 3.0f;
        float b = -2.393541571e-04f;
        b = fmaf(b, s2, 1.079666834e-04f);
        b = fmaf(b, s2, 1.402476381e-03f);
        b = fmaf(b, s2, -3.678024843e-03f);
        b = fmaf(b, s2, 5.716959691e-03f);
        b = fmaf(b, s2, -7.622124629e-03f);
        b = fmaf(b, s2, 9.441883054e-03f);
        b = fmaf(b, s2, 1.001674163e+00f);
        p = fmaf(b, s2, 2.832976859e+00f);
    }
    return 1.41421356237f * p * t;
}

// 1 - exp(-x) for x >= 0 (nuclear removal over a step): the series to x^5
// below 1/8 (truncation below x^6/720), else through exp
__device__ __forceinline__ float one_minus_exp_neg(float x) {
    if (x < 0.125f) return x * (1.0f - x * (0.5f - x * (0.16666667f - x * (0.041666668f - x * 0.0083333338f))));
    return 1.0f - __expf(-x);
}

__device__ __forceinline__ float node_lerp(const float *y, NodePos p) {
    return fmaf(p.f, y[p.i + 1] - y[p.i], y[p.i]);
}

// Energy lost while traversing r (density x mm), starting at E = E_i + x in
// segment i of the piecewise-linear CSDA relation E(R), whose range within
// the segment is rem = x / slope_i.  Whole segments crossed contribute their
// exact energy width; the last partial segment r * slope_j.  All in pairs.


__device__ __forceinline__ void rotate_dir(Lane &v, float ax, float ay) {
    const float th2 = ax * ax + ay * ay;
    if (th2 == 0.0f) return;
    const float sg = copysignf(1.0f, v.dz);
    const float a = -__builtin_amdgcn_rcpf(sg + v.dz);
    const float b = v.dx * v.dy * a;
    const float e1x = 1.0f + sg * v.dx * v.dx * a, e1y = sg * b, e1z = -sg * v.dx;
    const float e2x = b, e2y = sg + v.dy * v.dy * a, e2z = -v.dy;
    // cos(th) and sin(th)/th: series in th^2 below th^2 = 0.01 (multiple
    // scattering per step; truncation below 3e-10), else from sin and cos
    float c, k;
    if (th2 < 0.01f) {
        c = 1.0f - th2 * (0.5f - th2 * (0.041666668f - th2 * 0.0013888889f));
        k = 1.0f - th2 * (0.16666667f - th2 * (0.0083333338f - th2 * 0.00019841270f));
    } else {
        const float th = sqrt_hw(th2);
        float sn;
        __sincosf(th, &sn, &c);
        k = sn * __builtin_amdgcn_rcpf(th);
    }
    float nx = c * v.dx + k * (ax * e1x + ay * e2x);
    float ny = c * v.dy + k * (ax * e1y + ay * e2y);
    float nz = c * v.dz + k * (ax * e1z + ay * e2z);
    const float inv = rsqrtf(nx * nx + ny * ny + nz * nz);
    v.dx = nx * inv;
    v.dy = ny * inv;
    v.dz = nz * inv;
}




enum { ST_STOP = 0, ST_GEO = 1, ST_INNER = 2 };

__device__ __forceinline__ DF df_div_f(DF a, float b) {
    const float rb = __builtin_amdgcn_rcpf(b);
    const float q = a.h * rb;
    const DF r = df_sub(a, df_mul_f({q, 0.0f}, b));
    return fast2(q, (r.h + r.l) * rb);
}

// 1/b to within about half an ulp: hardware estimate and one Newton step
// (the raw estimate's error has a fixed sign)
__device__ __forceinline__ float rcp_nr(float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    return fmaf(r, fmaf(-b, r, 1.0f), r);
}

// Arithmetic of the two transport instantiations.  Exact (deterministic
// mode, checked against the FP64 reference to 1e-5 per voxel): double-float
// pairs.  Physics mode: plain FP32 on the high parts, the low parts constant
// zero and folded away; the per-step losses carry the straggling noise, next
// to which FP32 rounding is immaterial.
template <bool X>
struct Ar;

template <>
struct Ar<true> {
    static __device__ __forceinline__ DF pair(float h, float l) { return {h, l}; }
    static __device__ __forceinline__ DF add(DF a, DF b) { return df_add(a, b); }
    static __device__ __forceinline__ DF sub(DF a, DF b) { return df_sub(a, b); }
    static __device__ __forceinline__ DF mul(DF a, DF b) { return df_mul(a, b); }
    static __device__ __forceinline__ DF mul_f(DF a, float b) { return df_mul_f(a, b); }
    static __device__ __forceinline__ DF div(DF a, DF b) { return df_div(a, b); }
    static __device__ __forceinline__ DF div_f(DF a, float b) { return df_div_f(a, b); }
    static __device__ __forceinline__ bool le(DF a, DF b) { return df_le(a, b); }
};

template <>
struct Ar<false> {
    static __device__ __forceinline__ DF pair(float h, float) { return {h, 0.0f}; }
    static __device__ __forceinline__ DF add(DF a, DF b) { return {a.h + b.h, 0.0f}; }
    static __device__ __forceinline__ DF sub(DF a, DF b) { return {a.h - b.h, 0.0f}; }
    static __device__ __forceinline__ DF mul(DF a, DF b) { return {a.h * b.h, 0.0f}; }
    static __device__ __forceinline__ DF mul_f(DF a, float b) { return {a.h * b, 0.0f}; }
    static __device__ __forceinline__ DF div(DF a, DF b) { return {a.h * rcp_nr(b.h), 0.0f}; }
    static __device__ __forceinline__ DF div_f(DF a, float b) { return {a.h * rcp_nr(b), 0.0f}; }
    static __device__ __forceinline__ bool le(DF a, DF b) { return a.h <= b.h; }
};

// move by the path length h along d: the depth as a pair; in the patient
// (voxel-local frame) x and y as pairs too, in a slab plain FP32
template <bool Slab, bool X>
__device__ __forceinline__ void move(Lane &v, DF h) {
    using A = Ar<X>;
    const DF z = A::add(A::pair(v.pz, v.pzlo), A::mul_f(h, v.dz));
    v.pz = z.h;
    v.pzlo = z.l;
    if (Slab || !X) {
        v.px = fmaf(h.h, v.dx, v.px);
        v.py = fmaf(h.h, v.dy, v.py);
    } else {
        const DF x = df_add({v.px, v.pxlo}, df_mul_f(h, v.dx));
        const DF y = df_add({v.py, v.pylo}, df_mul_f(h, v.dy));
        v.px = x.h;
        v.pxlo = x.l;
        v.py = y.h;
        v.pylo = y.l;
    }
}

// (E, Elo) -= dE: exact pair arithmetic, or in physics mode the FP32 loss
// compensated into the pair (so the energy still telescopes)
template <bool X>
__device__ __forceinline__ void sub_energy(Lane &v, DF dE) {
    const DF e = df_sub({v.E, v.Elo}, X ? dE : DF{dE.h, 0.0f});
    v.E = e.h;
    v.Elo = e.l;
}

// tm: the material's high tables, tl: its low tables (read only when X)
template <bool X>
__device__ __forceinline__ DF csda_loss(const float *tab, const float *tm, const float *tl, int i, DF x, DF rem,
                                        DF r) {
    using A = Ar<X>;
    if (A::le(r, rem)) return A::mul(r, A::pair(tm[T_SH * NE + i], X ? tl[L_SL * NE + i] : 0.0f));
    DF dE = x;
    r = A::sub(r, rem);
    for (int j = i - 1; j >= 0; --j) {
        const DF dRj = A::pair(tm[T_DH * NE + j], X ? tl[L_DL * NE + j] : 0.0f);
        if (A::le(r, dRj)) return A::add(dE, A::mul(r, A::pair(tm[T_SH * NE + j], X ? tl[L_SL * NE + j] : 0.0f)));
        dE = A::add(dE, A::pair(tab[TAB_DWH + j], X ? tab[TAB_DWL + j] : 0.0f));
        r = A::sub(r, dRj);
    }
    return dE;
}

// One condensed-history step in a homogeneous region: CSDA loss from the
// range table, Bohr straggling, Gaussian multiple scattering applied at the
// step midpoint (hinge), nuclear removal turning the VP into its leading
// secondary.  rho_loss scales energy loss and straggling (range scenarios),
// rho scattering and nuclear removal.  dg: distance to the region boundary.
// Energy, residual range, path and density are pairs (double-float); the
// decisions (range-out, step length) and the physics sampling use FP32.
// let: the step's LET in MeV/mm (= keV/um) for the dose-averaged LET tally:
// the mean CSDA stopping power over the step (dE_csda / s); for a VP that
// stops, its energy over its residual path (E rho / R); at the cut-off, the
// slope of the CSDA relation's first segment times the density.
template <bool Slab, bool X>
__device__ int phys_step(Lane &v, const float *tab, int m, DF rho_loss, float rho, DF dg, float &dep,
                         float &esc, float &let) {
    using A = Ar<X>;
    dep = 0.0f;
    esc = 0.0f;
    let = 0.0f;
    v.nsteps++;
    const float *tm = tab + TAB_MAT0 + m * TAB_PER_MAT;
    if (v.E + v.Elo <= kELo) {
        let = rho_loss.h * tm[T_SH * NE];
        dep = v.E + v.Elo;
        v.E = v.Elo = 0.0f;
        return ST_STOP;
    }
    const float *tl = tab + TAB_LMAT0 + m * TAB_PER_LMAT;
    int i = seg_of(tab, v.E);
    // E - E_i: the high parts subtract exactly (same binade), the low parts add
    DF x = X ? two_sum(v.E - tab[TAB_E + i], v.Elo - tab[TAB_EL + i])
             : DF{(v.E - tab[TAB_E + i]) + v.Elo, 0.0f};
    if (x.h < 0.0f && i > 0) {
        --i;
        x = X ? two_sum(v.E - tab[TAB_E + i], v.Elo - tab[TAB_EL + i])
              : DF{(v.E - tab[TAB_E + i]) + v.Elo, 0.0f};
    }
    const DF S = A::pair(tm[T_SH * NE + i], X ? tl[L_SL * NE + i] : 0.0f);
    const DF rem = A::div(x, S);
    const float R = tm[T_R * NE + i] + rem.h;
    if (rho_loss.h * dg.h >= R) {
        let = (v.E + v.Elo) * rho_loss.h * __builtin_amdgcn_rcpf(R);
        dep = v.E + v.Elo;
        v.E = v.Elo = 0.0f;
        return ST_STOP;
    }
    const float smax = STEP_FRACTION * R * __builtin_amdgcn_rcpf(rho_loss.h);
    const bool geo = dg.h <= smax;
    const DF s = geo ? dg : DF{smax, 0.0f};
    const DF r = A::mul(rho_loss, s);   // density x mm (the tables' unit)
    DF dE = csda_loss<X>(tab, tm, tl, i, x, rem, r);
    if (s.h > 0.0f) let = (dE.h + dE.l) / (s.h + s.l);
    const float Ebar = v.E - 0.5f * dE.h;
    uint4 w = make_uint4(0u, 0u, 0u, 0xFFFFFFFFu);
    NodePos pb{0, 0.0f};
    if (v.physics) {
        w = draw(v);
        pb = node_pos_below(tab, Ebar, i);
    }
    if (v.physics & PH_STRAGGLE) {
        const float var = r.h * node_lerp(tm + T_W2 * NE, pb);
        const float z = normal_quantile(unit_open(w.z));
        dE = A::add(dE, {-(sqrt_hw(var) * z), 0.0f});
        const float tot = v.E + v.Elo;
        if (!(dE.h + dE.l > 0.0f)) dE = {0.0f, 0.0f};
        else if (dE.h + dE.l > tot) dE = {v.E, v.Elo};
    }
    dep = dE.h + dE.l;
    sub_energy<X>(v, dE);
    if (v.physics & PH_MCS) {
        const float th0 = sqrt_hw(rho * s.h * node_lerp(tm + T_T * NE, pb));
        float z1, z2;
        box_muller_fast(w.x, w.y, z1, z2);
        const DF h = {0.5f * s.h, 0.5f * s.l};
        move<Slab, X>(v, h);
        rotate_dir(v, th0 * z1, th0 * z2);
        move<Slab, X>(v, h);
    } else {
        move<Slab, X>(v, s);
    }
    if (v.physics & PH_NUCLEAR) {
        const float P = one_minus_exp_neg(rho * s.h * node_lerp(tm + T_SN * NE, pb));
        if (unit_open(w.w) < P) {
            const uint4 w2 = draw(v);
            const float E1 = v.E + v.Elo;
            const float loc = NUC_F_LOCAL * E1, out = NUC_F_ESCAPE * E1;
            v.E = (E1 - loc) - out;
            v.Elo = 0.0f;
            dep += loc;
            esc = out;
            float n1, n2;
            box_muller_fast(w2.x, w2.y, n1, n2);
            rotate_dir(v, NUC_SIGMA_RAD * n1, NUC_SIGMA_RAD * n2);
        }
    }
    return geo ? ST_GEO : ST_INNER;
}

// ------------------------------------------------------------ tallies
struct Acc {
    long long led[NLEDGER];
    unsigned long long steps, hist;
};

__device__ __forceinline__ long long to_fixed(float e, float scale) {
    return (long long)rintf(e * scale);
}

__device__ __forceinline__ void ledger_add(Acc &a, int j, float e, float scale) {
    a.led[j] += to_fixed(e, scale);
}

// dense tally: one 64-bit atomic per deposit
struct DenseSink {
    unsigned long long *tally;
    unsigned long long *let = nullptr;   // dose-averaged LET numerator, or none
    static constexpr bool kLet = true;
    __device__ __forceinline__ void add_let(uint32_t v, long long q) const {
        atomicAdd(let + v, (unsigned long long)q);
    }
    __device__ __forceinline__ void add(uint32_t v, const int *, long long q) const {
        atomicAdd(tally + v, (unsigned long long)q);
    }
};

// per-row tally of the influence-matrix builder: a non-returning 64-bit
// atomic into the row's dense slot grid and a store of 1 into the
// touched-block byte map (one byte per 32 voxels).  Every writer stores the
// same value and the marks are read only by later kernels, so the store is
// relaxed at workgroup scope: it stays in L2 (write-back, merged per line)
// instead of being written through to memory on every step.
struct SparseSink {
    unsigned long long *grid;
    uint8_t *mark;
    static constexpr bool kLet = false;
    unsigned long long *let = nullptr;
    __device__ __forceinline__ void add_let(uint32_t, long long) const {}
    __device__ __forceinline__ void add(uint32_t v, const int *, long long q) const {
        put(v, q);
    }
    __device__ __forceinline__ void put(uint32_t v, long long q) const {
        atomicAdd(grid + v, (unsigned long long)q);
        __hip_atomic_store(mark + (v >> 5), (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

// Row tile of the influence-matrix builder: a dense int64 box of the CT grid
// in LDS around the spot's central ray, shared by the waves of a workgroup
// that work on the same row.  Deposits inside the box are LDS atomics, the
// others go to the row's slot grid; the box is added into the slot grid once
// when its last user leaves.  On this GPU the int64 tally atomics to device
// memory are performed on the memory side, beyond the XCD's L2, and their
// rate bounds the step loop; the tile takes most of them off that path.
struct TileSink {
    long long *tile;     // nullptr: this batch does not use the tile
    int lo0, lo1, lo2;
    uint32_t n0, n1, n2;
    SparseSink gs;
    unsigned long long *let = nullptr;   // (no LET tally in influence matrices)
    static constexpr bool kLet = false;
    __device__ __forceinline__ void add_let(uint32_t, long long) const {}
    __device__ __forceinline__ void add(uint32_t v, const int *idx, long long q) const {
        if (tile) {
            const uint32_t u0 = (uint32_t)(idx[0] - lo0), u1 = (uint32_t)(idx[1] - lo1), u2 = (uint32_t)(idx[2] - lo2);
            if (u0 < n0 && u1 < n1 && u2 < n2) {
                atomicAdd(reinterpret_cast<unsigned long long *>(tile) + (u0 + n0 * (u1 + n1 * u2)),
                          (unsigned long long)q);
                return;
            }
        }
        gs.put(v, q);
    }
};

// ------------------------------------------------------------ aperture
// crossing number (ray casting) with the half-open rule
__device__ __forceinline__ bool in_polygon(const float2 *poly, int nv, float x, float y) {
    bool c = false;
    float2 b = poly[nv - 1];
    for (int i = 0; i < nv; ++i) {
        const float2 a = poly[i];
        if ((a.y > y) != (b.y > y)) {
            const float xc = a.x + (y - a.y) * (b.x - a.x) / (b.y - a.y);
            if (x < xc) c = !c;
        }
        b = a;
    }
    return c;
}

// Conservative distance from (x, y) to the aperture polygon's boundary, read
// from the field's distance raster: the stored distance at the cell centre
// less the farthest a point of the cell can be from it (distances are
// 1-Lipschitz).  Returns 0 when the point may lie near the boundary (the
// exact edge loops then decide) and sets `inside` when the bound is > 0.
__device__ __forceinline__ float sdf_bound(const FieldDev &f, float x, float y, bool &inside) {
    inside = false;
    if (!f.sdf || !(x == x) || !(y == y)) return 0.0f;
    const float fx = (x - f.sdf_x0) * f.sdf_ih, fy = (y - f.sdf_y0) * f.sdf_ih;
    if (!(fx >= 0.0f && fy >= 0.0f && fx < (float)f.sdf_nx && fy < (float)f.sdf_ny)) return f.sdf_far;
    const float d = f.sdf[(int)fy * f.sdf_nx + (int)fx];
    inside = d > 0.0f;
    return fmaxf(fabsf(d) - f.sdf_r, 0.0f);
}

// true when a BEV ray of lateral speed `lat` cannot reach the boundary within
// path length t, with room for the FP32 rounding of the exact edge distance
__device__ __forceinline__ bool no_edge_within(float lb, float lat, float t) {
    return lb > 0.0f && lat * t < lb * (1.0f - 1e-5f) - 1e-4f;
}

// The exact side of (x, y) and the path length along (u, v) to the first
// edge, from the edges listed for the point's raster cell (non-divergent
// block): the cell's reference point has a known side, each listed edge that
// the segment from it to (x, y) crosses flips the side (half-open
// orientation tests), and no unlisted edge lies within list_reach of (x, y).
// Returns 0 (the caller takes the loops over every edge) when the cell has
// no reference point, 1 when te is the exact first-edge distance or the
// caller's path length t ends before any edge, and 2 when only the side is
// known: the first listed hit and t both lie beyond list_reach laterally
// (lat = |(u, v)|), so an unlisted edge may come first and the caller takes
// the loop over every edge for te.  A listed hit within list_reach is the
// first hit: an earlier one would lie closer to (x, y), so on a listed edge.
// Each listed edge's crossing arithmetic is edge_distance's.
__device__ __forceinline__ int listed_edges(const FieldDev &f, const float2 *poly, int nv, float x, float y,
                                            float u, float v, float lat, float t, bool &inside, float &te) {
    if (!f.cell_off) return 0;
    const float fx = (x - f.sdf_x0) * f.sdf_ih, fy = (y - f.sdf_y0) * f.sdf_ih;
    if (!(fx >= 0.0f && fy >= 0.0f && fx < (float)f.sdf_nx && fy < (float)f.sdf_ny)) return 0;
    const int cell = (int)fy * f.sdf_nx + (int)fx;
    const uint32_t o0 = f.cell_off[cell], o1 = f.cell_off[cell + 1] & 0x3fffffffu;
    if (!(o0 & 0x40000000u)) return 0;
    const float2 r = f.cell_ref[cell];
    bool in = (o0 & 0x80000000u) != 0u;
    float best = INFINITY;
    const float sx = x - r.x, sy = y - r.y;
    for (uint32_t k = o0 & 0x3fffffffu; k < o1; ++k) {
        const int e = f.cell_edge[k];
        const float2 a = poly[e], b = poly[e + 1 < nv ? e + 1 : 0];
        const float ex = b.x - a.x, ey = b.y - a.y;
        const float o_r = ex * (r.y - a.y) - ey * (r.x - a.x);
        const float o_p = ex * (y - a.y) - ey * (x - a.x);
        const float o_a = sx * (a.y - r.y) - sy * (a.x - r.x);
        const float o_b = sx * (b.y - r.y) - sy * (b.x - r.x);
        if ((o_r > 0.0f) != (o_p > 0.0f) && (o_a > 0.0f) != (o_b > 0.0f)) in = !in;
        const float den = u * ey - v * ex;
        if (den != 0.0f) {
            const float wx = a.x - x, wy = a.y - y;
            const float inv = 1.0f / den;
            const float th = (wx * ey - wy * ex) * inv;
            const float lam = (wx * v - wy * u) * inv;
            if (th > 0.0f && lam >= 0.0f && lam <= 1.0f) best = fminf(best, th);
        }
    }
    inside = in;
    te = best;
    return lat * fminf(best, t) <= f.list_reach ? 1 : 2;
}

// path length along (u, v) until the beam's-eye-view ray from (x, y) meets an
// edge (a non-divergent block)
__device__ __forceinline__ float edge_distance(const float2 *poly, int nv, float x, float y, float u,
                                               float v) {
    float best = INFINITY;
    float2 a = poly[nv - 1];
    for (int i = 0; i < nv; ++i) {
        const float2 b = poly[i];
        const float ex = b.x - a.x, ey = b.y - a.y;
        const float den = u * ey - v * ex;
        if (den != 0.0f) {
            const float wx = a.x - x, wy = a.y - y;
            const float inv = 1.0f / den;
            const float t = (wx * ey - wy * ex) * inv;
            const float lam = (wx * v - wy * u) * inv;
            if (t > 0.0f && lam >= 0.0f && lam <= 1.0f) best = fminf(best, t);
        }
        a = b;
    }
    return best;
}

// Path length along the ray (x, y) + t (u, v) to the first wall of the block
// (INFINITY if none).  Every wall is the plane through the focus and an edge
// of the polygon: at opening scale s0 (s = s0 + t kw along the ray) the ray
// meets the wall of edge (a, b) where p + t d = s (a + lam (b - a)), linear
// in t.  A non-divergent block has s0 = 1, kw = 0: the beam's-eye-view
// ray-segment intersection.
__device__ __forceinline__ float edge_distance_div(const float2 *poly, int nv, float x, float y, float u,
                                                   float v, float s0, float kw) {
    float best = INFINITY;
    float2 a = poly[nv - 1];
    for (int i = 0; i < nv; ++i) {
        const float2 b = poly[i];
        const float ex = b.x - a.x, ey = b.y - a.y;
        const float ux = u - kw * a.x, uy = v - kw * a.y;
        const float den = ux * ey - uy * ex;
        if (den != 0.0f) {
            const float wx = s0 * a.x - x, wy = s0 * a.y - y;
            const float inv = 1.0f / den;
            const float t = (wx * ey - wy * ex) * inv;
            const float mu = (wx * uy - wy * ux) * inv;
            const float st = fmaf(t, kw, s0);
            if (t > 0.0f && st > 0.0f && mu >= 0.0f && mu <= st) best = fminf(best, t);
        }
        a = b;
    }
    return best;
}

// push the projected position EDGE_PUSH_MM further along the projected
// direction, depth unchanged, across the edge just reached (non-divergent)
__device__ __forceinline__ void edge_push(Lane &v) {
    const float n2 = v.dx * v.dx + v.dy * v.dy;
    if (n2 > 0.0f) {
        const float k = EDGE_PUSH_MM * rsqrtf(n2);
        v.px = fmaf(k, v.dx, v.px);
        v.py = fmaf(k, v.dy, v.py);
    }
}

// edge push in the block: along the scaled position's direction of travel
// d_xy - kw X, which crosses the wall just reached (d_xy for a non-divergent
// block, where kw = 0)
__device__ __forceinline__ void edge_push_blk(Lane &v, const FieldDev &f) {
    const float isc = 1.0f / fmaf(v.pz, f.fs, f.fc0), kw = v.dz * f.fs;
    const float cx = v.dx - kw * (v.px * isc), cy = v.dy - kw * (v.py * isc);
    const float n2 = cx * cx + cy * cy;
    if (n2 > 0.0f) {
        const float k = EDGE_PUSH_MM * rsqrtf(n2);
        v.px = fmaf(k, cx, v.px);
        v.py = fmaf(k, cy, v.py);
    }
}

// Inside a slab (range shifter or block) the depth is kept relative to the
// slab's upstream face as a pair (pz + pzlo) and the thickness is a pair, so
// the path to the exit plane is exact to the pairs' precision rather than to
// FP32 rounding of the step lengths or of the absolute beam-frame depth.
template <bool X>
__device__ __forceinline__ DF plane_distance(const Lane &v, DF thick, bool &down) {
    using A = Ar<X>;
    DF t = {INFINITY, 0.0f};
    down = true;
    if (v.dz > 0.0f) t = A::div_f(A::sub(thick, A::pair(v.pz, v.pzlo)), v.dz);
    else if (v.dz < 0.0f) { down = false; t = A::div_f(A::pair(-v.pz, -v.pzlo), v.dz); }
    return t.h > 0.0f ? t : DF{0.0f, 0.0f};
}

enum { EX_DOWN = 0, EX_GONE = 1 };

// homogeneous slab (range shifter): local depth 0 .. thick; on return the
// depth is the global plane z the VP left through
template <bool X>
__device__ int slab_transport(Lane &v, Acc &acc, float scale, const float *tab, int m, DF rho,
                              float zu, float zd, DF thick, int ledger) {
    v.pz = 0.0f;
    v.pzlo = 0.0f;
    for (int it = 0; it < MAX_STEPS; ++it) {
        bool down;
        const DF tp = plane_distance<X>(v, thick, down);
        float dep, esc;
        float let;
        const int st = phys_step<true, X>(v, tab, m, rho, rho.h, tp, dep, esc, let);
        ledger_add(acc, ledger, dep, scale);
        ledger_add(acc, L_NUC, esc, scale);
        if (st == ST_STOP) return EX_GONE;
        if (st == ST_GEO || v.pz >= thick.h || v.pz <= 0.0f) {
            const bool out_down = (st == ST_GEO) ? down : (v.pz >= thick.h);
            v.pz = out_down ? zd : zu;
            v.pzlo = 0.0f;
            if (out_down) return EX_DOWN;
            ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
            return EX_GONE;
        }
    }
    ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
    return EX_GONE;
}

// Methods B: between the block's entrance and exit planes the crossing
// number at the VP's projected position decides, at every step, opening
// (straight transport, no random numbers) or brass (brass tables).  D = false
// compiles the plain (non-divergent) geometry only; D = true adds the
// divergent block's.  A non-divergent block takes the same code, and so gives
// the same bits, in both.
template <bool X, bool D = true>
__device__ int block_transport(Lane &v, Acc &acc, float scale, const float *tab, const float2 *poly,
                               int nv, float rho_b, float zu, float zd, DF thick, const FieldDev &f_sdf) {
    v.pz = 0.0f;
    v.pzlo = 0.0f;
    for (int it = 0; it < MAX_BLOCK_ITER; ++it) {
        bool down;
        const DF tpp = plane_distance<X>(v, thick, down);
        const float tp = tpp.h;
        bool open = false;
        float te = INFINITY;
        if (nv >= 3 && !(D && f_sdf.div)) {
            bool inside;
            const float lb = sdf_bound(f_sdf, v.px, v.py, inside);
            const float lat = sqrtf(v.dx * v.dx + v.dy * v.dy);
            if (no_edge_within(lb, lat, tp)) {
                open = inside;
            } else {
                const int ls = listed_edges(f_sdf, poly, nv, v.px, v.py, v.dx, v.dy, lat, tp, open, te);
                if (ls == 0) open = in_polygon(poly, nv, v.px, v.py);
                if (ls != 1) te = edge_distance(poly, nv, v.px, v.py, v.dx, v.dy);
            }
        } else if (nv >= 3) {
            // divergent block: opening scale at this depth and its rate of
            // change along the ray
            const float sc = fmaf(v.pz, f_sdf.fs, f_sdf.fc0), kw = v.dz * f_sdf.fs;
            const float isc = 1.0f / sc;
            const float bx = v.px * isc, by = v.py * isc;
            const float cx = v.dx - kw * bx, cy = v.dy - kw * by;
            // far from every edge for the whole path to the exit plane: the
            // side is known and the exact edge distance exceeds tp, so the
            // decisions below are those of the exact loops (the scaled
            // position moves by at most tp |d_xy - kw (bx, by)| / min s)
            bool inside;
            const float lb = sdf_bound(f_sdf, bx, by, inside);
            if (no_edge_within(lb, sqrtf(cx * cx + cy * cy) / fminf(sc, fmaf(tp, kw, sc)), tp)) {
                open = inside;
            } else {
                open = in_polygon(poly, nv, bx, by);
                te = edge_distance_div(poly, nv, v.px, v.py, v.dx, v.dy, sc, kw);
            }
        }
        if (open) {
            if (tp <= te) {
                v.px = fmaf(tp, v.dx, v.px);
                v.py = fmaf(tp, v.dy, v.py);
                v.pz = down ? zd : zu;
                v.pzlo = 0.0f;
                if (down) return EX_DOWN;
                ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
                return EX_GONE;
            }
            move<true, X>(v, {te, 0.0f});
            if constexpr (D) edge_push_blk(v, f_sdf);
            else edge_push(v);
            continue;
        }
        const DF dg = te < tp ? DF{te, 0.0f} : tpp;
        float dep, esc;
        float let;
        const int st = phys_step<true, X>(v, tab, MAT_BRASS, {rho_b, 0.0f}, rho_b, dg, dep, esc, let);
        ledger_add(acc, L_BLOCK, dep, scale);
        ledger_add(acc, L_NUC, esc, scale);
        if (st == ST_STOP) return EX_GONE;
        if (st == ST_GEO && tp <= te) {
            v.pz = down ? zd : zu;
            v.pzlo = 0.0f;
            if (down) return EX_DOWN;
            ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
            return EX_GONE;
        }
        if (st == ST_GEO) {
            if constexpr (D) edge_push_blk(v, f_sdf);
            else edge_push(v);
        }
        if (v.pz >= thick.h) { v.pz = zd; v.pzlo = 0.0f; return EX_DOWN; }
        if (v.pz <= 0.0f) {
            v.pz = zu;
            v.pzlo = 0.0f;
            ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
            return EX_GONE;
        }
    }
    ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
    return EX_GONE;
}

// distance from (x, y) to the polygon's boundary (minimum over edges of the
// point-to-segment distance)
__device__ float dist_to_polygon(const float2 *poly, int nv, float x, float y) {
    float best = INFINITY;
    float2 a = poly[nv - 1];
    for (int i = 0; i < nv; ++i) {
        const float2 b = poly[i];
        const float ex = b.x - a.x, ey = b.y - a.y;
        const float wx = x - a.x, wy = y - a.y;
        const float l2 = ex * ex + ey * ey;
        float t = l2 > 0.0f ? (wx * ex + wy * ey) / l2 : 0.0f;
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        const float dx = wx - t * ex, dy = wy - t * ey;
        best = fminf(best, dx * dx + dy * dy);
        a = b;
    }
    return sqrtf(best);
}

// range shifter then aperture block, in the beam frame; on success (p, d) is
// on the VP's ray and tmin is the ray parameter of the last exit plane
enum { BL_STOP = 0, BL_PATIENT = 1, BL_DEFER = 2 };

template <bool X, bool D = true>
__device__ int beamline(Lane &v, Acc &acc, float scale, const float *tab, const float2 *poly,
                        const FieldDev &f, float &tmin, const SurDev *sur = nullptr, uint32_t tag = 0u) {
    tmin = -INFINITY;
    if (f.has_rs) {
        const float t = (f.rs_zu - v.pz) / v.dz;
        const float qx = fmaf(t, v.dx, v.px), qy = fmaf(t, v.dy, v.py);
        if (qx * qx + qy * qy <= f.rs_r2) {
            v.px = qx;
            v.py = qy;
            v.pz = f.rs_zu;
            if (slab_transport<X>(v, acc, scale, tab, MAT_PMMA, {f.rs_rho, f.rs_rhol}, f.rs_zu, f.rs_zd,
                               {f.rs_t, f.rs_tl}, L_RS) != EX_DOWN)
                return BL_STOP;
            tmin = 0.0f;
        }
    }
    if (f.has_block) {
        if (!(v.dz > 0.0f)) {
            ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
            return BL_STOP;
        }
        const float t = (f.blk_zu - v.pz) / v.dz;
        const float qx = fmaf(t, v.dx, v.px), qy = fmaf(t, v.dy, v.py);
        const int nv = f.nv;
        bool open = false, through = false;
        if (nv >= 3 && !(D && f.div)) {
            const float tx = f.blk_t / v.dz;
            bool inside;
            const float lb = sdf_bound(f, qx, qy, inside);
            const float lat = sqrtf(v.dx * v.dx + v.dy * v.dy);
            float te = INFINITY;
            if (no_edge_within(lb, lat, tx)) {
                open = inside;
                through = inside;
            } else {
                const int ls = listed_edges(f, poly, nv, qx, qy, v.dx, v.dy, lat, tx, open, te);
                if (ls == 0) open = in_polygon(poly, nv, qx, qy);
                if (open && ls != 1) te = edge_distance(poly, nv, qx, qy, v.dx, v.dy);
                through = open && te >= tx;
            }
        } else if (nv >= 3) {
            const float tx = f.blk_t / v.dz;
            // divergent block: opening scale on the upstream face
            const float sc = f.fc0, kw = v.dz * f.fs;
            const float isc = 1.0f / sc;
            const float bx = qx * isc, by = qy * isc;
            const float cx = v.dx - kw * bx, cy = v.dy - kw * by;
            bool inside;
            const float lb = sdf_bound(f, bx, by, inside);
            if (no_edge_within(lb, sqrtf(cx * cx + cy * cy) / fminf(sc, fmaf(tx, kw, sc)), tx)) {
                open = inside;
                through = inside;
            } else {
                open = in_polygon(poly, nv, bx, by);
                through = open && edge_distance_div(poly, nv, qx, qy, v.dx, v.dy, sc, kw) >= tx;
            }
        }
        if (through) {
            tmin = (f.blk_zd - v.pz) / v.dz;
            return BL_PATIENT;
        }
        if (!open && sur && sur->enabled && !(D && f.div)) {
            // enters through brass: far enough from the opening's edge, the
            // learned surrogate takes over the traversal (queued for it)
            const float de = nv >= 3 ? dist_to_polygon(poly, nv, qx, qy) : 1000.0f;
            if (de >= sur->d_fallback) {
                const unsigned long long slot = atomicAdd(sur->count, 1ull);
                if (slot < sur->capacity) {
                    DeferRec r;
                    r.spot = v.spot;
                    r.hist = v.hist;
                    r.nblk = v.nblk;
                    r.tag = tag;
                    r.x = qx;
                    r.y = qy;
                    r.u = v.dx;
                    r.v = v.dy;
                    r.w = v.dz;
                    r.E = v.E;
                    r.Elo = v.Elo;
                    r.pzlo = v.pzlo;
                    r.d_edge = de;
                    r.thick = f.blk_t;
                    r.pad[0] = r.pad[1] = 0.0f;
                    sur->rec[slot] = r;
                    return BL_DEFER;
                }
            }
        }
        v.px = qx;
        v.py = qy;
        v.pz = f.blk_zu;
        if (block_transport<X, D>(v, acc, scale, tab, poly, nv, f.blk_rho, f.blk_zu, f.blk_zd, {f.blk_t, f.blk_tl}, f) !=
            EX_DOWN)
            return BL_STOP;
        tmin = 0.0f;
    }
    return BL_PATIENT;
}

// ------------------------------------------------------------ patient
// CT calibration: density piecewise linear through (-1000, 0.00121)
// (0, 1) (1000, 1.6) (1500, 1.85) (3071, 2.8); class air / tissue / bone.
// The density is a pair: node values and slopes are FP64 constants split at
// compile time, the CT number is an exact integer.
struct PairC {
    float h, l;
};
constexpr PairC pairc(double x) { return {(float)x, (float)(x - (double)(float)x)}; }
constexpr PairC kCalY[4] = {pairc(0.00121), pairc(1.0), pairc(1.6), pairc(1.85)};
constexpr PairC kCalB[4] = {pairc((1.0 - 0.00121) / 1000.0), pairc(0.6 / 1000.0), pairc(0.25 / 500.0),
                            pairc(0.95 / 1571.0)};
constexpr float kCalX[4] = {-1000.0f, 0.0f, 1000.0f, 1500.0f};

template <bool X>
__device__ __forceinline__ DF hu_density(int hu, int &m) {
    const int hc = min(max(hu, -1000), 3071);
    m = hu < -900 ? MAT_AIR : hu < 150 ? MAT_WATER : MAT_BONE;
    if (!X) {
        // physics mode: the same piecewise-linear calibration as a sum of
        // clamped segments (register arithmetic; a per-segment lookup of the
        // nodes compiles to two dependent memory loads per step)
        const float x = (float)hc;
        float r = fmaf(kCalB[0].h, fminf(x, 0.0f) + 1000.0f, kCalY[0].h);
        r = fmaf(kCalB[1].h, fminf(fmaxf(x, 0.0f), 1000.0f), r);
        r = fmaf(kCalB[2].h, fminf(fmaxf(x - 1000.0f, 0.0f), 500.0f), r);
        r = fmaf(kCalB[3].h, fmaxf(x - 1500.0f, 0.0f), r);
        return {r, 0.0f};
    }
    const int k = hc <= 0 ? 0 : hc <= 1000 ? 1 : hc <= 1500 ? 2 : 3;
    const PairC y = k == 0 ? kCalY[0] : k == 1 ? kCalY[1] : k == 2 ? kCalY[2] : kCalY[3];
    const PairC b = k == 0 ? kCalB[0] : k == 1 ? kCalB[1] : k == 2 ? kCalB[2] : kCalB[3];
    const float x0 = k == 0 ? kCalX[0] : k == 1 ? kCalX[1] : k == 2 ? kCalX[2] : kCalX[3];
    return df_add({y.h, y.l}, df_mul_f({b.h, b.l}, (float)hc - x0));
}

__device__ __forceinline__ void hu_material(int hu, int &m, float &rho) {
    const DF d = hu_density<true>(hu, m);
    rho = d.h + d.l;
}

// keep a voxel-local coordinate pair inside [0, sp]
__device__ __forceinline__ void clamp_pair(float &h, float &l, float sp) {
    if (h < 0.0f || (h == 0.0f && l < 0.0f)) { h = 0.0f; l = 0.0f; }
    else if (h > sp || (h == sp && l > 0.0f)) { h = sp; l = 0.0f; }
}

// position of a VP inside the CT grid between steps
struct PState {
    int idx[3];
    uint32_t vox;   // linear index of voxel idx
    int hu;         // its CT number (CT geometry)
};

// Entry into the CT grid: beam frame -> CT frame with the scenario shift,
// ray-box intersection from the last exit plane (tmin), voxel-local
// coordinates.  Returns false when the VP misses the grid (its energy goes
// to the escaped ledger).
template <bool X>
__device__ bool patient_enter(Lane &v, Acc &acc, float scale, const GeomDev &g, const FieldDev &f,
                              const float *shift, float tmin, PState &ps) {
    float p[3], d[3];
    {
        const float bx = v.px, by = v.py, bz = v.pz;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            p[k] = (f.iso[k] + (bx * f.ex[k] + by * f.ey[k] + bz * f.ez[k])) - shift[k];
            d[k] = v.dx * f.ex[k] + v.dy * f.ey[k] + v.dz * f.ez[k];
        }
    }
    const int n[3] = {g.nx, g.ny, g.nz};
    float hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) hi[k] = g.lo[k] + n[k] * g.sp[k];
    float tnear = -INFINITY, tfar = INFINITY;
    int axn = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0f) {
            if (p[k] < g.lo[k] || p[k] >= hi[k]) {
                ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
                return false;
            }
            continue;
        }
        const float t1 = (g.lo[k] - p[k]) / d[k], t2 = (hi[k] - p[k]) / d[k];
        const float a = fminf(t1, t2), b = fmaxf(t1, t2);
        if (a > tnear) { tnear = a; axn = k; }
        tfar = fminf(tfar, b);
    }
    const float t0 = fmaxf(tnear, tmin);
    if (!(tfar > t0)) {
        ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
        return false;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = fmaf(t0, d[k], p[k]);
    if (t0 == tnear) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k == axn) p[k] = d[k] > 0.0f ? g.lo[k] : hi[k];
    }
    int idx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float c = floorf((p[k] - g.lo[k]) / g.sp[k]);
        idx[k] = !(c >= 0.0f) ? 0 : c > (float)(n[k] - 1) ? n[k] - 1 : (int)c;   // NaN -> 0
    }
    // From here the position is kept relative to the lower corner of the
    // current voxel (0 <= u_k <= spacing_k): FP32 resolves it to ~1e-7 of a
    // voxel wherever the voxel sits, so sub-voxel steps near the end of range
    // do not inherit the rounding of large absolute coordinates.
    {
        float u[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            u[k] = fminf(fmaxf(p[k] - (g.lo[k] + (float)idx[k] * g.sp[k]), 0.0f), g.sp[k]);
            if (t0 == tnear && k == axn) u[k] = d[k] > 0.0f ? 0.0f : g.sp[k];
        }
        v.px = u[0]; v.py = u[1]; v.pz = u[2];
        v.pxlo = v.pylo = v.pzlo = 0.0f;
    }
    v.dx = d[0]; v.dy = d[1]; v.dz = d[2];
    ps.idx[0] = idx[0];
    ps.idx[1] = idx[1];
    ps.idx[2] = idx[2];
    ps.vox = (uint32_t)idx[0] + (uint32_t)g.nx * ((uint32_t)idx[1] + (uint32_t)g.ny * (uint32_t)idx[2]);
    ps.hu = g.kind == 1 ? (int)g.hu[ps.vox] : 0;
    return true;
}

// One condensed-history step of a VP inside the CT grid; false once its
// transport has ended (stopped, or left the grid: then the escaped ledger).
template <class Sink, bool X>
__device__ bool patient_step(Lane &v, Acc &acc, float scale, const float *tab, const GeomDev &g, float range_scale,
                             const Sink &sink, PState &ps) {
    if (v.nsteps >= (uint32_t)MAX_STEPS) {
        ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
        return false;
    }
    const int n[3] = {g.nx, g.ny, g.nz};
    int *idx = ps.idx;
    uint32_t &vox = ps.vox;
    int &hu = ps.hu;
    {
        int m = MAT_WATER;
        DF rho = {1.0f, 0.0f};
        if (g.kind == 1) rho = hu_density<X>(hu, m);
        const DF rho_loss = Ar<X>::mul_f(rho, range_scale);
        // exit face: the axis with the shortest FP32 distance, then that
        // distance as a pair from the pair coordinate
        float dgf = INFINITY;
        int ax = -1, sgn = 0;
        {
            const float pp[3] = {v.px, v.py, v.pz}, pl[3] = {v.pxlo, v.pylo, v.pzlo}, dd[3] = {v.dx, v.dy, v.dz};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (dd[k] == 0.0f) continue;
                const bool up = dd[k] > 0.0f;
                const float t = fmaxf((((up ? g.sp[k] : 0.0f) - pp[k]) - pl[k]) * __builtin_amdgcn_rcpf(dd[k]), 0.0f);
                if (t < dgf) { dgf = t; ax = k; sgn = up ? 1 : -1; }
            }
        }
        DF dg = {dgf, 0.0f};
        if (X && ax >= 0) {
            // selects, not indexing: the per-axis values stay in registers
            const float pa = ax == 0 ? v.px : ax == 1 ? v.py : v.pz;
            const float la = ax == 0 ? v.pxlo : ax == 1 ? v.pylo : v.pzlo;
            const float da = ax == 0 ? v.dx : ax == 1 ? v.dy : v.dz;
            const float spa = ax == 0 ? g.sp[0] : ax == 1 ? g.sp[1] : g.sp[2];
            dg = df_div_f(df_sub({sgn > 0 ? spa : 0.0f, 0.0f}, {pa, la}), da);
            if (!(dg.h > 0.0f)) dg = {0.0f, 0.0f};
        }
        // the CT number behind the face this step may cross is fetched now,
        // so its latency overlaps the step's arithmetic
        int nidx = -1;
        uint32_t nvox = vox;
        int hu_next = hu;
        if (ax >= 0) {
            const int ia = ax == 0 ? idx[0] : ax == 1 ? idx[1] : idx[2];
            const int na = ax == 0 ? n[0] : ax == 1 ? n[1] : n[2];
            const int sa = ax == 0 ? 1 : ax == 1 ? g.nx : g.nx * g.ny;
            nidx = ia + sgn;
            if (nidx >= 0 && nidx < na) {
                nvox = vox + (uint32_t)(sgn * sa);
                if (g.kind == 1) hu_next = (int)g.hu[nvox];
            }
        }
        float dep, esc, let;
        const int st = phys_step<false, X>(v, tab, m, rho_loss, rho.h, dg, dep, esc, let);
        const long long qd = to_fixed(dep, scale);
        if (qd != 0) sink.add(vox, idx, qd);
        if constexpr (Sink::kLet) {
            if (sink.let != nullptr) {
                // numerator of the dose-averaged LET: rne(dep * LET * w/N * 2^(k - kLetShift))
                const long long ql = to_fixed(dep * let, scale * (1.0f / (float)(1 << kLetShift)));
                if (ql != 0) sink.add_let(vox, ql);
            }
        }
        acc.led[L_GRID] += qd;
        if (esc != 0.0f) ledger_add(acc, L_NUC, esc, scale);
        if (st == ST_STOP) return false;
        if (st == ST_GEO) {
            bool out = false;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k == ax) {
                    idx[k] = nidx;
                    out = nidx < 0 || nidx >= n[k];
                }
            }
            if (out) {
                ledger_add(acc, L_ESCAPED, v.E + v.Elo, scale);
                return false;
            }
            // near face of the next voxel, exactly
            const float face_next = sgn > 0 ? 0.0f : (ax == 0 ? g.sp[0] : ax == 1 ? g.sp[1] : g.sp[2]);
            if (ax == 0) { v.px = face_next; v.pxlo = 0.0f; }
            else if (ax == 1) { v.py = face_next; v.pylo = 0.0f; }
            else { v.pz = face_next; v.pzlo = 0.0f; }
            vox = nvox;
            hu = hu_next;
        }
        clamp_pair(v.px, v.pxlo, g.sp[0]);
        clamp_pair(v.py, v.pylo, g.sp[1]);
        clamp_pair(v.pz, v.pzlo, g.sp[2]);
    }
    return true;
}

template <class Sink, bool X>
__device__ void patient(Lane &v, Acc &acc, float scale, const float *tab, const GeomDev &g,
                        const FieldDev &f, const float *shift, float range_scale, const Sink &sink,
                        float tmin) {
    PState ps;
    if (!patient_enter<X>(v, acc, scale, g, f, shift, tmin, ps)) return;
    while (patient_step<Sink, X>(v, acc, scale, tab, g, range_scale, sink, ps)) {
    }
}

// ------------------------------------------------------------ source
__device__ void source(Lane &v, const SpotDev &sp, float vsad) {
    const uint4 w = draw(v);
    const float r = sqrtf(-2.0f * logf(unit_open(w.x)));
    float sn, c;
    sincospif(2.0f * unit_open(w.y), &sn, &c);
    v.px = fmaf(sp.sigma, r * c, sp.x);
    v.py = fmaf(sp.sigma, r * sn, sp.y);
    v.pz = 0.0f;
    v.pzlo = 0.0f;
    v.pxlo = v.pylo = 0.0f;
    v.dx = 0.0f; v.dy = 0.0f; v.dz = 1.0f;
    if (vsad > 0.0f) {
        // along the line from the virtual source through the start point
        const float inv = 1.0f / sqrtf(fmaf(v.px, v.px, fmaf(v.py, v.py, vsad * vsad)));
        v.dx = v.px * inv;
        v.dy = v.py * inv;
        v.dz = vsad * inv;
    }
    v.E = sp.e0;
    v.Elo = 0.0f;
    if (sp.esig > 0.0f) {
        const float z = 1.41421356237f * erfinvf(2.0f * unit_open(w.z) - 1.0f);
        v.E = fminf(fmaxf(fmaf(sp.esig, z, sp.e0), kELo), sp.emax);
    }
}

__device__ __forceinline__ int find_spot(const unsigned long long *off, int n, unsigned long long item) {
    int lo = 0, hi = n;   // off[lo] <= item < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

template <bool X>
__global__ __launch_bounds__(512) void transport_kernel(GeomDev g, FieldDev f, LaunchDev L) {
    __shared__ float tab[X ? TAB_FLOATS : TAB_HI_FLOATS];
    __shared__ float2 poly[POLY_LDS];
    for (int i = threadIdx.x; i < (X ? TAB_FLOATS : TAB_HI_FLOATS) / 4; i += blockDim.x)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(L.tables)[i];
    if (f.has_block)
        for (int i = threadIdx.x; i < f.nv; i += blockDim.x) poly[i] = f.poly[i];
    __syncthreads();

    Acc acc;
#pragma unroll
    for (int j = 0; j < NLEDGER; ++j) acc.led[j] = 0;
    acc.steps = acc.hist = 0;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long item = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         item < L.n_items; item += stride) {
        const int s = find_spot(L.item_off, L.n_spots, item);
        const SpotDev sp = L.spots[s];
        Lane v;
        v.k0 = L.key0;
        v.k1 = L.key1;
        v.spot = (uint32_t)s;
        v.hist = (uint32_t)(L.batch + (unsigned long long)L.n_batches * (item - L.item_off[s]));
        v.nblk = 0;
        v.nsteps = 0;
        v.physics = L.physics;
        source(v, sp, f.vsad);
        float tmin;
        if (beamline<X>(v, acc, sp.scale, tab, poly, f, tmin, &L.sur) == BL_PATIENT)
            patient<DenseSink, X>(v, acc, sp.scale, tab, g, f, L.shift, L.range_scale, DenseSink{L.tally, L.let_tally},
                                  tmin);
        acc.steps += v.nsteps;
        acc.hist += 1;
    }
    // wavefront reduction of the ledgers, one atomic per wavefront
#pragma unroll
    for (int j = 0; j < NLEDGER; ++j) {
        long long x = acc.led[j];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0 && x != 0) atomicAdd(L.ledger + j, (unsigned long long)x);
    }
    unsigned long long st = acc.steps, hs = acc.hist;
    for (int o = 32; o > 0; o >>= 1) {
        st += __shfl_xor(st, o, 64);
        hs += __shfl_xor(hs, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && hs != 0) {
        atomicAdd(L.stats + 0, st);
        atomicAdd(L.stats + 1, hs);
    }
}

// ------------------------------------------------------------ CSR mode
// A VP staged at its entry into the CT grid (64 B, four 16-byte words):
// voxel-local position, direction in the CT frame, energy pair, Philox block
// counter, history, step count, voxel (linear, per axis) and its CT number.
struct alignas(16) StagedVP {
    float px, py, pz, dx;
    float dy, dz, E, Elo;
    uint32_t nblk, hist, nsteps, vox;
    int i0, i1, i2, hu;
};
static_assert(sizeof(StagedVP) == 4 * kStageFields, "staging record");

constexpr uint32_t kRowNone = 0xFFFFFFFFu;   // workgroup row word: no row yet
constexpr uint32_t kRowPick = 0xFFFFFFFDu;   // a wave is picking the next row
constexpr uint32_t kRowEnd = 0xFFFFFFFEu;    // no work left in the epoch
constexpr uint32_t kTileBusy = 0xFFFFFFFFu;  // tile users field while it is added out

__device__ __forceinline__ unsigned long long rd_lds64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds the tile of row rl (epoch-local) into its slot grid and clears it; one wave.
__device__ void tile_flush(long long *tile, const RowDev &row, const QueueDev &Q, const GeomDev &g, uint32_t rl,
                           int lane) {
    const uint32_t n0 = (uint32_t)row.tn[0], n1 = (uint32_t)row.tn[1], n2 = (uint32_t)row.tn[2];
    const SparseSink gs{Q.grid + (size_t)rl * Q.gstride, Q.mark + (size_t)rl * Q.mstride};
    uint32_t e = 0;
    for (uint32_t u2 = 0; u2 < n2; ++u2)
        for (uint32_t u1 = 0; u1 < n1; ++u1, e += n0)
            for (uint32_t u0 = (uint32_t)lane; u0 < n0; u0 += 64) {
                const long long q = tile[e + u0];
                if (q != 0) {
                    tile[e + u0] = 0;
                    gs.put((uint32_t)(row.tlo[0] + (int)u0) +
                               (uint32_t)g.nx * ((uint32_t)(row.tlo[1] + (int)u1) + (uint32_t)g.ny * (uint32_t)(row.tlo[2] + (int)u2)),
                           q);
                }
            }
}

// Influence-matrix transport of an epoch's rows.  Each row has a chunk
// counter (chunk = 64 * hist_per_lane histories); a workgroup works on one
// current row at a time, its waves drawing chunks of it, and when the row is
// exhausted one wave picks the next: a fresh row from the epoch's row head,
// else (work stealing) any row with chunks left, else the end.  The
// workgroup's LDS tile holds one row's box at a time (RowDev::tlo/tn): a
// wave joins it for a chunk of that row, and the last wave to leave adds
// it into the slot grid; chunks of another row go straight to the slot
// grid.  Per chunk, in stage fills of up to 64 * kStageHpl histories:
// phase 1 runs source, beam line and CT entry with the lanes in lock step
// and stages the VPs that enter the grid (compacted with a ballot); phase 2
// is the patient step loop, where a lane whose VP has ended takes the next
// staged VP as soon as refill_min lanes are idle (or all remaining VPs fit).
// Each history's arithmetic and random stream are those of a lane running it
// alone, and the tallies are integer sums: the result does not depend on
// the schedule.  The only waits between waves are for the wave that is
// replacing the current row, which does so without waiting on anyone.
template <bool X, bool D>
// Physics mode: up to 1024 threads (16 waves at <= 128 VGPRs, one workgroup
// per CU with a ~120 KiB tile); double-float mode: up to 768 (12 waves at
// <= 168 VGPRs).  D: some field of the batch is divergent (virtual source or
// divergent block); without, the plain geometry is compiled alone.
__global__ __launch_bounds__(X ? 768 : 1024) void queue_kernel(GeomDev g, QueueDev Q) {
    __shared__ float tab[X ? TAB_FLOATS : TAB_HI_FLOATS];
    __shared__ float2 poly[POLY_LDS];
    __shared__ unsigned long long s_row;    // current row (high word; kRowNone while replaced)
    __shared__ unsigned long long s_tile;   // (row of the tile << 32) | users, kTileBusy while flushed
    extern __shared__ __attribute__((aligned(16))) long long tile[];   // Q.tile_cap int64
    for (int i = threadIdx.x; i < (X ? TAB_FLOATS : TAB_HI_FLOATS) / 4; i += blockDim.x)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(Q.tables)[i];
    for (int i = threadIdx.x; i < Q.n_poly_total; i += blockDim.x) poly[i] = Q.polys[i];
    for (int i = threadIdx.x; i < Q.tile_cap; i += blockDim.x) tile[i] = 0;
    if (threadIdx.x == 0) {
        s_row = (unsigned long long)kRowNone << 32;
        s_tile = (unsigned long long)kRowNone << 32;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int hps = min(Q.hist_per_lane, kStageHpl);   // histories per lane per stage fill
    StagedVP *const stg = reinterpret_cast<StagedVP *>(Q.stage) +
                          ((size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (size_t)(hps * 64);
    const unsigned long long chunk_h = 64ull * (unsigned long long)Q.hist_per_lane;
    unsigned long long iters = 0;
    for (;;) {
        // ---- bounded queue: a wavefront that has made iter_cap iterations
        // (chunks, row picks, waits) leaves and reports it; it holds no row
        // pick and no tile here, so the other waves finish as before
        if (++iters > Q.iter_cap) {
            if (lane == 0) atomicOr(Q.flags, kFlagAborted);
            break;
        }
        // ---- the workgroup's current row, and a chunk of it
        const uint32_t cur = __builtin_amdgcn_readfirstlane((uint32_t)(rd_lds64(&s_row) >> 32));
        if (cur == kRowEnd) break;
        if (cur == kRowPick) {   // another wave is picking the next row (it waits on nobody)
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        unsigned long long cj = ~0ull;
        uint32_t nch = 0;
        if (cur != kRowNone) {
            nch = (uint32_t)((Q.rows[Q.row_begin + cur].n_hist + chunk_h - 1) / chunk_h);
            if (lane == 0) cj = atomicAdd(Q.row_next + cur, 1ull);
            cj = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(cj >> 32)) << 32) |
                 __builtin_amdgcn_readfirstlane((uint32_t)cj);
        }
        if (cj >= nch) {
            // no row yet, or this one is exhausted: the one wave that swaps
            // the row word from cur to kRowPick picks the next row
            bool mine = false;
            if (lane == 0) {
                unsigned long long w = (unsigned long long)cur << 32;
                mine = __hip_atomic_compare_exchange_strong(&s_row, &w, (unsigned long long)kRowPick << 32,
                                                            __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (__builtin_amdgcn_readfirstlane((uint32_t)mine) != 0u) {
                // a fresh row from the epoch's head, else the first row with
                // chunks left (64 rows per probe), else the end
                unsigned long long f = 0;
                if (lane == 0) f = atomicAdd(Q.head, 1ull);
                f = __builtin_amdgcn_readfirstlane((uint32_t)f);   // < 2^32 rows
                uint32_t nr = kRowEnd;
                if (f < (unsigned long long)Q.n_rows) {
                    nr = (uint32_t)f;
                } else {
                    for (int r0 = 0; r0 < Q.n_rows; r0 += 64) {
                        const int r = r0 + lane;
                        bool left = false;
                        if (r < Q.n_rows) {
                            const unsigned long long nc = (Q.rows[Q.row_begin + r].n_hist + chunk_h - 1) / chunk_h;
                            left = __hip_atomic_load(Q.row_next + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < nc;
                        }
                        const unsigned long long m = __ballot(left);
                        if (m) {
                            nr = (uint32_t)(r0 + __ffsll((long long)m) - 1);
                            break;
                        }
                    }
                }
                if (lane == 0)
                    __hip_atomic_store(&s_row, (unsigned long long)nr << 32, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            continue;
        }
        const uint32_t rl = cur;
        const unsigned long long j = cj;
        const RowDev row = Q.rows[Q.row_begin + rl];
        const SpotDev sp = Q.spots[row.spot_global];
        const ScenDev sc = Q.scen[row.scen];
        const SparseSink gsink{Q.grid + (size_t)rl * Q.gstride, Q.mark + (size_t)rl * Q.mstride};
        // ---- join the tile for this chunk if it holds this row (or is free)
        bool joined = false;
        const uint32_t tn = (uint32_t)row.tn[0] * (uint32_t)row.tn[1] * (uint32_t)row.tn[2];
        if (tn != 0u && tn <= (uint32_t)Q.tile_cap) {
            if (lane == 0) {
                for (;;) {
                    unsigned long long t = rd_lds64(&s_tile);
                    const uint32_t tr = (uint32_t)(t >> 32), us = (uint32_t)t;
                    unsigned long long want;
                    if (us == kTileBusy) break;
                    if (tr == rl) want = t + 1ull;
                    else if (us == 0u) want = ((unsigned long long)rl << 32) | 1ull;   // free (and clear): take it
                    else break;
                    if (__hip_atomic_compare_exchange_strong(&s_tile, &t, want, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        joined = true;
                        break;
                    }
                }
            }
            joined = __builtin_amdgcn_readfirstlane((uint32_t)joined) != 0u;
        }
        const TileSink sink{joined ? tile : nullptr, row.tlo[0], row.tlo[1], row.tlo[2],
                            (uint32_t)row.tn[0], (uint32_t)row.tn[1], (uint32_t)row.tn[2], gsink};
        Acc acc;
#pragma unroll
        for (int k = 0; k < NLEDGER; ++k) acc.led[k] = 0;
        acc.steps = acc.hist = 0;
        Lane v;
        v.k0 = Q.key0;
        v.k1 = Q.seed_hi ^ row.field_id;
        v.spot = row.spot;
        v.physics = Q.physics;
        for (int t0 = 0; t0 < Q.hist_per_lane; t0 += hps) {
            if ((j * (unsigned long long)Q.hist_per_lane + t0) * 64ull >= row.n_hist) break;
            // phase 1
            uint32_t nst = 0;
            {
                const FieldDev &f = Q.fields[row.field];
                const float2 *fpoly = poly + Q.poly_off[row.field];
                for (int t = t0; t < min(Q.hist_per_lane, t0 + hps); ++t) {
                    const unsigned long long h0 = (j * (unsigned long long)Q.hist_per_lane + t) * 64ull;
                    if (h0 >= row.n_hist) break;
                    const unsigned long long h = h0 + lane;
                    bool in = false;
                    PState ps;
                    if (h < row.n_hist) {
                        v.hist = (uint32_t)h;
                        v.nblk = 0;
                        v.nsteps = 0;
                        source(v, sp, D ? f.vsad : 0.0f);
                        float tmin;
                        in = beamline<X, D>(v, acc, sp.scale, tab, fpoly, f, tmin, &Q.sur, (uint32_t)rl) == BL_PATIENT &&
                             patient_enter<X>(v, acc, sp.scale, g, f, sc.shift, tmin, ps);
                        if (!in) acc.steps += v.nsteps;
                        acc.hist += 1;
                    }
                    const unsigned long long rb = __ballot(in);
                    if (in) {
                        StagedVP r;
                        r.px = v.px; r.py = v.py; r.pz = v.pz; r.dx = v.dx;
                        r.dy = v.dy; r.dz = v.dz; r.E = v.E; r.Elo = v.Elo;
                        r.nblk = v.nblk; r.hist = v.hist; r.nsteps = v.nsteps; r.vox = ps.vox;
                        r.i0 = ps.idx[0]; r.i1 = ps.idx[1]; r.i2 = ps.idx[2]; r.hu = ps.hu;
                        stg[nst + (uint32_t)__popcll(rb & below)] = r;
                    }
                    nst += (uint32_t)__popcll(rb);
                }
            }
            // the staged entries are read back by other lanes of this wave
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            // phase 2
            uint32_t next = 0;
            bool active = false;
            PState ps;
            for (;;) {
                const unsigned long long idle = __ballot(!active);
                const uint32_t nidle = (uint32_t)__popcll(idle);
                const bool refill = next < nst && nidle >= min((uint32_t)Q.refill_min, nst - next);
                if (!refill && nidle == 64u) break;
                const uint32_t k = next + (uint32_t)__popcll(idle & below);
                if (refill && !active && k < nst) {
                    // word by word (single-word loads are not merged into
                    // 4-register tuples, so each field can land in the
                    // register the loop carries it in)
                    const uint32_t *rw = reinterpret_cast<const uint32_t *>(stg + k);
                    auto ld = [&](int i) {
                        return __hip_atomic_load(rw + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    };
                    v.px = __uint_as_float(ld(0)); v.py = __uint_as_float(ld(1));
                    v.pz = __uint_as_float(ld(2)); v.dx = __uint_as_float(ld(3));
                    v.dy = __uint_as_float(ld(4)); v.dz = __uint_as_float(ld(5));
                    v.E = __uint_as_float(ld(6)); v.Elo = __uint_as_float(ld(7));
                    v.pxlo = v.pylo = v.pzlo = 0.0f;
                    v.nblk = ld(8); v.hist = ld(9); v.nsteps = ld(10);
                    ps.vox = ld(11);
                    ps.idx[0] = (int)ld(12); ps.idx[1] = (int)ld(13); ps.idx[2] = (int)ld(14);
                    ps.hu = (int)ld(15);
                    active = true;
                }
                if (refill) next = min(nst, next + nidle);
                if (active) {
                    active = patient_step<TileSink, X>(v, acc, sp.scale, tab, g, sc.range_scale, sink, ps);
                    if (!active) acc.steps += v.nsteps;
                }
            }
        }
        // ---- leave the tile; the last user adds it out and frees it
        if (joined) {
            bool flusher = false;
            if (lane == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                for (;;) {
                    unsigned long long t = rd_lds64(&s_tile);
                    const bool last = (uint32_t)t == 1u;
                    const unsigned long long want = last ? (((unsigned long long)rl << 32) | kTileBusy) : t - 1ull;
                    if (__hip_atomic_compare_exchange_strong(&s_tile, &t, want, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        flusher = last;
                        break;
                    }
                }
            }
            flusher = __builtin_amdgcn_readfirstlane((uint32_t)flusher) != 0u;
            if (flusher) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                tile_flush(tile, row, Q, g, rl, lane);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0)
                    __hip_atomic_store(&s_tile, (unsigned long long)rl << 32, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int k = 0; k < NLEDGER; ++k) {
            long long x = acc.led[k];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
            if (lane == 0 && x != 0) atomicAdd(Q.ledger + (size_t)row.scen * NLEDGER + k, (unsigned long long)x);
        }
        unsigned long long sx = acc.steps, hx = acc.hist;
        for (int o = 32; o > 0; o >>= 1) {
            sx += __shfl_xor(sx, o, 64);
            hx += __shfl_xor(hx, o, 64);
        }
        if (lane == 0 && hx != 0) {
            atomicAdd(Q.stats + 0, sx);
            atomicAdd(Q.stats + 1, hx);
        }
    }
}

// ---- compaction of an epoch's rows into CSR (three passes per epoch)
// A chunk is 256 touched-block bytes (8192 voxels) of one row, handled by
// one wave: lane l reads mark bytes 4l..4l+3 as one word (the mark stride is
// a multiple of 256, so the word stays inside the row's marks), the marked
// blocks are listed in ascending order in the wave's LDS, and then the two
// half-waves read two blocks' 32 slot values (coalesced 256 B each) at a
// time, kCsrUnroll such pairs in flight before any is used.  A wave visits
// kCsrGroup consecutive (row, chunk) pairs at once, their mark words loaded
// together; the waves of the launch stride over the epoch's groups,
// consecutive waves on consecutive groups.  A chunk without marks costs one
// load (in flight with its group's) and a ballot.
constexpr int kCsrGroup = 4, kCsrUnroll = 4;

// mark words of the pairs [g * kCsrGroup, ...) of an epoch (0 past the end)
__device__ __forceinline__ void group_marks(const QueueDev &Q, size_t gi, size_t npair, int lane,
                                            uint32_t (&w)[kCsrGroup]) {
#pragma unroll
    for (int j = 0; j < kCsrGroup; ++j) {
        const size_t pair = gi * kCsrGroup + j;
        w[j] = 0u;
        if (pair < npair) {
            const size_t row = pair / Q.nchunk, chunk = pair - row * Q.nchunk;
            w[j] = *reinterpret_cast<const uint32_t *>(Q.mark + row * Q.mstride + chunk * 256 + 4 * lane);
        }
    }
}

// lists the marked blocks of a chunk (offsets 0..255) in ascending order;
// returns their count
__device__ __forceinline__ int chunk_blocks(uint32_t wv, int lane, int *list) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c += ((wv >> (8 * k)) & 0xFFu) != 0u;
    int pre = c;   // inclusive prefix over the lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(pre, o, 64);
        if (lane >= o) pre += y;
    }
    const int tot = __shfl(pre, 63, 64);
    int at = pre - c;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (((wv >> (8 * k)) & 0xFFu) != 0u) list[at++] = 4 * lane + k;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return tot;
}

// pass 1: non-zero count of every (row, chunk)
__global__ __launch_bounds__(256) void csr_count_kernel(QueueDev Q, unsigned int *cnt) {
    __shared__ int lists[4][256];
    const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
    int *list = lists[wv_id];
    const size_t npair = (size_t)Q.n_rows * Q.nchunk;
    const size_t ngroup = (npair + kCsrGroup - 1) / kCsrGroup;
    const size_t nwave = (size_t)gridDim.x * 4;
    for (size_t gi = (size_t)blockIdx.x * 4 + wv_id; gi < ngroup; gi += nwave) {
        uint32_t w[kCsrGroup];
        group_marks(Q, gi, npair, lane, w);
#pragma unroll
        for (int j = 0; j < kCsrGroup; ++j) {
            const size_t pair = gi * kCsrGroup + j;
            if (pair >= npair) break;
            unsigned int c = 0;
            if (__ballot(w[j] != 0u) != 0ull) {
                const size_t row = pair / Q.nchunk, chunk = pair - row * Q.nchunk;
                const size_t b0 = chunk * 256;
                const unsigned long long *grid = Q.grid + row * Q.gstride;
                const int nm = chunk_blocks(w[j], lane, list);
                for (int p = 0; 2 * p < nm; p += kCsrUnroll) {
                    unsigned long long q[kCsrUnroll];
#pragma unroll
                    for (int u = 0; u < kCsrUnroll; ++u) {
                        const int idx = 2 * (p + u) + (lane >> 5);
                        q[u] = idx < nm ? grid[(b0 + list[idx]) * 32 + (lane & 31)] : 0ull;
                    }
#pragma unroll
                    for (int u = 0; u < kCsrUnroll; ++u) c += q[u] != 0ull;
                }
                for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
                __builtin_amdgcn_wave_barrier();   // list reused by the next chunk
            }
            if (lane == 0) cnt[pair] = c;
        }
    }
}

// pass 2: per row, exclusive prefix of its chunk counts and the row total
__global__ __launch_bounds__(1024) void csr_chunk_scan_kernel(const unsigned int *cnt, unsigned int *coff,
                                                              unsigned int *rowcnt, size_t nchunk) {
    __shared__ unsigned int part[1024];
    __shared__ unsigned int carry;
    const int row = blockIdx.x, t = threadIdx.x;
    const unsigned int *c = cnt + (size_t)row * nchunk;
    unsigned int *o = coff + (size_t)row * nchunk;
    if (t == 0) carry = 0u;
    __syncthreads();
    for (size_t s0 = 0; s0 < nchunk; s0 += 1024) {
        const unsigned int x = s0 + t < nchunk ? c[s0 + t] : 0u;
        part[t] = x;
        __syncthreads();
        for (int k = 1; k < 1024; k <<= 1) {
            const unsigned int y = t >= k ? part[t - k] : 0u;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        if (s0 + t < nchunk) o[s0 + t] = carry + part[t] - x;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) rowcnt[row] = carry;
}

// exclusive scan of this epoch's row counts into global CSR offsets (rows
// are stored in row order, so the offsets are the final row pointers)
__global__ __launch_bounds__(1024) void csr_offsets_kernel(const unsigned int *nnz, int n_rows, int row_begin,
                                                           unsigned long long *row_off,
                                                           unsigned long long *row_nnz,
                                                           unsigned long long *used,
                                                           unsigned long long capacity, unsigned int *flags) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const unsigned long long x = t < n_rows ? nnz[t] : 0ull;
    part[t] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const unsigned long long y = t >= o ? part[t - o] : 0ull;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    const unsigned long long base = *used;
    if (t < n_rows) {
        row_off[row_begin + t] = base + part[t] - x;
        row_nnz[row_begin + t] = x;
    }
    __syncthreads();
    if (t == 1023) {
        *used = base + part[1023];
        if (base + part[1023] > capacity) atomicOr(flags, 1u);
    }
}

// pass 3: emit (voxel, q) of every chunk at its place in ascending voxel
// order and clear exactly the touched blocks and their marks
__global__ __launch_bounds__(256) void csr_emit_kernel(QueueDev Q, const unsigned int *cnt, const unsigned int *coff,
                                                       const unsigned long long *row_off,
                                                       const unsigned long long *row_nnz, int32_t *col,
                                                       long long *qv, unsigned long long capacity,
                                                       unsigned int *flags) {
    __shared__ int lists[4][256];
    const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
    int *list = lists[wv_id];
    const size_t npair = (size_t)Q.n_rows * Q.nchunk;
    const size_t ngroup = (npair + kCsrGroup - 1) / kCsrGroup;
    const size_t nwave = (size_t)gridDim.x * 4;
    for (size_t gi = (size_t)blockIdx.x * 4 + wv_id; gi < ngroup; gi += nwave) {
        uint32_t w[kCsrGroup];
        group_marks(Q, gi, npair, lane, w);
#pragma unroll
        for (int j = 0; j < kCsrGroup; ++j) {
            const size_t pair = gi * kCsrGroup + j;
            if (pair >= npair) break;
            if (__ballot(w[j] != 0u) == 0ull) continue;
            const size_t row = pair / Q.nchunk, chunk = pair - row * Q.nchunk;
            const size_t b0 = chunk * 256;
            uint8_t *mark = Q.mark + row * Q.mstride;
            unsigned long long *grid = Q.grid + row * Q.gstride;
            const int nm = chunk_blocks(w[j], lane, list);
            const unsigned long long rb = row_off[Q.row_begin + row];
            const bool write = rb + row_nnz[Q.row_begin + row] <= capacity;
            const unsigned long long p0 = rb + coff[pair];
            unsigned long long pos = p0;
            for (int p = 0; 2 * p < nm; p += kCsrUnroll) {
                unsigned long long q[kCsrUnroll];
                size_t v[kCsrUnroll];
#pragma unroll
                for (int u = 0; u < kCsrUnroll; ++u) {
                    const int idx = 2 * (p + u) + (lane >> 5);
                    v[u] = idx < nm ? (b0 + list[idx]) * 32 + (lane & 31) : 0;
                    q[u] = idx < nm ? grid[v[u]] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < kCsrUnroll; ++u) {
                    const int idx = 2 * (p + u) + (lane >> 5);
                    const unsigned long long bal = __ballot(q[u] != 0ull);
                    if (q[u] != 0ull && write) {
                        const unsigned long long at = pos + __popcll(bal & ((1ull << lane) - 1ull));
                        col[at] = (int32_t)v[u];
                        qv[at] = (long long)q[u];
                    }
                    if (idx < nm) grid[v[u]] = 0ull;
                    pos += __popcll(bal);
                }
            }
            if (w[j] != 0u) *reinterpret_cast<uint32_t *>(mark + b0 + 4 * lane) = 0u;
            if (lane == 0 && pos - p0 != cnt[pair]) atomicOr(flags, 2u);
            __builtin_amdgcn_wave_barrier();   // list reused by the next chunk
        }
    }
}

// Rate of non-returning int64 atomic adds to device memory with the address
// pattern of the transport's deposits: each lane walks a track of `len`
// consecutive voxels along x (the beam axis of a lateral field) from a
// random depth, at a lateral (y, z) offset drawn around one of 64 spot axes
// with a Gaussian of sigma voxels (sum of 4 uniforms), so that hot spots
// form where tracks overlap.  Work: n_tracks x len atomics.
__global__ __launch_bounds__(256) void atomic_rate_kernel(unsigned long long *grid, int nx, int ny, int nz,
                                                          unsigned long long n_tracks, int len, float sigma,
                                                          uint32_t seed) {
    for (unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_tracks;
         t += (unsigned long long)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)t * 0x9E3779B9u ^ seed;
        auto next = [&]() {   // xorshift32
            x ^= x << 13; x ^= x >> 17; x ^= x << 5;
            return x;
        };
        next(); next();
        const uint32_t spot = (uint32_t)(t >> 12) & 63u;   // neighbouring tracks share a spot
        const float cy = 0.25f * ny + 0.5f * ny * (float)((spot * 2654435761u) >> 16 & 0xFFFFu) / 65536.0f;
        const float cz = 0.25f * nz + 0.5f * nz * (float)((spot * 2246822519u) >> 16 & 0xFFFFu) / 65536.0f;
        float gy = 0.0f, gz = 0.0f;
        for (int k = 0; k < 4; ++k) {
            gy += (float)(next() >> 8) * 0x1p-24f;
            gz += (float)(next() >> 8) * 0x1p-24f;
        }
        // sum of 4 U(0,1): mean 2, variance 1/3
        const int y = min(max((int)(cy + (gy - 2.0f) * 1.7320508f * sigma), 0), ny - 1);
        const int z = min(max((int)(cz + (gz - 2.0f) * 1.7320508f * 0.5f * sigma), 0), nz - 1);
        const int x0 = (int)(next() % (uint32_t)max(nx - len, 1));
        unsigned long long *row = grid + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z);
        for (int i = 0; i < len && x0 + i < nx; ++i) atomicAdd(row + x0 + i, 1ull);
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, size_t n, unsigned long long v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void csr_scatter_kernel(const int32_t *col, const long long *qv, unsigned long long begin,
                                   unsigned long long end, unsigned long long *dense) {
    for (unsigned long long i = begin + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < end;
         i += (unsigned long long)gridDim.x * blockDim.x)
        atomicAdd(dense + col[i], (unsigned long long)qv[i]);
}

__global__ void csr_values_kernel(const int32_t *col, const long long *qv, size_t n, GeomDev g, double mev_scale,
                                  float *val) {
    const float vol_kg = g.sp[0] * g.sp[1] * g.sp[2] * 1e-6f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float rho = 1.0f;
        int m;
        if (g.kind == 1) hu_material(g.hu[col[i]], m, rho);
        val[i] = (float)qv[i] * ((float)mev_scale / (rho * vol_kg));
    }
}

// ------------------------------------------------------------ dynamic voxel spacing
// Influence-matrix rows merged into cells (the planning system's coarser
// voxels for organs at risk, Methods C): a cell is a run of consecutive
// voxels given by a non-decreasing voxel -> cell map, cstart[c] its first
// voxel.  Cell mass (kg) = the sum of its voxels' masses, in voxel order.
__global__ void cell_mass_kernel(GeomDev g, const int32_t *cstart, int n_cells, double *mass) {
    const double vol_kg = (double)g.sp[0] * (double)g.sp[1] * (double)g.sp[2] * 1e-6;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x) {
        double m = 0.0;
        for (int v = cstart[c]; v < cstart[c + 1]; ++v) {
            float rho = 1.0f;
            int mm;
            if (g.kind == 1) hu_material(g.hu[v], mm, rho);
            m += (double)rho;
        }
        mass[c] = m * vol_kg;
    }
}

// cells per piece (a wavefront per piece of at most kCellPiece entries of one
// row): runs of one cell that start inside the piece; flags columns outside
// the grid (bit 1) and columns not ascending within a row (bit 2)
__global__ __launch_bounds__(256) void cell_count_kernel(const long long *rp, const CellPiece *pcs,
                                                         long long n_pieces, const int32_t *col,
                                                         const int32_t *cmap, int nvox, unsigned long long *cnt,
                                                         unsigned *err) {
    const long long p = (long long)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (p >= n_pieces) return;
    const int lane = (int)(threadIdx.x & 63);
    const CellPiece pc = pcs[p];
    const long long b = pc.begin, e = pc.begin + pc.len;
    int carry = -1, carry_col = -1;
    if (b > rp[pc.row]) {
        // the entry before the piece (checked by the piece that owns it)
        carry_col = col[b - 1];
        carry = (unsigned)carry_col < (unsigned)nvox ? cmap[carry_col] : -1;
    }
    unsigned long long n = 0;
    for (long long i0 = b; i0 < e; i0 += 64) {
        const long long i = i0 + lane;
        const bool valid = i < e;
        int c = -1, v = -1;
        if (valid) {
            v = col[i];
            if ((unsigned)v >= (unsigned)nvox) atomicOr(err, 1u);
            else c = cmap[v];
        }
        int pv = __shfl_up(v, 1);
        int pc_ = __shfl_up(c, 1);
        if (lane == 0) {
            pv = carry_col;
            pc_ = carry;
        }
        if (valid && (i > b || carry_col >= 0) && v <= pv) atomicOr(err, 2u);
        n += (unsigned long long)__popcll(__ballot(valid && c >= 0 && c != pc_));
        carry = __shfl(c, 63);
        carry_col = __shfl(v, 63);
    }
    if (lane == 0) cnt[p] = n;
}

// merged rows, a wavefront per piece: the runs that start inside the piece
// belong to it; segmented sums of their int64 energies (exact) over 64-entry
// windows, carried across windows; the piece's last run is followed past the
// piece's end up to the next start or the row's end.  The value is the
// cell's energy over its mass.
__global__ __launch_bounds__(256) void cell_emit_kernel(const long long *rp, const CellPiece *pcs, long long n_pieces,
                                                        const int32_t *col, const long long *q, const int32_t *cmap,
                                                        const long long *pout, const double *mass, double mev_scale,
                                                        int32_t *ocell, long long *oq, float *oval) {
    const long long p = (long long)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (p >= n_pieces) return;
    const int lane = (int)(threadIdx.x & 63);
    const CellPiece pc = pcs[p];
    const long long re = rp[pc.row + 1];
    const long long b = pc.begin, e = pc.begin + pc.len;
    const long long o0 = pout[p], o1 = pout[p + 1];
    if (o0 == o1) return;   // no run starts in this piece
    int carry_cell = b > rp[pc.row] ? cmap[col[b - 1]] : -1;
    long long carry_sum = 0, starts_before = 0, e_eff = re;
    auto put = [&](long long k, int c, long long sum) {
        const long long pos = o0 + k;
        if (k >= 0 && pos < o1) {
            if (ocell) ocell[pos] = c;
            if (oq) oq[pos] = sum;
            if (oval) oval[pos] = (float)((double)sum * mev_scale / mass[c]);
        }
    };
    for (long long i0 = b;; i0 += 64) {
        const long long i = i0 + lane;
        const bool valid0 = i < re;
        const int c = valid0 ? cmap[col[i]] : -1;
        int pcl = __shfl_up(c, 1);
        if (lane == 0) pcl = carry_cell;
        const bool start0 = valid0 && c != pcl;
        if (i0 + 64 > e) {
            // the first start at or after the piece's end closes its last run
            const unsigned long long m0 = __ballot(start0 && i >= e);
            if (m0) {
                const long long first = i0 + (long long)(__ffsll((long long)m0) - 1);
                e_eff = first < e_eff ? first : e_eff;
            }
        }
        const bool valid = valid0 && i < e_eff;
        const bool start = start0 && valid;
        const bool v0 = __shfl(valid ? 1 : 0, 0) != 0, s0 = __shfl(start ? 1 : 0, 0) != 0;
        // the run left open by the last window ends here
        if (lane == 0 && carry_cell >= 0 && (s0 || !v0)) put(starts_before - 1, carry_cell, carry_sum);
        if (!v0) break;
        long long x = valid ? q[i] : 0;
        if (lane == 0 && !start) x += carry_sum;
        long long sum = x;
        int f = start ? 1 : 0;
        for (int d = 1; d < 64; d <<= 1) {
            const long long so = __shfl_up(sum, d);
            const int fo = __shfl_up(f, d);
            if (lane >= d && !f) sum += so;
            if (lane >= d) f |= fo;
        }
        const unsigned long long m = __ballot(start);
        const int last = (int)((e_eff - i0 < 64 ? e_eff - i0 : 64) - 1);
        const bool next_start = __shfl_down(start ? 1 : 0, 1) != 0;
        if (valid && lane < last && next_start)
            put(starts_before + (long long)__popcll(m & ((2ull << lane) - 1ull)) - 1, c, sum);
        carry_cell = __shfl(c, last);
        carry_sum = __shfl(sum, last);
        starts_before += (long long)__popcll(m);
    }
}

// ------------------------------------------------------------ surrogate data
// Plain brass traversals for the surrogate's training data: each entry state
// (x, y on the block's upstream face, direction cosines u, v, energy) crosses
// the field's block with the plain transport (crossing number at every step).
// Per VP: the 8 network inputs, the 3 normalised targets and the outcome
// (1 transmitted, 0 stopped or lost, -1 entered through the opening).
__global__ __launch_bounds__(256) void surrogate_sample_kernel(FieldDev f, const float *entries, int n,
                                                               uint32_t key0, uint32_t key1, unsigned physics,
                                                               const float *tables, float *xo, float *yo,
                                                               float *to) {
    __shared__ float tab[TAB_HI_FLOATS];
    __shared__ float2 poly[POLY_LDS];
    for (int i = threadIdx.x; i < TAB_HI_FLOATS / 4; i += blockDim.x)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(tables)[i];
    for (int i = threadIdx.x; i < f.nv; i += blockDim.x) poly[i] = f.poly[i];
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float *e = entries + (size_t)i * 5;
        Lane v;
        v.k0 = key0;
        v.k1 = key1;
        v.spot = 0;
        v.hist = (uint32_t)i;
        v.nblk = 0;
        v.nsteps = 0;
        v.physics = physics;
        v.px = e[0];
        v.py = e[1];
        v.pz = f.blk_zu;
        v.pzlo = 0.0f;
        v.pxlo = v.pylo = 0.0f;
        v.dx = e[2];
        v.dy = e[3];
        v.dz = sqrtf(fmaxf(1.0f - e[2] * e[2] - e[3] * e[3], 0.0f));
        v.E = e[4];
        v.Elo = 0.0f;
        const float x0 = v.px, y0 = v.py, u0 = v.dx, w0 = v.dy, z0 = v.dz, E0 = v.E;
        const int nv = f.nv;
        const bool open = nv >= 3 && in_polygon(poly, nv, x0, y0);
        const float de = nv >= 3 ? dist_to_polygon(poly, nv, x0, y0) : 1000.0f;
        float *xr = xo + (size_t)i * 8;
        xr[0] = x0 / 20.0f;
        xr[1] = y0 / 20.0f;
        xr[2] = u0 / 0.05f;
        xr[3] = w0 / 0.05f;
        xr[4] = (E0 - 150.0f) / 50.0f;
        xr[5] = fminf(de, 100.0f) / 10.0f;
        xr[6] = f.blk_t / 30.0f;
        xr[7] = 0.0f;   // brass
        float *yr = yo + (size_t)i * 3;
        yr[0] = yr[1] = yr[2] = 0.0f;
        if (open) {
            to[i] = -1.0f;
            continue;
        }
        Acc acc;
#pragma unroll
        for (int k = 0; k < NLEDGER; ++k) acc.led[k] = 0;
        const int ex =
            block_transport<false>(v, acc, 1.0f, tab, poly, nv, f.blk_rho, f.blk_zu, f.blk_zd, {f.blk_t, f.blk_tl}, f);
        if (ex != EX_DOWN) {
            to[i] = 0.0f;
            continue;
        }
        to[i] = 1.0f;
        const float Eo = v.E + v.Elo;
        const float c = fminf(fmaxf(u0 * v.dx + w0 * v.dy + z0 * v.dz, -1.0f), 1.0f);
        const float tx = f.blk_t / z0;
        const float xs = fmaf(tx, u0, x0), ys = fmaf(tx, w0, y0);
        yr[0] = ((E0 - Eo) / E0 - 0.5f) / 0.25f;
        yr[1] = acosf(c) / 0.05f;
        yr[2] = sqrtf((v.px - xs) * (v.px - xs) + (v.py - ys) * (v.py - ys)) / 2.0f;
    }
}


// Resume one deferred VP: where the network is confident the traversal is
// sampled from it (transmission, then one mixture component and its
// outgoing energy loss, angle and offset; azimuth uniform, shared by angle
// and offset); otherwise the plain brass transport runs from the recorded
// state.  Then the patient.
template <class Sink, bool X>
__device__ void resume_deferred(Lane &v, Acc &acc, float scale, const float *tab, const float2 *poly,
                                const FieldDev &f, const float *o, float p_lo, float p_hi, const GeomDev &g,
                                const float *shift, float range_scale, const Sink &sink) {
    const float ptrans = 1.0f / (1.0f + __expf(-o[0]));
    bool go = true;
    if (!(ptrans < p_lo || ptrans > p_hi)) {
        go = block_transport<X>(v, acc, scale, tab, poly, f.nv, f.blk_rho, f.blk_zu, f.blk_zd, {f.blk_t, f.blk_tl}, f) ==
             EX_DOWN;
    } else {
        v.E += v.Elo;
        v.Elo = 0.0f;
        const uint4 w = draw(v);
        if (!(unit_open(w.x) < ptrans)) {
            ledger_add(acc, L_BLOCK, v.E, scale);   // stopped in brass
            go = false;
        } else {
            // mixture component from the softmax of the weight logits
            float mw = o[1];
            for (int c = 1; c < 4; ++c) mw = fmaxf(mw, o[1 + c]);
            float pc[4], tot = 0.0f;
            for (int c = 0; c < 4; ++c) { pc[c] = __expf(o[1 + c] - mw); tot += pc[c]; }
            const float uc = unit_open(w.y) * tot;
            int c = 0;
            float acc_p = pc[0];
            while (c < 3 && uc > acc_p) { ++c; acc_p += pc[c]; }
            const uint4 w2 = draw(v);
            float z0, z1, z2, z3;
            box_muller_fast(w2.x, w2.y, z0, z1);
            box_muller_fast(w2.z, w2.w, z2, z3);
            const float y0 = o[5 + 3 * c + 0] + __expf(o[17 + 3 * c + 0]) * z0;
            const float y1 = o[5 + 3 * c + 1] + __expf(o[17 + 3 * c + 1]) * z1;
            const float y2 = o[5 + 3 * c + 2] + __expf(o[17 + 3 * c + 2]) * z2;
            const float frac = fminf(fmaxf(0.5f + 0.25f * y0, 0.0f), 1.0f);
            const float theta = fmaxf(y1, 0.0f) * 0.05f;
            const float off = fmaxf(y2, 0.0f) * 2.0f;
            const float phi = unit_open(w.z);   // turns
            const float cph = __builtin_amdgcn_cosf(phi), sph = __builtin_amdgcn_sinf(phi);
            const float Eout = v.E * (1.0f - frac);
            ledger_add(acc, L_BLOCK, v.E - Eout, scale);
            const float tx = f.blk_t / v.dz;
            v.px = fmaf(tx, v.dx, v.px) + off * cph;
            v.py = fmaf(tx, v.dy, v.py) + off * sph;
            rotate_dir(v, theta * cph, theta * sph);
            v.pz = f.blk_zd;
            v.E = Eout;
            if (!(v.dz > 0.0f) || Eout <= kELo) {
                ledger_add(acc, (v.dz > 0.0f) ? L_BLOCK : L_ESCAPED, Eout, scale);
                go = false;
            }
        }
    }
    if (go) patient<Sink, X>(v, acc, scale, tab, g, f, shift, range_scale, sink, 0.0f);
}

__device__ __forceinline__ void lane_from_record(Lane &v, const DeferRec &r, uint32_t k0, uint32_t k1,
                                                 unsigned physics, float zu) {
    v.k0 = k0;
    v.k1 = k1;
    v.spot = r.spot;
    v.hist = r.hist;
    v.nblk = r.nblk;
    v.nsteps = 0;
    v.physics = physics;
    v.px = r.x;
    v.py = r.y;
    v.pz = zu;
    v.pzlo = r.pzlo;
    v.pxlo = v.pylo = 0.0f;
    v.dx = r.u;
    v.dy = r.v;
    v.dz = r.w;
    v.E = r.E;
    v.Elo = r.Elo;
}

__device__ __forceinline__ void flush_ledger_steps(Acc &acc, unsigned long long *ledger, unsigned long long *stats) {
#pragma unroll
    for (int j = 0; j < NLEDGER; ++j) {
        long long x = acc.led[j];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((threadIdx.x & 63) == 0 && x != 0) atomicAdd(ledger + j, (unsigned long long)x);
        acc.led[j] = 0;
    }
    unsigned long long st = acc.steps;
    for (int o = 32; o > 0; o >>= 1) st += __shfl_xor(st, o, 64);
    if ((threadIdx.x & 63) == 0 && st != 0) atomicAdd(stats + 0, st);
    acc.steps = 0;
}

// dense runs: one field, one scenario per launch
template <bool X>
__global__ __launch_bounds__(256) void sur_resume_kernel(GeomDev g, FieldDev f, LaunchDev L, const DeferRec *rec,
                                                         const float *out, unsigned long long n, float p_lo,
                                                         float p_hi) {
    __shared__ float tab[X ? TAB_FLOATS : TAB_HI_FLOATS];
    __shared__ float2 poly[POLY_LDS];
    for (int i = threadIdx.x; i < (X ? TAB_FLOATS : TAB_HI_FLOATS) / 4; i += blockDim.x)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(L.tables)[i];
    for (int i = threadIdx.x; i < f.nv; i += blockDim.x) poly[i] = f.poly[i];
    __syncthreads();
    Acc acc;
#pragma unroll
    for (int j = 0; j < NLEDGER; ++j) acc.led[j] = 0;
    acc.steps = acc.hist = 0;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const DeferRec r = rec[i];
        Lane v;
        lane_from_record(v, r, L.key0, L.key1, L.physics, f.blk_zu);
        resume_deferred<DenseSink, X>(v, acc, L.spots[r.spot].scale, tab, poly, f, out + i * MLP_OUT, p_lo, p_hi, g, L.shift,
                        L.range_scale, DenseSink{L.tally, L.let_tally});
        acc.steps += v.nsteps;
    }
    flush_ledger_steps(acc, L.ledger, L.stats);
}

// influence-matrix runs: the record's tag is its row within the epoch, which
// selects the field, spot, scenario and the row's sparse slot
template <bool X>
__global__ __launch_bounds__(256) void sur_resume_csr_kernel(GeomDev g, QueueDev Q, const DeferRec *rec,
                                                             const float *out, unsigned long long n, float p_lo,
                                                             float p_hi) {
    __shared__ float tab[X ? TAB_FLOATS : TAB_HI_FLOATS];
    __shared__ float2 poly[POLY_LDS];
    for (int i = threadIdx.x; i < (X ? TAB_FLOATS : TAB_HI_FLOATS) / 4; i += blockDim.x)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(Q.tables)[i];
    for (int i = threadIdx.x; i < Q.n_poly_total; i += blockDim.x) poly[i] = Q.polys[i];
    __syncthreads();
    Acc acc;
#pragma unroll
    for (int j = 0; j < NLEDGER; ++j) acc.led[j] = 0;
    acc.steps = acc.hist = 0;
    int cur_scen = -1;   // scenario whose ledger this lane is accumulating
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const DeferRec r = rec[i];
        const int rl = (int)r.tag;
        const RowDev row = Q.rows[Q.row_begin + rl];
        const FieldDev f = Q.fields[row.field];
        const ScenDev sc = Q.scen[row.scen];
        const SparseSink sink{Q.grid + (size_t)rl * Q.gstride, Q.mark + (size_t)rl * Q.mstride};
        if (row.scen != cur_scen) {
            // ledgers are per scenario: this lane's sums so far go out with
            // plain per-lane atomics (lanes of a wave may differ in scenario)
            if (cur_scen >= 0)
                for (int j = 0; j < NLEDGER; ++j)
                    if (acc.led[j] != 0) {
                        atomicAdd(Q.ledger + (size_t)cur_scen * NLEDGER + j, (unsigned long long)acc.led[j]);
                        acc.led[j] = 0;
                    }
            cur_scen = row.scen;
        }
        Lane v;
        lane_from_record(v, r, Q.key0, Q.seed_hi ^ row.field_id, Q.physics, f.blk_zu);
        resume_deferred<SparseSink, X>(v, acc, Q.spots[row.spot_global].scale, tab, poly + Q.poly_off[row.field], f,
                        out + i * MLP_OUT, p_lo, p_hi, g, sc.shift, sc.range_scale, sink);
        acc.steps += v.nsteps;
    }
    // every lane of the wave is back here: the ledgers reduce per wave and
    // scenario (an epoch's records span one or two scenarios), one atomic per
    // group instead of one per lane
    bool pending = cur_scen >= 0;
    for (;;) {
        const unsigned long long m = __ballot(pending);
        if (!m) break;
        const int leader = __ffsll((long long)m) - 1;
        const int sc = __shfl(cur_scen, leader, 64);
        const bool mine = pending && cur_scen == sc;
#pragma unroll
        for (int j = 0; j < NLEDGER; ++j) {
            long long x = mine ? acc.led[j] : 0ll;
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
            if ((int)(threadIdx.x & 63) == leader && x != 0)
                atomicAdd(Q.ledger + (size_t)sc * NLEDGER + j, (unsigned long long)x);
        }
        if (mine) pending = false;
    }
    unsigned long long st = acc.steps;
    for (int o = 32; o > 0; o >>= 1) st += __shfl_xor(st, o, 64);
    if ((threadIdx.x & 63) == 0 && st != 0) atomicAdd(Q.stats + 0, st);
}

// ------------------------------------------------------------ batches, dose
// fold one batch: total += q_b, sum of squares += q_b^2 (FP64), clear q_b
__global__ void fold_batch_kernel(unsigned long long *qb, long long *qt, double *s2, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const long long q = (long long)qb[i];
        if (q != 0) {
            qt[i] += q;
            const double d = (double)q;
            s2[i] += d * d;
            qb[i] = 0ull;
        }
    }
}

__global__ void dose_kernel(const long long *q, const double *s2, int B, GeomDev g, double mev_scale,
                            float *dose, float *sigma, size_t n) {
    const float vol_kg = g.sp[0] * g.sp[1] * g.sp[2] * 1e-6f;   // mm^3 -> cm^3 -> kg at 1 g/cm^3
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        float rho = 1.0f;
        int m;
        if (g.kind == 1) hu_material(g.hu[i], m, rho);
        const float conv = (float)mev_scale / (rho * vol_kg);   // Gy per (q unit)
        const long long qi = q[i];
        if (dose) dose[i] = (float)qi * conv;
        if (sigma) {
            // batch estimator of the standard error of the mean (FP64)
            const double D = (double)qi;
            const double var = fmax((double)B * s2[i] - D * D, 0.0) / (double)(B - 1);
            sigma[i] = (float)sqrt(var) * conv;
        }
    }
}

}  // namespace

hipError_t launch_transport(const GeomDev &g, const FieldDev &f, const LaunchDev &L, int blocks,
                            int threads, hipStream_t s) {
    if (threads != 256 && threads != 512) threads = kThreads;
    // deterministic mode: the double-float instantiation
    if (L.physics == 0) hipLaunchKernelGGL(transport_kernel<true>, dim3(blocks), dim3(threads), 0, s, g, f, L);
    else hipLaunchKernelGGL(transport_kernel<false>, dim3(blocks), dim3(threads), 0, s, g, f, L);
    return hipGetLastError();
}

int queue_threads(unsigned physics, int threads) {
    const int cap = physics == 0 ? 768 : 1024;
    if (threads != 256 && threads != 512 && threads != 768 && threads != 1024) threads = cap;
    return std::min(threads, cap);
}

// LDS per CU (160 KiB) shared by the workgroups that give the CU its target
// waves (16 in physics mode, 12 in double-float mode), less the static tables
int queue_tile_cap(unsigned physics, int threads) {
    threads = queue_threads(physics, threads);
    const int waves_cu = physics == 0 ? 12 : 16;
    const int wgs = std::max(1, waves_cu / (threads / 64));
    const int stat = (physics == 0 ? TAB_FLOATS : TAB_HI_FLOATS) * 4 + POLY_LDS * 8 + 256;
    const int per_wg = 160 * 1024 / wgs - stat;
    return std::max(0, per_wg / 8);
}

hipError_t launch_queue(const GeomDev &g, const QueueDev &Q, int blocks, int threads, hipStream_t s) {
    threads = queue_threads(Q.physics, threads);
    const size_t tile_bytes = (size_t)Q.tile_cap * sizeof(long long);
    if (Q.physics == 0) {
        if (Q.div) hipLaunchKernelGGL((queue_kernel<true, true>), dim3(blocks), dim3(threads), tile_bytes, s, g, Q);
        else hipLaunchKernelGGL((queue_kernel<true, false>), dim3(blocks), dim3(threads), tile_bytes, s, g, Q);
    } else {
        if (Q.div) hipLaunchKernelGGL((queue_kernel<false, true>), dim3(blocks), dim3(threads), tile_bytes, s, g, Q);
        else hipLaunchKernelGGL((queue_kernel<false, false>), dim3(blocks), dim3(threads), tile_bytes, s, g, Q);
    }
    return hipGetLastError();
}

// workgroups (4 waves each) of the compaction passes: one wave per group of
// kCsrGroup (row, chunk) pairs up to 4096 workgroups, the waves striding over
// the rest
static unsigned csr_pass_blocks(const QueueDev &Q) {
    const size_t ngroup = ((size_t)Q.n_rows * Q.nchunk + kCsrGroup - 1) / kCsrGroup;
    return (unsigned)std::max<size_t>(1, std::min<size_t>((ngroup + 3) / 4, 4096));
}

hipError_t launch_csr_count(const QueueDev &Q, unsigned int *cnt, hipStream_t s) {
    hipLaunchKernelGGL(csr_count_kernel, dim3(csr_pass_blocks(Q)), dim3(256), 0, s, Q, cnt);
    return hipGetLastError();
}

hipError_t launch_csr_chunk_scan(const unsigned int *cnt, unsigned int *coff, unsigned int *rowcnt, int n_rows,
                                 size_t nchunk, hipStream_t s) {
    hipLaunchKernelGGL(csr_chunk_scan_kernel, dim3(n_rows), dim3(1024), 0, s, cnt, coff, rowcnt, nchunk);
    return hipGetLastError();
}

hipError_t launch_csr_offsets(const unsigned int *nnz, int n_rows, int row_begin, unsigned long long *row_off,
                              unsigned long long *row_nnz, unsigned long long *used, unsigned long long capacity,
                              unsigned int *flags, hipStream_t s) {
    hipLaunchKernelGGL(csr_offsets_kernel, dim3(1), dim3(1024), 0, s, nnz, n_rows, row_begin, row_off, row_nnz, used,
                       capacity, flags);
    return hipGetLastError();
}

hipError_t launch_csr_emit(const QueueDev &Q, const unsigned int *cnt, const unsigned int *coff,
                           const unsigned long long *row_off, const unsigned long long *row_nnz, int32_t *col,
                           long long *qv, unsigned long long capacity, unsigned int *flags, hipStream_t s) {
    hipLaunchKernelGGL(csr_emit_kernel, dim3(csr_pass_blocks(Q)), dim3(256), 0, s, Q, cnt, coff, row_off,
                       row_nnz, col, qv, capacity, flags);
    return hipGetLastError();
}

hipError_t launch_atomic_rate(unsigned long long *grid, int nx, int ny, int nz, unsigned long long n_tracks, int len,
                              float sigma, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(atomic_rate_kernel, dim3(4096), dim3(256), 0, s, grid, nx, ny, nz, n_tracks, len, sigma, seed);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_csr_scatter(const int32_t *col, const long long *qv, unsigned long long begin,
                              unsigned long long end, unsigned long long *dense, hipStream_t s) {
    const unsigned long long n = end - begin;
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    if (blocks > 0) hipLaunchKernelGGL(csr_scatter_kernel, dim3(blocks), dim3(256), 0, s, col, qv, begin, end, dense);
    return hipGetLastError();
}

hipError_t launch_csr_values(const int32_t *col, const long long *qv, size_t n, const GeomDev &g,
                             double mev_scale, float *val, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    if (blocks > 0) hipLaunchKernelGGL(csr_values_kernel, dim3(blocks), dim3(256), 0, s, col, qv, n, g, mev_scale, val);
    return hipGetLastError();
}


hipError_t launch_cell_mass(const GeomDev &g, const int32_t *cstart, int n_cells, double *mass, hipStream_t s) {
    const int blocks = std::max(1, std::min((n_cells + 255) / 256, 8192));
    hipLaunchKernelGGL(cell_mass_kernel, dim3(blocks), dim3(256), 0, s, g, cstart, n_cells, mass);
    return hipGetLastError();
}

hipError_t launch_cell_count(const long long *rp, const CellPiece *pcs, long long n_pieces, const int32_t *col,
                             const int32_t *cmap, int nvox, unsigned long long *cnt, unsigned *err, hipStream_t s) {
    if (n_pieces == 0) return hipSuccess;
    const long long blocks = (n_pieces * 64 + 255) / 256;
    hipLaunchKernelGGL(cell_count_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rp, pcs, n_pieces, col, cmap, nvox,
                       cnt, err);
    return hipGetLastError();
}

hipError_t launch_cell_emit(const long long *rp, const CellPiece *pcs, long long n_pieces, const int32_t *col,
                            const long long *q, const int32_t *cmap, const long long *pout, const double *mass,
                            double mev_scale, int32_t *ocell, long long *oq, float *oval, hipStream_t s) {
    if (n_pieces == 0) return hipSuccess;
    const long long blocks = (n_pieces * 64 + 255) / 256;
    hipLaunchKernelGGL(cell_emit_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rp, pcs, n_pieces, col, q, cmap,
                       pout, mass, mev_scale, ocell, oq, oval);
    return hipGetLastError();
}

hipError_t launch_sur_resume(const GeomDev &g, const FieldDev &f, const LaunchDev &L, const DeferRec *rec,
                             const float *out, unsigned long long n, float p_lo, float p_hi, hipStream_t s) {
    const int blocks = (int)std::max<unsigned long long>(1, std::min<unsigned long long>((n + 255) / 256, 4096));
    if (L.physics == 0)
        hipLaunchKernelGGL(sur_resume_kernel<true>, dim3(blocks), dim3(256), 0, s, g, f, L, rec, out, n, p_lo, p_hi);
    else
        hipLaunchKernelGGL(sur_resume_kernel<false>, dim3(blocks), dim3(256), 0, s, g, f, L, rec, out, n, p_lo, p_hi);
    return hipGetLastError();
}

hipError_t launch_sur_resume_csr(const GeomDev &g, const QueueDev &Q, const DeferRec *rec, const float *out,
                                 unsigned long long n, float p_lo, float p_hi, hipStream_t s) {
    const int blocks = (int)std::max<unsigned long long>(1, std::min<unsigned long long>((n + 255) / 256, 4096));
    if (Q.physics == 0)
        hipLaunchKernelGGL(sur_resume_csr_kernel<true>, dim3(blocks), dim3(256), 0, s, g, Q, rec, out, n, p_lo, p_hi);
    else
        hipLaunchKernelGGL(sur_resume_csr_kernel<false>, dim3(blocks), dim3(256), 0, s, g, Q, rec, out, n, p_lo, p_hi);
    return hipGetLastError();
}

hipError_t launch_surrogate_sample(const FieldDev &f, const float *entries, int n, uint32_t key0, uint32_t key1,
                                   unsigned physics, const float *tables, float *x, float *y, float *t, hipStream_t s) {
    const int blocks = std::max(1, std::min((n + 255) / 256, 4096));
    hipLaunchKernelGGL(surrogate_sample_kernel, dim3(blocks), dim3(256), 0, s, f, entries, n, key0, key1, physics,
                       tables, x, y, t);
    return hipGetLastError();
}

hipError_t launch_fold_batch(unsigned long long *qb, long long *qt, double *s2, size_t n, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    hipLaunchKernelGGL(fold_batch_kernel, dim3(blocks), dim3(256), 0, s, qb, qt, s2, n);
    return hipGetLastError();
}

hipError_t launch_dose(const long long *q, const double *s2, int B, const GeomDev &g, double mev_scale,
                       float *dose, float *sigma, size_t n, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    hipLaunchKernelGGL(dose_kernel, dim3(blocks), dim3(256), 0, s, q, s2, B, g, mev_scale, dose, sigma, n);
    return hipGetLastError();
}

// Scratch of the allocation-free dense run.  In host code the name `scratch`
// is only a host-side stand-in for the array: kernels and copies get the
// device address from scratch_device_ptr(), never the name itself.
static __device__ __align__(256) unsigned long long scratch[kScratchBytes / sizeof(unsigned long long)];

hipError_t scratch_device_ptr(int device, void **out) {
    static std::mutex mu;
    static void *addr[kMaxScratchDevices] = {};
    if (!out || device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the symbol is looked up on the current device
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace vpmc
