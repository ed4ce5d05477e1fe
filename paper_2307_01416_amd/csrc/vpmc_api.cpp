// Host runtime of libvpmc: argument validation (before any HIP call),
// device buffers, fixed-point scaling, batch loop and the C ABI of
// include/vpmc.h.
#include <math.h>

#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/vpmc.h"
#include "vpmc_internal.hpp"

using namespace vpmc;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? VPMC_E_OOM : VPMC_E_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                    \
    } while (0)

bool finite3(const float *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct FieldState {
    bool set = false;
    FieldDev dev{};
    std::vector<float2> poly;
    DevBuf poly_buf, sdf_buf, cell_off_buf, cell_edge_buf, cell_ref_buf;
};

// Signed distance (FP64, + inside) from the cell centres of a raster over
// the polygon's bounding box widened by `margin` to the polygon boundary;
// the side follows the same half-open crossing-number rule as the kernels.
struct Raster {
    double x0, y0, h;
    int nx, ny;
    std::vector<float> d;
};

Raster polygon_raster(const std::vector<float2> &poly, double margin) {
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (const float2 &p : poly) {
        xmin = std::min(xmin, (double)p.x); xmax = std::max(xmax, (double)p.x);
        ymin = std::min(ymin, (double)p.y); ymax = std::max(ymax, (double)p.y);
    }
    Raster r;
    const double ext = std::max(xmax - xmin, ymax - ymin) + 2.0 * margin;
    r.h = std::max(0.25, ext / 512.0);
    r.x0 = xmin - margin;
    r.y0 = ymin - margin;
    r.nx = (int)std::ceil((xmax - xmin + 2.0 * margin) / r.h);
    r.ny = (int)std::ceil((ymax - ymin + 2.0 * margin) / r.h);
    r.d.resize((size_t)r.nx * r.ny);
    const int nv = (int)poly.size();
    for (int j = 0; j < r.ny; ++j)
        for (int i = 0; i < r.nx; ++i) {
            const double x = r.x0 + (i + 0.5) * r.h, y = r.y0 + (j + 0.5) * r.h;
            bool in = false;
            double best = 1e300;
            for (int a = nv - 1, b = 0; b < nv; a = b++) {
                const double ax = poly[a].x, ay = poly[a].y, bx = poly[b].x, by = poly[b].y;
                if ((ay > y) != (by > y)) {
                    const double xc = ax + (y - ay) * (bx - ax) / (by - ay);
                    if (x < xc) in = !in;
                }
                const double ex = bx - ax, ey = by - ay, l2 = ex * ex + ey * ey;
                double t = l2 > 0.0 ? ((x - ax) * ex + (y - ay) * ey) / l2 : 0.0;
                t = std::min(std::max(t, 0.0), 1.0);
                const double dx = x - ax - t * ex, dy = y - ay - t * ey;
                best = std::min(best, dx * dx + dy * dy);
            }
            r.d[(size_t)j * r.nx + i] = (float)(in ? std::sqrt(best) : -std::sqrt(best));
        }
    return r;
}

// Per raster cell near the boundary: a reference point (FP32, at least
// 1e-4 mm from every edge, within 0.01 mm of the cell centre) with its side
// by the crossing-number rule, and the edges (k, k+1) within kListRadius of
// it.  A point p of the cell is on the reference point's side unless listed
// edges cross the segment from it to p, and a ray from p meets no unlisted
// edge within kListRadius - |p - ref|, so the kernels test a handful of edges
// instead of every edge there.  Cells farther than kListRadius + h from the
// boundary get no reference point (the raster's distance bound decides them).
// off[cell]: bits 0-29 the first entry of the cell in edge[], bit 30 a
// reference point exists, bit 31 it is inside; the next cell's bits 0-29 end
// the list.
struct CellLists {
    std::vector<uint32_t> off;
    std::vector<uint16_t> edge;
    std::vector<float2> ref;
};

bool crossing_inside(const std::vector<float2> &poly, double x, double y) {
    const int nv = (int)poly.size();
    bool in = false;
    for (int a = nv - 1, b = 0; b < nv; a = b++) {
        const double ax = poly[a].x, ay = poly[a].y, bx = poly[b].x, by = poly[b].y;
        if ((ay > y) != (by > y)) {
            const double xc = ax + (y - ay) * (bx - ax) / (by - ay);
            if (x < xc) in = !in;
        }
    }
    return in;
}

double segment_distance(const float2 &a, const float2 &b, double x, double y) {
    const double ex = (double)b.x - a.x, ey = (double)b.y - a.y, l2 = ex * ex + ey * ey;
    double t = l2 > 0.0 ? ((x - a.x) * ex + (y - a.y) * ey) / l2 : 0.0;
    t = std::min(std::max(t, 0.0), 1.0);
    const double dx = x - a.x - t * ex, dy = y - a.y - t * ey;
    return std::sqrt(dx * dx + dy * dy);
}

CellLists cell_lists(const std::vector<float2> &poly, const Raster &r, double radius) {
    const int nv = (int)poly.size();
    CellLists L;
    L.off.assign((size_t)r.nx * r.ny + 1, 0u);
    L.ref.assign((size_t)r.nx * r.ny, make_float2(0.f, 0.f));
    for (int j = 0; j < r.ny; ++j)
        for (int i = 0; i < r.nx; ++i) {
            const size_t cell = (size_t)j * r.nx + i;
            L.off[cell] = (uint32_t)L.edge.size();
            if (std::fabs((double)r.d[cell]) > radius + r.h) continue;   // no edge within reach of the cell
            // reference point: the cell centre in FP32, moved (by at most
            // 0.01 mm) off any edge it lies within 1e-4 mm of
            float2 q = make_float2((float)(r.x0 + (i + 0.5) * r.h), (float)(r.y0 + (j + 0.5) * r.h));
            for (int tries = 0; tries < 8; ++tries) {
                double dmin = 1e300;
                for (int k = 0; k < nv; ++k) dmin = std::min(dmin, segment_distance(poly[k], poly[(k + 1) % nv], q.x, q.y));
                if (dmin > 1e-4) break;
                q = make_float2(q.x + 0.0013f, q.y + 0.0009f);
            }
            L.ref[cell] = q;
            L.off[cell] |= 0x40000000u;
            if (crossing_inside(poly, q.x, q.y)) L.off[cell] |= 0x80000000u;
            for (int k = 0; k < nv; ++k)
                if (segment_distance(poly[k], poly[(k + 1) % nv], q.x, q.y) <= radius) L.edge.push_back((uint16_t)k);
        }
    L.off[(size_t)r.nx * r.ny] = (uint32_t)L.edge.size();
    return L;
}

}  // namespace

struct vpmc_ctx {
    int device = -1;
    float *d_tables = nullptr;
    void *scratch = nullptr;   // device address of this GPU's static scratch (vpmc_run_spots_noalloc)
    // geometry
    bool has_geom = false;
    GeomDev geom{};
    DevBuf hu_buf;
    size_t nvox = 0;
    FieldState fields[VPMC_MAX_FIELDS];
    // scratch (grow-only)
    DevBuf tallies, qbatch, s2, ledger, spots, offsets, stage_dose, stage_sigma, stats, let_tallies;
    bool last_let = false;   // the last dense run tallied the LET numerator
    size_t bytes = 0;
    // last run
    int last_k = 0, last_nscen = 0;
    vpmc_stats last_stats{};
    std::vector<hipEvent_t> events;
    // influence-matrix builder
    DevBuf slot_grid, slot_mark, slot_cnt, slot_coff, slot_rowcnt, q_stage, q_rownext;
    int n_slots = 0;
    size_t slot_nvox = 0;
    bool slots_dirty = false;
    DevBuf rows, chunk_off, heads, row_off, row_nnz, used, flags, fields_tab, poly_off, polys, scen_tab, csr_col, csr_q;
    unsigned long long csr_cap = 0, csr_total = 0, csr_cap_hint = 0;
    int csr_rows = 0;
    bool csr_valid = false;
    unsigned csr_flags = 0;
    // autotuned launch shapes (0 = not tuned)
    int tuned_csr_hpl = 0, tuned_csr_blocks = 0, tuned_dense_blocks = 0;
    int tuned_csr_hpl_field[VPMC_MAX_FIELDS] = {};   // per field (CSR), 0 = not tuned
    int tuned_csr_threads = 0, tuned_dense_threads = 0;
    hipStream_t cap_stream = nullptr;   // private stream for graph capture
    // aperture surrogate
    DevBuf mlp_w, mlp_wb, mlp_m, mlp_v, mlp_g, mlp_act, mlp_io, mlp_dx, mlp_dy, mlp_dt, mlp_idx;
    bool mlp_ready = false;
    int mlp_step = 0;
    int mlp_batch_cap = 0;
    DevBuf sur_rec, sur_cnt, sur_out;
    // spot-weight optimiser: structure-restricted rows, bucketed copies and
    // gradient pieces (kept for VPMC_OPT_REUSE), work buffers
    struct OptBuckets {
        DevBuf off, key, val, work;
        long long n_work = 0;
        bool valid = false;
    } opt_broi, opt_bfull;
    DevBuf opt_rp, opt_col, opt_val, opt_roi, opt_amax, opt_cnt, opt_rcnt, opt_crp, opt_ccol, opt_cval, opt_piece,
        opt_poff, opt_resid, opt_fpart, opt_gpart, opt_vec, opt_scal, opt_err, opt_hist, opt_dose, opt_sidx,
        opt_rstruct;
    long long opt_npieces = 0;
    int opt_nstruct = 0;
    // dynamic voxel spacing (vpmc_csr_cells)
    DevBuf cl_rp, cl_map, cl_start, cl_mass, cl_cnt, cl_out, cl_col, cl_q, cl_ocell, cl_oq, cl_oval, cl_piece;
    bool opt_valid = false;
    int opt_dims[5] = {0, 0, 0, 0, 0};   // n_scen, n_spots, row_stride, row_offset, nvox
    std::vector<int64_t> opt_rp_host;
    std::vector<uint8_t> opt_roi_host;
    const void *opt_col_src = nullptr, *opt_val_src = nullptr;
    float sur_dfb = 3.0f, sur_plo = 0.02f, sur_phi = 0.98f;
};

namespace {

int mlp_buffers(vpmc_ctx *c, int cap, MlpBuffers *b);

int ensure(vpmc_ctx *c, DevBuf &b, size_t bytes, size_t cap_limit) {
    if (bytes <= b.cap) return VPMC_OK;
    const size_t grow = bytes - b.cap;
    if (cap_limit && c->bytes + grow > cap_limit)
        return fail(VPMC_E_OOM, "scratch of %zu bytes exceeds max_device_bytes=%zu", c->bytes + grow,
                    cap_limit);
    if (b.ptr) {
        HIP_TRY(hipFree(b.ptr));
        c->bytes -= b.cap;
        b.ptr = nullptr;
        b.cap = 0;
    }
    HIP_TRY(hipMalloc(&b.ptr, bytes));
    b.cap = bytes;
    c->bytes += bytes;
    return VPMC_OK;
}

void release(DevBuf &b) {
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.cap = 0;
}

double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

bool segments_intersect(const float2 &p1, const float2 &p2, const float2 &q1, const float2 &q2) {
    const double d1 = cross2(q2.x - q1.x, q2.y - q1.y, p1.x - q1.x, p1.y - q1.y);
    const double d2 = cross2(q2.x - q1.x, q2.y - q1.y, p2.x - q1.x, p2.y - q1.y);
    const double d3 = cross2(p2.x - p1.x, p2.y - p1.y, q1.x - p1.x, q1.y - p1.y);
    const double d4 = cross2(p2.x - p1.x, p2.y - p1.y, q2.x - p1.x, q2.y - p1.y);
    if (((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) && ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0)))
        return true;
    auto on_seg = [](const float2 &a, const float2 &b, const float2 &p, double d) {
        return d == 0 && std::min(a.x, b.x) <= p.x && p.x <= std::max(a.x, b.x) &&
               std::min(a.y, b.y) <= p.y && p.y <= std::max(a.y, b.y);
    };
    return on_seg(q1, q2, p1, d1) || on_seg(q1, q2, p2, d2) || on_seg(p1, p2, q1, d3) ||
           on_seg(p1, p2, q2, d4);
}

int validate_polygon(const float *xy, int n) {
    if (n == 0) return VPMC_OK;
    if (n < 3) return fail(VPMC_E_POLYGON, "aperture polygon needs 0 (closed) or >= 3 vertices, got %d", n);
    if (n > VPMC_MAX_VERTICES)
        return fail(VPMC_E_POLYGON, "aperture polygon has %d vertices (max %d)", n, VPMC_MAX_VERTICES);
    if (!xy) return fail(VPMC_E_ARG, "xy_mm is NULL");
    double area = 0.0;
    for (int i = 0; i < n; ++i) {
        const int j = (i + 1) % n;
        if (!isfinite(xy[2 * i]) || !isfinite(xy[2 * i + 1]))
            return fail(VPMC_E_POLYGON, "vertex %d is not finite", i);
        area += (double)xy[2 * i] * xy[2 * j + 1] - (double)xy[2 * j] * xy[2 * i + 1];
    }
    if (fabs(0.5 * area) < 1e-6) return fail(VPMC_E_POLYGON, "aperture polygon has zero area");
    std::vector<float2> v(n);
    for (int i = 0; i < n; ++i) v[i] = make_float2(xy[2 * i], xy[2 * i + 1]);
    for (int i = 0; i < n; ++i) {
        const float2 &a = v[i], &b = v[(i + 1) % n];
        if (a.x == b.x && a.y == b.y) return fail(VPMC_E_POLYGON, "repeated vertex %d", i);
        for (int j = i + 2; j < n; ++j) {
            if (i == 0 && j == n - 1) continue;   // adjacent through the closing edge
            if (segments_intersect(a, b, v[j], v[(j + 1) % n]))
                return fail(VPMC_E_POLYGON, "aperture polygon edges %d and %d intersect", i, j);
        }
    }
    return VPMC_OK;
}

int validate_beam(const vpmc_beam *b) {
    if (!b) return fail(VPMC_E_ARG, "beam is NULL");
    if (!finite3(b->iso_mm) || !finite3(b->ex) || !finite3(b->ey) || !finite3(b->ez))
        return fail(VPMC_E_ARG, "beam frame has non-finite values");
    const float *e[3] = {b->ex, b->ey, b->ez};
    for (int i = 0; i < 3; ++i) {
        const double n = e[i][0] * (double)e[i][0] + e[i][1] * (double)e[i][1] + e[i][2] * (double)e[i][2];
        if (fabs(n - 1.0) > 1e-4) return fail(VPMC_E_ARG, "beam axis %d is not a unit vector", i);
        for (int j = i + 1; j < 3; ++j) {
            const double d = e[i][0] * (double)e[j][0] + e[i][1] * (double)e[j][1] + e[i][2] * (double)e[j][2];
            if (fabs(d) > 1e-4) return fail(VPMC_E_ARG, "beam axes %d and %d are not orthogonal", i, j);
        }
    }
    const double cz[3] = {b->ex[1] * (double)b->ey[2] - b->ex[2] * (double)b->ey[1],
                          b->ex[2] * (double)b->ey[0] - b->ex[0] * (double)b->ey[2],
                          b->ex[0] * (double)b->ey[1] - b->ex[1] * (double)b->ey[0]};
    if (cz[0] * b->ez[0] + cz[1] * b->ez[1] + cz[2] * b->ez[2] < 0.999)
        return fail(VPMC_E_ARG, "beam frame is not right-handed");
    return VPMC_OK;
}

int validate_spots(const vpmc_spot *spots, int n, double *T) {
    if (n < 0) return fail(VPMC_E_ARG, "n_spots < 0");
    if (n > 0 && !spots) return fail(VPMC_E_ARG, "spots is NULL");
    *T = 0.0;
    for (int i = 0; i < n; ++i) {
        const vpmc_spot &s = spots[i];
        if (!isfinite(s.x_mm) || !isfinite(s.y_mm) || !isfinite(s.sigma_mm) || s.sigma_mm < 0 ||
            !isfinite(s.energy_sigma_mev) || s.energy_sigma_mev < 0 || !isfinite(s.weight) || s.weight < 0)
            return fail(VPMC_E_ARG, "spot %d has invalid position, sigma or weight", i);
        if (!(s.energy_mev > E_LO) || !(s.energy_mev <= E_HI))
            return fail(VPMC_E_RANGE, "spot %d energy %g MeV outside (1, 256]", i, (double)s.energy_mev);
        const double emax = std::min((double)s.energy_mev + 6.0 * s.energy_sigma_mev, E_HI);
        *T += (double)s.weight * emax;
    }
    return VPMC_OK;
}

int validate_scen(const vpmc_scenario *sc, int n) {
    if (n < 1) return fail(VPMC_E_ARG, "n_scen must be >= 1");
    if (!sc) return fail(VPMC_E_ARG, "scenarios is NULL");
    for (int i = 0; i < n; ++i)
        if (!finite3(sc[i].shift_mm) || !(sc[i].range_scale >= 0.5f && sc[i].range_scale <= 2.0f))
            return fail(VPMC_E_ARG, "scenario %d invalid (shift finite, range_scale in [0.5, 2])", i);
    return VPMC_OK;
}

int pick_k(const vpmc_opts *o, double T, int *k_out) {
    int k = o->fixed_point_bits;
    const double lim = ldexp(1.0, 62);
    if (k == 0) {
        k = 40;
        while (k > 0 && T * ldexp(1.0, k) > lim) --k;
        if (k < 16) return fail(VPMC_E_RANGE, "weighted energy bound %g too large for int64 tallies", T);
    } else {
        if (k < 1 || k > 62) return fail(VPMC_E_ARG, "fixed_point_bits must be 0 or in [1, 62]");
        if (T * ldexp(1.0, k) > lim)
            return fail(VPMC_E_RANGE, "fixed_point_bits=%d overflows for energy bound %g", k, T);
    }
    *k_out = k;
    return VPMC_OK;
}

// Device bytes a dense run needs at least (tallies, batch grids, LET,
// staging, spot tables); checked against max_device_bytes before any HIP
// call.  The allocator re-checks with what the context already holds.
size_t dense_bytes(size_t nvox, int n_scen, int n_spots, int B, bool let, bool dev_out, bool dose, bool sigma) {
    size_t b = (size_t)n_scen * nvox * 8 * (let ? 2 : 1);
    if (B > 1) b += nvox * 16;
    b += (size_t)n_scen * NLEDGER * 8 + (size_t)std::max(1, n_spots) * sizeof(SpotDev) + 16 +
         (size_t)B * (n_spots + 1) * 8;
    if (!dev_out) b += (dose ? nvox * 4 : 0) + (sigma ? nvox * 4 : 0);
    return b;
}

// Bytes of one resident influence-matrix row (dense int64 slot, touched-block
// bytes, chunk counters); a CSR run keeps at least one and spends at most half
// of max_device_bytes on them.
size_t csr_slot_bytes(size_t nvox) {
    const size_t nblk = (nvox + 31) / 32, nchunk = (nblk + 255) / 256;
    return nblk * 32 * 8 + ((nblk + 255) & ~(size_t)255) + nchunk * 8 + 4;
}

// ---------------------------------------------------------------- CSR runner
struct BatchField {
    int field_id;
    const vpmc_spot *spots;
    int n_spots;
};

int grow_keep(vpmc_ctx *c, DevBuf &b, size_t keep_bytes, size_t bytes, size_t cap_limit, hipStream_t st) {
    if (bytes <= b.cap) return VPMC_OK;
    if (cap_limit && c->bytes + (bytes - b.cap) > cap_limit)
        return fail(VPMC_E_OOM, "CSR storage of %zu bytes exceeds max_device_bytes", bytes);
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, bytes));
    if (b.ptr) {
        if (keep_bytes) HIP_TRY(hipMemcpyAsync(p, b.ptr, keep_bytes, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(b.ptr));
        c->bytes -= b.cap;
    }
    b.ptr = p;
    b.cap = bytes;
    c->bytes += bytes;
    return VPMC_OK;
}

// LDS tile box of a row (voxel indices, x fastest): the voxels along the
// spot's central ray from its CT entry to 1.15 x its CSDA range in water
// (less the range shifter) + 10 mm,
// widened laterally by the largest half-width (<= 15 mm, 0.5 mm steps) that
// keeps the box within cap voxels.  No box (tn = 0) when the ray misses the
// grid or no width fits.
static void tile_box(const FieldDev &f, const SpotDev &sp, const ScenDev &sc, const GeomDev &g, int cap, int lo[3],
                     int n[3]) {
    lo[0] = lo[1] = lo[2] = 0;
    n[0] = n[1] = n[2] = 0;
    if (cap <= 0) return;
    const int gn[3] = {g.nx, g.ny, g.nz};
    double p0[3], d[3], glo[3], ghi[3];
    for (int k = 0; k < 3; ++k) {
        p0[k] = (double)f.iso[k] + sp.x * (double)f.ex[k] + sp.y * (double)f.ey[k] - (double)sc.shift[k];
        d[k] = f.ez[k];
        glo[k] = g.lo[k];
        ghi[k] = g.lo[k] + gn[k] * (double)g.sp[k];
    }
    double tn = -1e30, tf = 1e30;
    for (int k = 0; k < 3; ++k) {
        if (std::fabs(d[k]) < 1e-12) {
            if (p0[k] < glo[k] || p0[k] >= ghi[k]) return;
            continue;
        }
        const double t1 = (glo[k] - p0[k]) / d[k], t2 = (ghi[k] - p0[k]) / d[k];
        tn = std::max(tn, std::min(t1, t2));
        tf = std::min(tf, std::max(t1, t2));
    }
    if (!(tf > tn)) return;
    // water range left after the range shifter (its water-equivalent
    // thickness taken low, 0.95 x rho x t), with 15 % and 10 mm to spare
    double rw = 10.0 * range_host(MAT_WATER, std::min((double)sp.e0, E_HI));
    if (f.has_rs) rw -= 0.95 * (double)f.rs_rho * (double)f.rs_t;
    const double reach = 1.15 * std::max(rw, 0.0) + 10.0;
    const double t1 = std::min(tf, tn + reach);
    int mn[3], mx[3], a = 0;
    for (int k = 0; k < 3; ++k) {
        auto cell = [&](double t) {
            const int i = (int)std::floor((p0[k] + t * d[k] - glo[k]) / g.sp[k]);
            return std::min(std::max(i, 0), gn[k] - 1);
        };
        mn[k] = std::min(cell(tn), cell(t1));
        mx[k] = std::max(cell(tn), cell(t1));
        if (std::fabs(d[k]) > std::fabs(d[a])) a = k;
    }
    for (double h = 15.0; h >= 0.0; h -= 0.5) {
        int l[3], w[3];
        size_t vol = 1;
        for (int k = 0; k < 3; ++k) {
            const int hk = k == a ? 0 : (int)std::floor(h / g.sp[k]);
            l[k] = std::max(0, mn[k] - hk);
            w[k] = std::min(gn[k] - 1, mx[k] + hk) - l[k] + 1;
            vol *= (size_t)w[k];
        }
        if (vol <= (size_t)cap) {
            for (int k = 0; k < 3; ++k) {
                lo[k] = l[k];
                n[k] = w[k];
            }
            return;
        }
    }
}

int run_csr(vpmc_ctx *c, const std::vector<BatchField> &bf, const vpmc_scenario *scen, int n_scen, const vpmc_opts *o,
            int k, float *dose_gy, double *ledger_mev, int64_t *row_ptr) {
    const size_t nvox = c->nvox;
    const bool dev_out = (o->flags & VPMC_DEVICE_PTRS) != 0;
    const size_t cap = o->max_device_bytes;
    hipStream_t st = (hipStream_t)o->hip_stream;
    // histories per lane: the caller's, else the one tuned for a field, else
    // the last tuned one, else 4 (per epoch: the field with most of its rows)
    auto field_hpl = [&](uint32_t field_id) {
        if (o->hist_per_lane > 0) return o->hist_per_lane;
        if (field_id < VPMC_MAX_FIELDS && c->tuned_csr_hpl_field[field_id]) return c->tuned_csr_hpl_field[field_id];
        return c->tuned_csr_hpl ? c->tuned_csr_hpl : 4;
    };
    int rc;

    // fields, polygons, spots (flattened), rows in (scenario, field, spot) order
    const int nf = (int)bf.size();
    std::vector<FieldDev> ftab(nf);
    std::vector<int> poff(nf);
    std::vector<float2> polys;
    std::vector<SpotDev> sd;
    std::vector<int> spot_base(nf);
    for (int f = 0; f < nf; ++f) {
        const FieldState &fs = c->fields[bf[f].field_id];
        ftab[f] = fs.dev;
        poff[f] = (int)polys.size();
        polys.insert(polys.end(), fs.poly.begin(), fs.poly.end());
        spot_base[f] = (int)sd.size();
        for (int i = 0; i < bf[f].n_spots; ++i) {
            const vpmc_spot &s = bf[f].spots[i];
            SpotDev d{};
            d.x = s.x_mm; d.y = s.y_mm; d.e0 = s.energy_mev; d.sigma = s.sigma_mm; d.esig = s.energy_sigma_mev;
            d.emax = (float)std::min((double)s.energy_mev + 6.0 * s.energy_sigma_mev, E_HI);
            d.nh = s.n_histories;
            d.scale = s.n_histories ? (float)ldexp((double)s.weight / (double)s.n_histories, k) : 0.0f;
            sd.push_back(d);
        }
    }
    if (polys.size() > (size_t)POLY_LDS)
        return fail(VPMC_E_ARG, "fields have %zu aperture vertices in total (max %d)", polys.size(), POLY_LDS);
    if (polys.empty()) polys.push_back(make_float2(0.f, 0.f));
    if (sd.empty()) sd.push_back(SpotDev{});
    std::vector<RowDev> rows;
    for (int sc = 0; sc < n_scen; ++sc)
        for (int f = 0; f < nf; ++f)
            for (int i = 0; i < bf[f].n_spots; ++i) {
                RowDev r{};
                r.field = f;
                r.field_id = (uint32_t)bf[f].field_id;
                r.spot = (uint32_t)i;
                r.spot_global = (uint32_t)(spot_base[f] + i);
                r.scen = sc;
                r.n_hist = bf[f].spots[i].n_histories;
                rows.push_back(r);
            }
    const int R = (int)rows.size();
    std::vector<ScenDev> stab(n_scen);
    for (int i = 0; i < n_scen; ++i) {
        for (int q = 0; q < 3; ++q) stab[i].shift[q] = scen[i].shift_mm[q];
        stab[i].range_scale = scen[i].range_scale;
    }

    // launch shape of the work queue and the LDS tile it leaves per workgroup
    int dev_cus = 256;
    size_t lds_wg = 64 * 1024;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
            dev_cus = prop.multiProcessorCount;
            lds_wg = prop.sharedMemPerBlock;
        }
    }
    const int q_threads = queue_threads(o->physics,
                                        o->block_threads ? o->block_threads
                                                         : (c->tuned_csr_threads ? c->tuned_csr_threads : 1024));
    const int q_blocks = o->grid_blocks ? o->grid_blocks
                         : (c->tuned_csr_blocks ? c->tuned_csr_blocks
                                                : std::max(1, dev_cus * (o->physics == 0 ? 12 : 16) / (q_threads / 64)));
    int tile_cap = queue_tile_cap(o->physics, q_threads);
    {
        const size_t stat = (o->physics == 0 ? TAB_FLOATS : TAB_HI_FLOATS) * 4 + POLY_LDS * 8 + 256;
        tile_cap = (int)std::min<size_t>((size_t)tile_cap, lds_wg > stat ? (lds_wg - stat) / 8 : 0);
    }
    for (RowDev &r : rows)
        tile_box(ftab[r.field], sd[r.spot_global], stab[r.scen], c->geom, tile_cap, r.tlo, r.tn);

    // slots: dense int64 grid + touched-block bytes per resident row
    const size_t nblk = (nvox + 31) / 32, nchunk = (nblk + 255) / 256;
    const size_t gstride = nblk * 32, mstride = (nblk + 255) & ~(size_t)255;
    const size_t slot_bytes = csr_slot_bytes(nvox);
    // row slots: half of the cap, else 40 % of the free device memory up to
    // 96 GiB (about 1100 head rows of 84 MB: fewer, longer epochs, so the
    // tail of each epoch's last chunks weighs less)
    size_t budget = cap ? (cap > c->bytes ? cap - c->bytes : 0) / 2 : ((size_t)24 << 30);
    if (!cap) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            budget = std::max(budget, std::min((size_t)(0.4 * (double)(free_b + (c->n_slots ? c->slot_grid.cap : 0))),
                                               (size_t)96 << 30));
    }
    int G = o->max_slots > 0 ? std::min(o->max_slots, kMaxSlots) : kMaxSlots;
    G = (int)std::min<size_t>((size_t)G, budget / slot_bytes);
    G = std::min(G, std::max(R, 1));
    if (G < 1) return fail(VPMC_E_OOM, "no room for one influence-matrix slot (%zu bytes)", slot_bytes);
    if (c->n_slots < G || c->slot_nvox != nvox || c->slots_dirty) {
        const int Ga = std::max(G, c->slot_nvox == nvox ? c->n_slots : 0);
        if ((rc = ensure(c, c->slot_grid, (size_t)Ga * gstride * 8, cap))) return rc;
        if ((rc = ensure(c, c->slot_mark, (size_t)Ga * mstride, cap))) return rc;
        if ((rc = ensure(c, c->slot_cnt, (size_t)Ga * nchunk * 4, cap))) return rc;
        if ((rc = ensure(c, c->slot_coff, (size_t)Ga * nchunk * 4, cap))) return rc;
        if ((rc = ensure(c, c->slot_rowcnt, (size_t)Ga * 4, cap))) return rc;
        HIP_TRY(hipMemsetAsync(c->slot_grid.ptr, 0, (size_t)Ga * gstride * 8, st));
        HIP_TRY(hipMemsetAsync(c->slot_mark.ptr, 0, (size_t)Ga * mstride, st));
        c->n_slots = Ga;
        c->slot_nvox = nvox;
        c->slots_dirty = false;
    }

    // epochs, their histories per lane and chunk prefixes
    const int E = (R + G - 1) / std::max(G, 1);
    std::vector<unsigned long long> choff;
    std::vector<size_t> ep_choff(E);
    std::vector<unsigned long long> ep_chunks(E);
    std::vector<int> ep_hpl(E);
    int hpl_max = 1;
    for (int e = 0; e < E; ++e) {
        const int r0 = e * G, r1 = std::min(R, r0 + G);
        int best_f = -1, best_n = 0;
        for (int r = r0; r < r1;) {   // rows of one field are contiguous within a scenario
            int r2 = r;
            while (r2 < r1 && rows[r2].field_id == rows[r].field_id) ++r2;
            if (r2 - r > best_n) { best_n = r2 - r; best_f = (int)rows[r].field_id; }
            r = r2;
        }
        ep_hpl[e] = field_hpl(best_f < 0 ? 0u : (uint32_t)best_f);
        hpl_max = std::max(hpl_max, ep_hpl[e]);
        const unsigned long long chunk = 64ull * (unsigned long long)ep_hpl[e];
        ep_choff[e] = choff.size();
        unsigned long long acc = 0;
        choff.push_back(0);
        for (int r = r0; r < r1; ++r) {
            acc += (rows[r].n_hist + chunk - 1) / chunk;
            choff.push_back(acc);
        }
        ep_chunks[e] = acc;
    }
    if ((rc = ensure(c, c->rows, std::max<size_t>(1, rows.size()) * sizeof(RowDev), cap))) return rc;
    if ((rc = ensure(c, c->chunk_off, std::max<size_t>(1, choff.size()) * 8, cap))) return rc;
    if ((rc = ensure(c, c->heads, std::max(1, E) * 8, cap))) return rc;
    if ((rc = ensure(c, c->row_off, std::max(1, R) * 8, cap))) return rc;
    if ((rc = ensure(c, c->row_nnz, std::max(1, R) * 8, cap))) return rc;
    if ((rc = ensure(c, c->used, 8, cap))) return rc;
    if ((rc = ensure(c, c->flags, 8, cap))) return rc;
    if ((rc = ensure(c, c->fields_tab, nf * sizeof(FieldDev), cap))) return rc;
    if ((rc = ensure(c, c->poly_off, nf * sizeof(int), cap))) return rc;
    if ((rc = ensure(c, c->polys, polys.size() * sizeof(float2), cap))) return rc;
    if ((rc = ensure(c, c->spots, sd.size() * sizeof(SpotDev), cap))) return rc;
    if ((rc = ensure(c, c->scen_tab, n_scen * sizeof(ScenDev), cap))) return rc;
    if ((rc = ensure(c, c->ledger, (size_t)n_scen * NLEDGER * 8, cap))) return rc;
    if ((rc = ensure(c, c->stats, 16, cap))) return rc;
    if (rows.size()) HIP_TRY(hipMemcpyAsync(c->rows.ptr, rows.data(), rows.size() * sizeof(RowDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->chunk_off.ptr, choff.data(), choff.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->fields_tab.ptr, ftab.data(), nf * sizeof(FieldDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->poly_off.ptr, poff.data(), nf * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->polys.ptr, polys.data(), polys.size() * sizeof(float2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->spots.ptr, sd.data(), sd.size() * sizeof(SpotDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->scen_tab.ptr, stab.data(), n_scen * sizeof(ScenDev), hipMemcpyHostToDevice, st));
    // initial CSR capacity: the previous run's total, else a per-row guess
    unsigned long long want = c->csr_cap_hint ? c->csr_cap_hint : (unsigned long long)std::max(R, 1) * 16384ull;
    want = std::min<unsigned long long>(want, (unsigned long long)std::max(R, 1) * nvox);
    if (c->csr_cap < want) {
        if ((rc = grow_keep(c, c->csr_col, 0, want * 4, cap, st))) return rc;
        if ((rc = grow_keep(c, c->csr_q, 0, want * 8, cap, st))) return rc;
        c->csr_cap = want;
    }
    c->csr_valid = false;
    c->slots_dirty = true;   // cleared again when every epoch has been compacted

    // surrogate queue: sized for the largest epoch (VPs beyond it cross the
    // block with the plain transport)
    const bool sur_on = (o->flags & VPMC_SURROGATE) != 0;
    unsigned long long sur_cap = 0, deferred = 0;
    if (sur_on) {
        for (int e = 0; e < E; ++e) {
            unsigned long long h = 0;
            for (int r = e * G; r < std::min(R, (e + 1) * G); ++r) h += rows[r].n_hist;
            sur_cap = std::max(sur_cap, h);
        }
        sur_cap = std::max(1ull, std::min(sur_cap, kSurMaxRecords));
        if ((rc = ensure(c, c->sur_rec, sur_cap * sizeof(DeferRec), cap))) return rc;
        if ((rc = ensure(c, c->sur_out, sur_cap * MLP_OUT * sizeof(float), cap))) return rc;
        if ((rc = ensure(c, c->sur_cnt, sizeof(unsigned long long), cap))) return rc;
    }

    QueueDev Q{};
    if (sur_on) {
        Q.sur.enabled = 1;
        Q.sur.d_fallback = c->sur_dfb;
        Q.sur.count = (unsigned long long *)c->sur_cnt.ptr;
        Q.sur.capacity = sur_cap;
        Q.sur.rec = (DeferRec *)c->sur_rec.ptr;
    }
    Q.rows = (const RowDev *)c->rows.ptr;
    Q.hist_per_lane = hpl_max;
    Q.fields = (const FieldDev *)c->fields_tab.ptr;
    Q.poly_off = (const int *)c->poly_off.ptr;
    Q.polys = (const float2 *)c->polys.ptr;
    Q.n_poly_total = (int)polys.size();
    Q.spots = (const SpotDev *)c->spots.ptr;
    Q.scen = (const ScenDev *)c->scen_tab.ptr;
    Q.key0 = (uint32_t)(o->seed & 0xffffffffu);
    Q.seed_hi = (uint32_t)(o->seed >> 32);
    Q.physics = o->physics;
    Q.div = 0;
    for (const FieldDev &fd : ftab)
        if (fd.div || fd.vsad > 0.0f) Q.div = 1;
    Q.grid = (unsigned long long *)c->slot_grid.ptr;
    Q.mark = (uint8_t *)c->slot_mark.ptr;
    Q.nvox = nvox; Q.nblk = nblk; Q.nchunk = nchunk;
    Q.gstride = gstride; Q.mstride = mstride;
    Q.ledger = (unsigned long long *)c->ledger.ptr;
    Q.stats = (unsigned long long *)c->stats.ptr;
    Q.tables = c->d_tables;
    Q.iter_cap = o->queue_cap ? (unsigned long long)o->queue_cap : kDefaultQueueCap;
    Q.flags = (unsigned int *)c->flags.ptr;

    if ((rc = ensure(c, c->q_stage, queue_stage_floats(q_blocks, q_threads, hpl_max) * sizeof(float), cap))) return rc;
    if ((rc = ensure(c, c->q_rownext, (size_t)std::max(R, 1) * 8, cap))) return rc;
    Q.stage = (float *)c->q_stage.ptr;
    Q.refill_min = kRefillMin;
    Q.tile_cap = tile_cap;
    while (c->events.size() < 4) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        c->events.push_back(ev);
    }
    // counters are cleared by fill kernels (no memset nodes in a captured graph)
    auto clear_counters = [&]() -> int {
        HIP_TRY(launch_fill_u64((unsigned long long *)c->ledger.ptr, (size_t)n_scen * NLEDGER, 0ull, st));
        HIP_TRY(launch_fill_u64((unsigned long long *)c->stats.ptr, 2, 0ull, st));
        HIP_TRY(launch_fill_u64((unsigned long long *)c->heads.ptr, (size_t)std::max(1, E), 0ull, st));
        HIP_TRY(launch_fill_u64((unsigned long long *)c->q_rownext.ptr, (size_t)std::max(1, R), 0ull, st));
        HIP_TRY(launch_fill_u64((unsigned long long *)c->used.ptr, 1, 0ull, st));
        HIP_TRY(launch_fill_u64((unsigned long long *)c->flags.ptr, 1, 0ull, st));
        return VPMC_OK;
    };
    auto epoch_queue = [&](int e) {
        QueueDev Qe = Q;
        Qe.row_begin = e * G;
        Qe.n_rows = std::min(R, (e + 1) * G) - e * G;
        Qe.chunk_off = (const unsigned long long *)c->chunk_off.ptr + ep_choff[e];
        Qe.n_chunks = ep_chunks[e];
        Qe.hist_per_lane = ep_hpl[e];
        Qe.head = (unsigned long long *)c->heads.ptr + e;
        Qe.row_next = (unsigned long long *)c->q_rownext.ptr + Qe.row_begin;
        return Qe;
    };
    // compaction passes of one epoch (count per chunk, scan per row; emit)
    auto count_rows = [&](const QueueDev &Qe) -> hipError_t {
        hipError_t he = launch_csr_count(Qe, (unsigned int *)c->slot_cnt.ptr, st);
        if (he == hipSuccess)
            he = launch_csr_chunk_scan((const unsigned int *)c->slot_cnt.ptr, (unsigned int *)c->slot_coff.ptr,
                                       (unsigned int *)c->slot_rowcnt.ptr, Qe.n_rows, nchunk, st);
        return he;
    };
    auto emit_rows = [&](const QueueDev &Qe) -> hipError_t {
        return launch_csr_emit(Qe, (const unsigned int *)c->slot_cnt.ptr, (const unsigned int *)c->slot_coff.ptr,
                               (const unsigned long long *)c->row_off.ptr, (const unsigned long long *)c->row_nnz.ptr,
                               (int32_t *)c->csr_col.ptr, (long long *)c->csr_q.ptr, c->csr_cap,
                               (unsigned int *)c->flags.ptr, st);
    };
    HIP_TRY(hipEventRecord(c->events[0], st));
    double transport_ms = 0.0;
    unsigned long long used_host = 0;
    bool done = false;
    if ((o->flags & VPMC_GRAPH) && !sur_on) {
        // whole run as one graph: rows that do not fit the current CSR
        // capacity raise the overflow flag, and the eager path below reruns
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        // capture on a private stream (the legacy default stream cannot be
        // captured); the graph is then launched on the caller's stream
        if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user_st = st;
        st = c->cap_stream;
        HIP_TRY(hipStreamSynchronize(user_st));
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int crc = clear_counters();
        for (int e = 0; e < E && crc == VPMC_OK; ++e) {
            const QueueDev Qe = epoch_queue(e);
            hipError_t he = hipSuccess;
            if (Qe.n_chunks) he = launch_queue(c->geom, Qe, q_blocks, q_threads, st);
            if (he == hipSuccess) he = count_rows(Qe);
            if (he == hipSuccess)
                he = launch_csr_offsets((const unsigned int *)c->slot_rowcnt.ptr, Qe.n_rows, Qe.row_begin,
                                        (unsigned long long *)c->row_off.ptr, (unsigned long long *)c->row_nnz.ptr,
                                        (unsigned long long *)c->used.ptr, c->csr_cap, (unsigned int *)c->flags.ptr, st);
            if (he == hipSuccess) he = emit_rows(Qe);
            if (he != hipSuccess) crc = fail(VPMC_E_DEVICE, "graph capture launch: %s", hipGetErrorString(he));
        }
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        st = user_st;
        if (crc) { if (graph) (void)hipGraphDestroy(graph); return crc; }
        HIP_TRY(ce);
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie == hipSuccess) {
            HIP_TRY(hipEventRecord(c->events[2], st));
            ie = hipGraphLaunch(exec, st);
            HIP_TRY(hipEventRecord(c->events[3], st));
        }
        (void)hipGraphDestroy(graph);
        HIP_TRY(hipStreamSynchronize(st));
        if (exec) (void)hipGraphExecDestroy(exec);
        HIP_TRY(ie);
        unsigned long long fl8 = 0, used_now = 0;
        HIP_TRY(hipMemcpy(&fl8, c->flags.ptr, 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&used_now, c->used.ptr, 8, hipMemcpyDeviceToHost));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->events[2], c->events[3]));
        if (!(fl8 & 1ull)) {
            transport_ms = ms;   // whole graph (transport dominated)
            used_host = used_now;
            done = true;
        } else {
            const unsigned long long ncap = std::max<unsigned long long>(used_now, c->csr_cap * 2);
            if ((rc = grow_keep(c, c->csr_col, 0, ncap * 4, cap, st))) return rc;
            if ((rc = grow_keep(c, c->csr_q, 0, ncap * 8, cap, st))) return rc;
            c->csr_cap = ncap;
        }
    }
    if (!done) {
        if ((rc = clear_counters())) return rc;
        for (int e = 0; e < E; ++e) {
            const QueueDev Qe = epoch_queue(e);
            if (sur_on) HIP_TRY(launch_fill_u64((unsigned long long *)c->sur_cnt.ptr, 1, 0ull, st));
            HIP_TRY(hipEventRecord(c->events[2], st));
            if (Qe.n_chunks) HIP_TRY(launch_queue(c->geom, Qe, q_blocks, q_threads, st));
            if (sur_on && Qe.n_chunks) {
                // deferred brass entries of this epoch: network, then resume
                unsigned long long cnt = 0;
                HIP_TRY(hipMemcpyAsync(&cnt, c->sur_cnt.ptr, sizeof cnt, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                const unsigned long long nq = std::min(cnt, sur_cap);
                deferred += nq;
                const DeferRec *rec = (const DeferRec *)c->sur_rec.ptr;
                float *sout = (float *)c->sur_out.ptr;
                if (nq) {
                    HIP_TRY(mlp_infer(nullptr, rec, (int)nq, (const __bf16 *)c->mlp_wb.ptr, (const float *)c->mlp_w.ptr,
                                      sout, st));
                    HIP_TRY(launch_sur_resume_csr(c->geom, Qe, rec, sout, nq, c->sur_plo, c->sur_phi, st));
                }
            }
            HIP_TRY(hipEventRecord(c->events[3], st));
            HIP_TRY(count_rows(Qe));
            HIP_TRY(launch_csr_offsets((const unsigned int *)c->slot_rowcnt.ptr, Qe.n_rows, Qe.row_begin,
                                       (unsigned long long *)c->row_off.ptr, (unsigned long long *)c->row_nnz.ptr,
                                       (unsigned long long *)c->used.ptr, ~0ull, (unsigned int *)c->flags.ptr, st));
            unsigned long long used_now = 0;
            unsigned int fl_now = 0;
            HIP_TRY(hipMemcpyAsync(&used_now, c->used.ptr, 8, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(&fl_now, c->flags.ptr, 4, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, c->events[2], c->events[3]));
            transport_ms += ms;
            if (used_now > c->csr_cap) {   // grow, keeping the rows already written
                const unsigned long long ncap = std::max<unsigned long long>(used_now, c->csr_cap * 2);
                if ((rc = grow_keep(c, c->csr_col, used_host * 4, ncap * 4, cap, st))) return rc;
                if ((rc = grow_keep(c, c->csr_q, used_host * 8, ncap * 8, cap, st))) return rc;
                c->csr_cap = ncap;
            }
            HIP_TRY(emit_rows(Qe));   // also clears the epoch's slots
            used_host = used_now;
            if (fl_now & kFlagAborted) break;   // no further epochs: the run fails below
        }
    }
    unsigned int fl = 0;
    std::vector<unsigned long long> roff(std::max(R, 1)), rnnz(std::max(R, 1));
    std::vector<long long> led((size_t)n_scen * NLEDGER);
    unsigned long long stv[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&fl, c->flags.ptr, 4, hipMemcpyDeviceToHost, st));
    if (R) {
        HIP_TRY(hipMemcpyAsync(roff.data(), c->row_off.ptr, R * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(rnnz.data(), c->row_nnz.ptr, R * 8, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(led.data(), c->ledger.ptr, led.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(stv, c->stats.ptr, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (fl & 2u) return fail(VPMC_E_DEVICE, "influence-matrix count and emit passes disagree");
    c->slots_dirty = false;   // every launched epoch was compacted, which clears its slots
    if (fl & kFlagAborted)
        return fail(VPMC_E_ABORTED, "a wavefront reached the work-queue cap of %llu iterations; no rows written",
                    (unsigned long long)Q.iter_cap);
    std::vector<int64_t> rp((size_t)R + 1);
    for (int r = 0; r < R; ++r) rp[r] = (int64_t)roff[r];
    rp[R] = (int64_t)used_host;
    for (int r = 0; r < R; ++r)
        if (roff[r] + rnnz[r] != (r + 1 < R ? roff[r + 1] : used_host))
            return fail(VPMC_E_DEVICE, "influence-matrix row offsets inconsistent at row %d", r);
    HIP_TRY(hipMemcpy(row_ptr, rp.data(), rp.size() * 8, dev_out ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    c->csr_total = used_host;
    c->csr_rows = R;
    c->csr_valid = true;
    c->csr_flags = o->flags;
    c->csr_cap_hint = used_host;
    c->last_k = k;
    if (ledger_mev)
        for (size_t i = 0; i < led.size(); ++i) ledger_mev[i] = ldexp((double)led[i], -k);
    // plan dose per scenario from its rows (contiguous in row order)
    c->last_nscen = 0;
    c->last_let = false;
    if (dose_gy) {
        if ((rc = ensure(c, c->tallies, (size_t)n_scen * nvox * 8, cap))) return rc;
        if (!dev_out && (rc = ensure(c, c->stage_dose, nvox * sizeof(float), cap))) return rc;
        const int rows_per_scen = R / std::max(n_scen, 1);
        for (int sc = 0; sc < n_scen; ++sc) {
            unsigned long long *dense = (unsigned long long *)c->tallies.ptr + (size_t)sc * nvox;
            HIP_TRY(hipMemsetAsync(dense, 0, nvox * 8, st));
            const unsigned long long b = rows_per_scen ? roff[(size_t)sc * rows_per_scen] : 0;
            const unsigned long long en = (sc + 1 < n_scen && rows_per_scen) ? roff[(size_t)(sc + 1) * rows_per_scen] : used_host;
            HIP_TRY(launch_csr_scatter((const int32_t *)c->csr_col.ptr, (const long long *)c->csr_q.ptr, b, en, dense, st));
            float *dd = dev_out ? dose_gy + (size_t)sc * nvox : (float *)c->stage_dose.ptr;
            HIP_TRY(launch_dose((const long long *)dense, nullptr, 1, c->geom, ldexp(MEV_TO_J, -k), dd, nullptr, nvox, st));
            if (!dev_out) HIP_TRY(hipMemcpyAsync(dose_gy + (size_t)sc * nvox, dd, nvox * 4, hipMemcpyDeviceToHost, st));
        }
        c->last_nscen = n_scen;
    }
    HIP_TRY(hipEventRecord(c->events[1], st));
    HIP_TRY(hipStreamSynchronize(st));
    float tot = 0.f;
    HIP_TRY(hipEventElapsedTime(&tot, c->events[0], c->events[1]));
    vpmc_stats S{};
    S.transport_ms = transport_ms;
    S.total_ms = tot;
    S.steps = stv[0];
    S.histories = stv[1];
    S.launches = (uint64_t)E;
    S.deferred = deferred;
    c->last_stats = S;
    return VPMC_OK;
}

// carve the activation buffers of a batch of up to `cap` samples
int mlp_buffers(vpmc_ctx *c, int cap, MlpBuffers *b) {
    const size_t H = MLP_HIDDEN;
    const size_t bytes = (size_t)cap * (MLP_IN * 2 + 4 * H * 2 + 4 * H * 4 + MLP_OUT * 4 * 2 + MLP_OUT_LD * 2 +
                                        H * 2 * 2 + 4) +
                         (size_t)kMlpSplit * H * H * 4 + ((size_t)cap / 32 + 1) * H * 4 +
                         32 * 256;   // 17 carvings, each rounded up to 256 B
    if (c->mlp_batch_cap < cap) {
        int rc = ensure(c, c->mlp_act, bytes, 0);
        if (rc) return rc;
        c->mlp_batch_cap = cap;
    }
    char *p = (char *)c->mlp_act.ptr;
    char *const end = p + c->mlp_act.cap;
    auto take = [&](size_t n) { char *q = p; p += (n + 255) & ~(size_t)255; return (void *)q; };
    b->w = (float *)c->mlp_w.ptr;
    b->wb = (__bf16 *)c->mlp_wb.ptr;
    b->x = (__bf16 *)take((size_t)cap * MLP_IN * 2);
    for (int i = 0; i < 4; ++i) b->h[i] = (__bf16 *)take((size_t)cap * H * 2);
    for (int i = 0; i < 4; ++i) b->z[i] = (float *)take((size_t)cap * H * 4);
    b->out = (float *)take((size_t)cap * MLP_OUT * 4);
    b->dout = (float *)take((size_t)cap * MLP_OUT * 4);
    b->dout_b = (__bf16 *)take((size_t)cap * MLP_OUT_LD * 2);
    b->dzb_a = (__bf16 *)take((size_t)cap * H * 2);
    b->dzb_b = (__bf16 *)take((size_t)cap * H * 2);
    b->wpart = (float *)take((size_t)kMlpSplit * H * H * 4);
    b->bpart = (float *)take(((size_t)cap / 32 + 1) * H * 4);
    b->loss = (float *)take((size_t)cap * 4);
    if (p > end) return fail(VPMC_E_OOM, "surrogate activation buffer too small");
    return VPMC_OK;
}

int mlp_require(vpmc_ctx *c) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    if (!c->mlp_ready) return fail(VPMC_E_STATE, "surrogate weights not set");
    HIP_TRY(hipSetDevice(c->device));
    return VPMC_OK;
}

}  // namespace

extern "C" {

int vpmc_version(void) { return 102; }

int vpmc_surrogate_param_count(void) { return mlp_param_count(); }

int vpmc_surrogate_set_weights(vpmc_ctx *c, const float *params, int n) {
    if (!c || !params) return fail(VPMC_E_ARG, "ctx/params is NULL");
    const int np = mlp_param_count();
    if (n != np) return fail(VPMC_E_ARG, "surrogate has %d parameters, got %d", np, n);
    for (int i = 0; i < n; ++i)
        if (!isfinite(params[i])) return fail(VPMC_E_ARG, "parameter %d is not finite", i);
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    int rc;
    if ((rc = ensure(c, c->mlp_w, np * 4, 0)) || (rc = ensure(c, c->mlp_wb, np * 2, 0)) ||
        (rc = ensure(c, c->mlp_m, np * 4, 0)) || (rc = ensure(c, c->mlp_v, np * 4, 0)) ||
        (rc = ensure(c, c->mlp_g, np * 4, 0)))
        return rc;
    HIP_TRY(hipMemcpy(c->mlp_w.ptr, params, np * 4, hipMemcpyHostToDevice));
    HIP_TRY(mlp_to_bf16((const float *)c->mlp_w.ptr, (__bf16 *)c->mlp_wb.ptr, np, nullptr));
    HIP_TRY(hipMemset(c->mlp_m.ptr, 0, np * 4));
    HIP_TRY(hipMemset(c->mlp_v.ptr, 0, np * 4));
    HIP_TRY(hipDeviceSynchronize());
    c->mlp_ready = true;
    c->mlp_step = 0;
    return VPMC_OK;
}

// Weights file: the 8 bytes "VPMCMLP1", a little-endian uint32 parameter
// count, then that many little-endian FP32 parameters in the layout of
// vpmc_surrogate_set_weights.
static const char kMlpMagic[8] = {'V', 'P', 'M', 'C', 'M', 'L', 'P', '1'};

int vpmc_surrogate_load(vpmc_ctx *c, const char *path) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!path) {   // disable: runs with VPMC_SURROGATE fail until weights are set again
        c->mlp_ready = false;
        return VPMC_OK;
    }
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(VPMC_E_ARG, "cannot open surrogate weights '%s'", path);
    const int np = mlp_param_count();
    char magic[8];
    uint32_t n = 0;
    std::vector<float> w(np);
    const bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kMlpMagic, 8) == 0 && fread(&n, 4, 1, fp) == 1 &&
                    n == (uint32_t)np && fread(w.data(), 4, np, fp) == (size_t)np && fgetc(fp) == EOF;
    fclose(fp);
    if (!ok) return fail(VPMC_E_ARG, "'%s' is not a surrogate weights file of %d parameters", path, np);
    return vpmc_surrogate_set_weights(c, w.data(), np);
}

int vpmc_surrogate_save(vpmc_ctx *c, const char *path) {
    if (!c || !path) return fail(VPMC_E_ARG, "ctx/path is NULL");
    const int np = mlp_param_count();
    std::vector<float> w(np);
    int rc = vpmc_surrogate_get_weights(c, w.data(), np);
    if (rc) return rc;
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(VPMC_E_ARG, "cannot create '%s'", path);
    const uint32_t n = (uint32_t)np;
    const bool ok = fwrite(kMlpMagic, 1, 8, fp) == 8 && fwrite(&n, 4, 1, fp) == 1 &&
                    fwrite(w.data(), 4, np, fp) == (size_t)np;
    if (fclose(fp) != 0 || !ok) return fail(VPMC_E_ARG, "writing '%s' failed", path);
    return VPMC_OK;
}

int vpmc_surrogate_config(vpmc_ctx *c, float d_fallback_mm, float p_lo, float p_hi) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!(d_fallback_mm >= 0.0f) || !isfinite(d_fallback_mm) || !(p_lo >= 0.0f) || !(p_lo <= p_hi) ||
        !(p_hi <= 1.0f))
        return fail(VPMC_E_ARG, "need d_fallback_mm >= 0 and 0 <= p_lo <= p_hi <= 1");
    c->sur_dfb = d_fallback_mm;
    c->sur_plo = p_lo;
    c->sur_phi = p_hi;
    return VPMC_OK;
}

int vpmc_surrogate_get_weights(vpmc_ctx *c, float *params, int n) {
    int rc = mlp_require(c);
    if (rc) return rc;
    if (!params || n != mlp_param_count()) return fail(VPMC_E_ARG, "need %d parameters", mlp_param_count());
    HIP_TRY(hipMemcpy(params, c->mlp_w.ptr, (size_t)n * 4, hipMemcpyDeviceToHost));
    return VPMC_OK;
}

int vpmc_surrogate_sample(vpmc_ctx *c, int field_id, const float *entries, int n, uint64_t seed, unsigned physics,
                          float *x, float *y, float *trans) {
    if (!c || !entries || !x || !y || !trans || n < 1) return fail(VPMC_E_ARG, "bad sample arguments");
    if (field_id < 0 || field_id >= VPMC_MAX_FIELDS || !c->fields[field_id].set)
        return fail(VPMC_E_STATE, "field %d not set", field_id);
    if (!c->fields[field_id].dev.has_block) return fail(VPMC_E_STATE, "field %d has no block", field_id);
    if (physics & ~VPMC_PHYS_ALL) return fail(VPMC_E_ARG, "unknown physics bits");
    for (int i = 0; i < n; ++i) {
        const float *e = entries + (size_t)i * 5;
        if (!isfinite(e[0]) || !isfinite(e[1]) || !(e[2] * e[2] + e[3] * e[3] < 1.0f) || !(e[4] > E_LO && e[4] <= E_HI))
            return fail(e[4] > E_LO && e[4] <= E_HI ? VPMC_E_ARG : VPMC_E_RANGE, "entry %d invalid", i);
    }
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    int rc;
    if ((rc = ensure(c, c->mlp_io, (size_t)n * (5 + 8 + 3 + 1) * 4 + 64, 0))) return rc;
    float *de = (float *)c->mlp_io.ptr, *dx = de + (size_t)n * 5, *dy = dx + (size_t)n * 8, *dt = dy + (size_t)n * 3;
    HIP_TRY(hipMemcpy(de, entries, (size_t)n * 5 * 4, hipMemcpyHostToDevice));
    HIP_TRY(launch_surrogate_sample(c->fields[field_id].dev, de, n, (uint32_t)(seed & 0xffffffffu),
                                    (uint32_t)(seed >> 32) ^ (uint32_t)field_id, physics, c->d_tables, dx, dy, dt,
                                    nullptr));
    HIP_TRY(hipMemcpy(x, dx, (size_t)n * 8 * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(y, dy, (size_t)n * 3 * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(trans, dt, (size_t)n * 4, hipMemcpyDeviceToHost));
    return VPMC_OK;
}

int vpmc_surrogate_forward(vpmc_ctx *c, const float *x, int n, float *out) {
    int rc = mlp_require(c);
    if (rc) return rc;
    if (!x || !out || n < 0) return fail(VPMC_E_ARG, "bad forward arguments");
    if (n == 0) return VPMC_OK;
    // fused inference in chunks of up to 1M samples
    const int cap = std::min(n, 1 << 20);
    if ((rc = ensure(c, c->mlp_io, (size_t)cap * (MLP_IN + MLP_OUT) * 4, 0))) return rc;
    float *dx = (float *)c->mlp_io.ptr, *dout = dx + (size_t)cap * MLP_IN;
    for (int s0 = 0; s0 < n; s0 += cap) {
        const int m = std::min(cap, n - s0);
        HIP_TRY(hipMemcpy(dx, x + (size_t)s0 * MLP_IN, (size_t)m * MLP_IN * 4, hipMemcpyHostToDevice));
        HIP_TRY(mlp_infer(dx, nullptr, m, (const __bf16 *)c->mlp_wb.ptr, (const float *)c->mlp_w.ptr, dout, nullptr));
        HIP_TRY(hipMemcpy(out + (size_t)s0 * MLP_OUT, dout, (size_t)m * MLP_OUT * 4, hipMemcpyDeviceToHost));
    }
    return VPMC_OK;
}

int vpmc_surrogate_loss_grad(vpmc_ctx *c, const float *x, const float *y, const float *trans, int n, float *grad,
                             double *loss) {
    int rc = mlp_require(c);
    if (rc) return rc;
    if (!x || !y || !trans || !grad || n < 1 || n > MLP_MAX_BATCH)
        return fail(VPMC_E_ARG, "need 1..%d samples and all buffers", MLP_MAX_BATCH);
    MlpBuffers b;
    if ((rc = mlp_buffers(c, n, &b))) return rc;
    if ((rc = ensure(c, c->mlp_io, (size_t)n * (MLP_IN + 4) * 4 + 64, 0))) return rc;
    double *dl = (double *)c->mlp_io.ptr;
    float *dx = (float *)(dl + 2), *dy = dx + (size_t)n * MLP_IN, *dt = dy + (size_t)n * 3;
    HIP_TRY(hipMemset(dl, 0, sizeof(double)));
    HIP_TRY(hipMemcpy(dx, x, (size_t)n * MLP_IN * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dy, y, (size_t)n * 3 * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dt, trans, (size_t)n * 4, hipMemcpyHostToDevice));
    HIP_TRY(mlp_to_bf16(dx, b.x, (size_t)n * MLP_IN, nullptr));
    HIP_TRY(mlp_loss_grad(b, dy, dt, n, (float *)c->mlp_g.ptr, dl, nullptr));
    double lmean = 0.0;
    HIP_TRY(hipMemcpy(&lmean, dl, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(grad, c->mlp_g.ptr, (size_t)mlp_param_count() * 4, hipMemcpyDeviceToHost));
    if (loss) *loss = lmean;
    return VPMC_OK;
}

int vpmc_surrogate_train(vpmc_ctx *c, const float *x, const float *y, const float *trans, int n, int epochs, int batch,
                         float lr, uint64_t seed, float *loss_per_epoch) {
    int rc = mlp_require(c);
    if (rc) return rc;
    if (!x || !y || !trans || n < 1 || epochs < 1 || batch < 16 || batch > MLP_MAX_BATCH || !(lr > 0.0f))
        return fail(VPMC_E_ARG, "bad training arguments");
    MlpBuffers b;
    if ((rc = mlp_buffers(c, batch, &b))) return rc;
    if ((rc = ensure(c, c->mlp_dx, (size_t)n * MLP_IN * 4, 0)) || (rc = ensure(c, c->mlp_dy, (size_t)n * 3 * 4, 0)) ||
        (rc = ensure(c, c->mlp_dt, (size_t)n * 4, 0)) || (rc = ensure(c, c->mlp_idx, (size_t)n * 4, 0)) ||
        (rc = ensure(c, c->mlp_io, (size_t)batch * 4 * 4 + 64, 0)))
        return rc;
    HIP_TRY(hipMemcpy(c->mlp_dx.ptr, x, (size_t)n * MLP_IN * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->mlp_dy.ptr, y, (size_t)n * 3 * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->mlp_dt.ptr, trans, (size_t)n * 4, hipMemcpyHostToDevice));
    double *bl = (double *)c->mlp_io.ptr;   // sum over the epoch's batches of the batch-mean loss
    float *by = (float *)(bl + 2), *bt = by + (size_t)batch * 3;
    std::vector<int> perm(n);
    uint64_t st = seed ^ 0x9E3779B97F4A7C15ull;
    const int np = mlp_param_count();
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {   // Fisher-Yates with xorshift64*
            st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
            const int j = (int)(((st * 0x2545F4914F6CDD1Dull) >> 11) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        HIP_TRY(hipMemcpy(c->mlp_idx.ptr, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemsetAsync(bl, 0, sizeof(double), nullptr));
        int nb = 0;
        for (int s0 = 0; s0 + batch <= n; s0 += batch, ++nb) {
            const int *idx = (const int *)c->mlp_idx.ptr + s0;
            HIP_TRY(mlp_gather((const float *)c->mlp_dx.ptr, idx, batch, MLP_IN, b.x, nullptr, nullptr));
            HIP_TRY(mlp_gather((const float *)c->mlp_dy.ptr, idx, batch, 3, nullptr, by, nullptr));
            HIP_TRY(mlp_gather((const float *)c->mlp_dt.ptr, idx, batch, 1, nullptr, bt, nullptr));
            HIP_TRY(mlp_loss_grad(b, by, bt, batch, (float *)c->mlp_g.ptr, bl, nullptr));
            HIP_TRY(mlp_adam((float *)c->mlp_w.ptr, (const float *)c->mlp_g.ptr, (float *)c->mlp_m.ptr,
                             (float *)c->mlp_v.ptr, (__bf16 *)c->mlp_wb.ptr, np, lr, ++c->mlp_step, nullptr));
        }
        double lsum = 0.0;
        HIP_TRY(hipMemcpy(&lsum, bl, sizeof(double), hipMemcpyDeviceToHost));
        if (loss_per_epoch) loss_per_epoch[ep] = nb ? (float)(lsum / nb) : 0.0f;
    }
    return VPMC_OK;
}

const char *vpmc_last_error(const vpmc_ctx *) { return g_err; }

int vpmc_create(vpmc_ctx **out, int hip_device) {
    if (!out) return fail(VPMC_E_ARG, "out is NULL");
    *out = nullptr;
    if (hip_device < -1) return fail(VPMC_E_ARG, "hip_device must be >= -1");
    vpmc_ctx *c = new (std::nothrow) vpmc_ctx();
    if (!c) return fail(VPMC_E_OOM, "host allocation failed");
    c->device = hip_device;
    (void)host_tables();
    if (hip_device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || hip_device >= n) {
            delete c;
            return fail(VPMC_E_DEVICE, "HIP device %d not available (%d devices)", hip_device, n);
        }
        std::vector<float> blob(TAB_FLOATS);
        pack_device_tables(blob.data());
        if ((e = hipSetDevice(hip_device)) != hipSuccess ||
            (e = hipMalloc(&c->d_tables, sizeof(float) * TAB_FLOATS)) != hipSuccess ||
            (e = hipMemcpy(c->d_tables, blob.data(), sizeof(float) * TAB_FLOATS, hipMemcpyHostToDevice)) !=
                hipSuccess) {
            if (c->d_tables) (void)hipFree(c->d_tables);
            delete c;
            return fail(VPMC_E_DEVICE, "table upload failed: %s", hipGetErrorString(e));
        }
        c->bytes = sizeof(float) * TAB_FLOATS;
        // the static scratch's device address on this device (current here)
        if ((e = scratch_device_ptr(hip_device, &c->scratch)) != hipSuccess) {
            (void)hipFree(c->d_tables);
            delete c;
            return fail(VPMC_E_DEVICE, "scratch address lookup failed: %s", hipGetErrorString(e));
        }
    }
    *out = c;
    return VPMC_OK;
}

void vpmc_destroy(vpmc_ctx *c) {
    if (!c) return;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        if (c->d_tables) (void)hipFree(c->d_tables);
        release(c->hu_buf);
        for (auto &f : c->fields) {
            release(f.poly_buf);
            release(f.sdf_buf);
            release(f.cell_off_buf);
            release(f.cell_edge_buf);
            release(f.cell_ref_buf);
        }
        for (DevBuf *b : {&c->tallies, &c->let_tallies, &c->qbatch, &c->s2, &c->ledger, &c->spots, &c->offsets,
                          &c->stage_dose, &c->stage_sigma, &c->stats, &c->slot_grid, &c->slot_mark, &c->slot_cnt,
                          &c->slot_coff, &c->slot_rowcnt, &c->q_stage, &c->q_rownext, &c->rows, &c->chunk_off, &c->heads, &c->row_off, &c->row_nnz, &c->used,
                          &c->flags, &c->fields_tab, &c->poly_off, &c->polys, &c->scen_tab, &c->csr_col,
                          &c->csr_q, &c->mlp_w, &c->mlp_wb, &c->mlp_m, &c->mlp_v, &c->mlp_g, &c->mlp_act,
                          &c->mlp_io, &c->mlp_dx, &c->mlp_dy, &c->mlp_dt, &c->mlp_idx, &c->sur_rec,
                          &c->sur_cnt, &c->sur_out, &c->opt_rp, &c->opt_col, &c->opt_val, &c->opt_roi, &c->opt_amax,
                          &c->opt_cnt, &c->opt_rcnt, &c->opt_crp, &c->opt_ccol, &c->opt_cval, &c->opt_piece,
                          &c->opt_poff, &c->opt_resid, &c->opt_fpart, &c->opt_gpart, &c->opt_vec, &c->opt_scal,
                          &c->opt_err, &c->opt_hist, &c->opt_dose, &c->opt_sidx, &c->opt_rstruct,
                          &c->opt_broi.off, &c->opt_broi.key,
                          &c->opt_broi.val, &c->opt_broi.work, &c->opt_bfull.off, &c->opt_bfull.key,
                          &c->opt_bfull.val, &c->opt_bfull.work, &c->cl_rp, &c->cl_map, &c->cl_start,
                          &c->cl_mass, &c->cl_cnt, &c->cl_out, &c->cl_col, &c->cl_q, &c->cl_ocell, &c->cl_oq, &c->cl_piece,
                          &c->cl_oval})
            release(*b);
        for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    }
    delete c;
}

int vpmc_atomic_rate(vpmc_ctx *c, int nx, int ny, int nz, uint64_t n_atomics, double *atomics_per_s) {
    if (!c || !atomics_per_s) return fail(VPMC_E_ARG, "ctx and atomics_per_s are required");
    if (nx < 16 || ny < 16 || nz < 16 || (size_t)nx * ny * nz >= ((size_t)1 << 31))
        return fail(VPMC_E_ARG, "grid must be at least 16^3 and below 2^31 voxels");
    if (n_atomics < 1024 || n_atomics > ((uint64_t)1 << 40)) return fail(VPMC_E_ARG, "n_atomics outside [1024, 2^40]");
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    const size_t nvox = (size_t)nx * ny * nz;
    unsigned long long *grid = nullptr;
    HIP_TRY(hipMalloc(&grid, nvox * 8));
    const int len = 100;   // voxels per track (~ steps per history of the head case)
    const unsigned long long tracks = (n_atomics + len - 1) / len;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipMemset(grid, 0, nvox * 8);
    // one warm-up pass, then the timed pass
    if (e == hipSuccess) e = launch_atomic_rate(grid, nx, ny, nz, std::min<unsigned long long>(tracks, 1 << 20), len,
                                                4.0f, 1u, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch_atomic_rate(grid, nx, ny, nz, tracks, len, 4.0f, 2u, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(grid);
    HIP_TRY(e);
    *atomics_per_s = ms > 0.0f ? (double)tracks * len / (ms * 1e-3) : 0.0;
    return VPMC_OK;
}

int vpmc_table_host(int material, int which, double *out, int n) {
    if (material < 0 || material >= NMAT || which < 0 || which > 4 || !out || n < 0)
        return fail(VPMC_E_ARG, "bad table request");
    const HostTables &t = host_tables();
    const double *src = which == 0 ? t.E : which == 1 ? t.R[material] : which == 2 ? t.W2[material]
                      : which == 3 ? t.T[material] : t.SN[material];
    memcpy(out, src, sizeof(double) * std::min(n, NE));
    return NE;
}

int vpmc_load_geometry(vpmc_ctx *c, int kind, const int16_t *hu, int nx, int ny, int nz,
                       const float spacing_mm[3], const float origin_mm[3], unsigned flags) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (kind != VPMC_GEOM_WATER && kind != VPMC_GEOM_HU) return fail(VPMC_E_ARG, "unknown geometry kind %d", kind);
    if (nx < 1 || ny < 1 || nz < 1) return fail(VPMC_E_ARG, "grid dimensions must be >= 1");
    const size_t nvox = (size_t)nx * ny * nz;
    if (nvox >= ((size_t)1 << 31)) return fail(VPMC_E_ARG, "grid has %zu voxels (max 2^31-1)", nvox);
    if (!spacing_mm || !origin_mm || !finite3(spacing_mm) || !finite3(origin_mm))
        return fail(VPMC_E_ARG, "spacing/origin missing or not finite");
    if (!(spacing_mm[0] > 0 && spacing_mm[1] > 0 && spacing_mm[2] > 0))
        return fail(VPMC_E_ARG, "spacing must be positive");
    if (kind == VPMC_GEOM_HU && !hu) return fail(VPMC_E_ARG, "HU geometry needs hu data");
    if (flags & ~VPMC_DEVICE_PTRS) return fail(VPMC_E_ARG, "unknown flags");
    GeomDev g{};
    g.kind = kind;
    g.nx = nx; g.ny = ny; g.nz = nz;
    for (int k = 0; k < 3; ++k) { g.sp[k] = spacing_mm[k]; g.lo[k] = origin_mm[k]; }
    if (c->device < 0) {
        // validation-only context: the grid's shape is kept for the checks of
        // later calls, the CT numbers are not read
        c->geom = g;
        c->nvox = nvox;
        c->has_geom = true;
        c->last_nscen = 0;
        return VPMC_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    if (kind == VPMC_GEOM_HU) {
        int rc = ensure(c, c->hu_buf, nvox * sizeof(int16_t), 0);
        if (rc) return rc;
        HIP_TRY(hipMemcpy(c->hu_buf.ptr, hu, nvox * sizeof(int16_t),
                          (flags & VPMC_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
        g.hu = (const int16_t *)c->hu_buf.ptr;
    }
    c->geom = g;
    c->nvox = nvox;
    c->has_geom = true;
    c->last_nscen = 0;
    return VPMC_OK;
}

int vpmc_set_aperture(vpmc_ctx *c, int field_id, const vpmc_beam *beam, const float *xy_mm, int n_vertices,
                      const vpmc_block *block, const vpmc_rs *rs) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (field_id < 0 || field_id >= VPMC_MAX_FIELDS)
        return fail(VPMC_E_ARG, "field_id %d outside [0, %d)", field_id, VPMC_MAX_FIELDS);
    int rc = validate_beam(beam);
    if (rc) return rc;
    if (n_vertices < 0) return fail(VPMC_E_POLYGON, "n_vertices < 0");
    if (!block && n_vertices != 0) return fail(VPMC_E_ARG, "polygon given without a block");
    if (block) {
        if (!(block->thickness_mm > 0 && isfinite(block->thickness_mm)) ||
            !(block->density_gcc > 0 && isfinite(block->density_gcc)) ||
            !(block->downstream_mm >= 0 && isfinite(block->downstream_mm)))
            return fail(VPMC_E_ARG, "block thickness/density must be > 0 and downstream >= 0");
        if ((rc = validate_polygon(xy_mm, n_vertices))) return rc;
    }
    double rs_t = 0.0;
    if (rs) {
        if (!(rs->wet_mm > 0 && isfinite(rs->wet_mm)) || !(rs->diameter_mm > 0 && isfinite(rs->diameter_mm)) ||
            !(rs->downstream_mm >= 0 && isfinite(rs->downstream_mm)))
            return fail(VPMC_E_ARG, "range shifter wet/diameter must be > 0 and downstream >= 0");
        if (block && rs->downstream_mm < block->downstream_mm + block->thickness_mm)
            return fail(VPMC_E_ARG, "range shifter overlaps or lies downstream of the block");
        rs_t = rs_thickness_mm(rs->wet_mm);
    }
    FieldState &f = c->fields[field_id];
    FieldDev d{};
    d.fs = 0.0f;    // non-divergent block, parallel beam (vpmc_set_divergence)
    d.fc0 = 1.0f;
    for (int k = 0; k < 3; ++k) {
        d.iso[k] = beam->iso_mm[k];
        d.ex[k] = beam->ex[k];
        d.ey[k] = beam->ey[k];
        d.ez[k] = beam->ez[k];
    }
    std::vector<float2> poly;
    if (block) {
        d.has_block = 1;
        d.nv = n_vertices;
        d.blk_zu = -(block->downstream_mm + block->thickness_mm);
        d.blk_zd = -block->downstream_mm;
        d.blk_rho = block->density_gcc;
        d.blk_t = block->thickness_mm;
        d.blk_tl = 0.0f;   // the caller's thickness is an FP32 value
        poly.resize(n_vertices);
        for (int i = 0; i < n_vertices; ++i) poly[i] = make_float2(xy_mm[2 * i], xy_mm[2 * i + 1]);
    }
    if (rs) {
        d.has_rs = 1;
        d.rs_zd = -rs->downstream_mm;
        d.rs_zu = (float)(-(rs->downstream_mm + rs_t));
        d.rs_r2 = 0.25f * rs->diameter_mm * rs->diameter_mm;
        d.rs_rho = (float)kMaterials[MAT_PMMA].density;
        d.rs_rhol = (float)(kMaterials[MAT_PMMA].density - (double)d.rs_rho);
        d.rs_t = (float)rs_t;
        d.rs_tl = (float)(rs_t - (double)d.rs_t);
    }
    Raster ras{};
    if (poly.size() >= 3) {
        ras = polygon_raster(poly, kSdfMargin);
        d.sdf_x0 = (float)ras.x0;
        d.sdf_y0 = (float)ras.y0;
        d.sdf_ih = (float)(1.0 / ras.h);
        // farthest point of a cell from its centre, plus room for FP32 rounding
        d.sdf_r = (float)(ras.h * 0.70710678118654752 + 1e-3);
        d.sdf_far = (float)(kSdfMargin - 1e-3);
        d.sdf_nx = ras.nx;
        d.sdf_ny = ras.ny;
    }
    CellLists lists;
    if (poly.size() >= 3) {
        lists = cell_lists(poly, ras, kListRadius);
        // a ray from p (within h sqrt(2) of its cell's reference point) meets
        // no unlisted edge within this path length in the BEV plane
        d.list_reach = (float)(kListRadius - (0.5 * ras.h * 1.4142135623730951 + 0.011) - 1e-3);
    }
    if (c->device >= 0 && !poly.empty()) {
        HIP_TRY(hipSetDevice(c->device));
        if ((rc = ensure(c, f.poly_buf, poly.size() * sizeof(float2), 0))) return rc;
        HIP_TRY(hipMemcpy(f.poly_buf.ptr, poly.data(), poly.size() * sizeof(float2), hipMemcpyHostToDevice));
        if (!ras.d.empty()) {
            if ((rc = ensure(c, f.sdf_buf, ras.d.size() * sizeof(float), 0))) return rc;
            HIP_TRY(hipMemcpy(f.sdf_buf.ptr, ras.d.data(), ras.d.size() * sizeof(float), hipMemcpyHostToDevice));
            if ((rc = ensure(c, f.cell_off_buf, lists.off.size() * sizeof(uint32_t), 0)) ||
                (rc = ensure(c, f.cell_ref_buf, lists.ref.size() * sizeof(float2), 0)) ||
                (rc = ensure(c, f.cell_edge_buf, std::max<size_t>(1, lists.edge.size()) * sizeof(uint16_t), 0)))
                return rc;
            HIP_TRY(hipMemcpy(f.cell_off_buf.ptr, lists.off.data(), lists.off.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(f.cell_ref_buf.ptr, lists.ref.data(), lists.ref.size() * sizeof(float2),
                              hipMemcpyHostToDevice));
            if (!lists.edge.empty())
                HIP_TRY(hipMemcpy(f.cell_edge_buf.ptr, lists.edge.data(), lists.edge.size() * sizeof(uint16_t),
                                  hipMemcpyHostToDevice));
        }
    }
    d.poly = (const float2 *)f.poly_buf.ptr;
    d.sdf = ras.d.empty() ? nullptr : (const float *)f.sdf_buf.ptr;
    d.cell_off = ras.d.empty() ? nullptr : (const uint32_t *)f.cell_off_buf.ptr;
    d.cell_ref = ras.d.empty() ? nullptr : (const float2 *)f.cell_ref_buf.ptr;
    d.cell_edge = ras.d.empty() ? nullptr : (const uint16_t *)f.cell_edge_buf.ptr;
    f.dev = d;
    f.poly = std::move(poly);
    f.set = true;
    return VPMC_OK;
}

int vpmc_set_divergence(vpmc_ctx *c, int field_id, float vsad_mm, float focus_mm) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (field_id < 0 || field_id >= VPMC_MAX_FIELDS)
        return fail(VPMC_E_ARG, "field_id %d outside [0, %d)", field_id, VPMC_MAX_FIELDS);
    if (!c->fields[field_id].set) return fail(VPMC_E_STATE, "field %d has no aperture/beam set", field_id);
    if (!(vsad_mm >= 0.0f && std::isfinite(vsad_mm)) || !(focus_mm >= 0.0f && std::isfinite(focus_mm)))
        return fail(VPMC_E_ARG, "vsad_mm and focus_mm must be finite and >= 0");
    FieldDev &d = c->fields[field_id].dev;
    double up = 0.0;   // the upstream-most face of the beam-line components
    if (d.has_block) up = std::max(up, -(double)d.blk_zu);
    if (d.has_rs) up = std::max(up, -(double)d.rs_zu);
    if (vsad_mm > 0.0f && (double)vsad_mm <= up)
        return fail(VPMC_E_ARG, "the virtual source must lie upstream of the range shifter and the block");
    if (focus_mm > 0.0f && !d.has_block) return fail(VPMC_E_ARG, "focus_mm needs an aperture block");
    if (focus_mm > 0.0f && (double)focus_mm <= -(double)d.blk_zu)
        return fail(VPMC_E_ARG, "the focus must lie upstream of the block's upstream face");
    d.vsad = vsad_mm;
    d.div = focus_mm > 0.0f ? 1 : 0;
    if (d.div) {
        const double fs = 1.0 / ((double)focus_mm + (double)d.blk_zd);   // 1 / (focus - downstream distance)
        d.fs = (float)fs;
        d.fc0 = (float)(((double)d.blk_zu + (double)focus_mm) * fs);
    } else {
        d.fs = 0.0f;
        d.fc0 = 1.0f;
    }
    return VPMC_OK;
}

}  // extern "C"

namespace {

// Checks shared by the dense and CSR runs of one field; T receives the
// weighted energy bound of the spots (for the fixed-point exponent).
int validate_run(const vpmc_ctx *c, int field_id, const vpmc_spot *spots, int n_spots, const vpmc_scenario *scen,
                 int n_scen, const vpmc_opts *o, double *T) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!o) return fail(VPMC_E_ARG, "opts is NULL");
    if (!c->has_geom) return fail(VPMC_E_STATE, "no geometry loaded");
    if (field_id < 0 || field_id >= VPMC_MAX_FIELDS) return fail(VPMC_E_ARG, "field_id out of range");
    if (!c->fields[field_id].set) return fail(VPMC_E_STATE, "field %d has no aperture/beam set", field_id);
    int rc;
    if ((rc = validate_spots(spots, n_spots, T))) return rc;
    if ((rc = validate_scen(scen, n_scen))) return rc;
    if (o->physics & ~VPMC_PHYS_ALL) return fail(VPMC_E_ARG, "unknown physics bits");
    if (o->n_batches < 0 || o->n_batches > 1024) return fail(VPMC_E_ARG, "n_batches outside [0, 1024]");
    return VPMC_OK;
}

// Device spot records (scale = w/N * 2^k) and, per batch b, the prefix of
// history counts per spot (history h of a spot belongs to batch h mod B).
void dense_spot_tables(const vpmc_spot *spots, int n_spots, int k, int B, std::vector<SpotDev> &sd,
                       std::vector<unsigned long long> &off) {
    sd.assign(std::max(1, n_spots), SpotDev{});
    off.assign((size_t)B * (n_spots + 1), 0ull);
    for (int i = 0; i < n_spots; ++i) {
        const vpmc_spot &s = spots[i];
        SpotDev &d = sd[i];
        d.x = s.x_mm; d.y = s.y_mm; d.e0 = s.energy_mev; d.sigma = s.sigma_mm; d.esig = s.energy_sigma_mev;
        d.emax = (float)std::min((double)s.energy_mev + 6.0 * s.energy_sigma_mev, E_HI);
        d.nh = s.n_histories;
        d.scale = s.n_histories ? (float)ldexp((double)s.weight / (double)s.n_histories, k) : 0.0f;
    }
    for (int b = 0; b < B; ++b) {
        unsigned long long *ob = off.data() + (size_t)b * (n_spots + 1);
        for (int i = 0; i < n_spots; ++i) {
            const unsigned long long nh = spots[i].n_histories;
            const unsigned long long nb = nh > (unsigned long long)b ? (nh - b + B - 1) / B : 0ull;
            ob[i + 1] = ob[i] + nb;
        }
    }
}

// Launch record of one batch of one scenario of a dense run.
LaunchDev dense_launch(const vpmc_opts *o, int field_id, const vpmc_scenario &sc, const SpotDev *spots,
                       const unsigned long long *ob, int n_spots, unsigned long long items, int b, int B,
                       unsigned long long *tally, unsigned long long *let_tally, unsigned long long *ledger,
                       unsigned long long *stats, const float *tables) {
    LaunchDev L{};
    L.spots = spots;
    L.item_off = ob;
    L.n_spots = n_spots;
    L.n_items = items;
    L.batch = b;
    L.n_batches = B;
    L.key0 = (uint32_t)(o->seed & 0xffffffffu);
    L.key1 = (uint32_t)(o->seed >> 32) ^ (uint32_t)field_id;
    L.physics = o->physics;
    for (int q = 0; q < 3; ++q) L.shift[q] = sc.shift_mm[q];
    L.range_scale = sc.range_scale;
    L.tally = tally;
    L.let_tally = let_tally;
    L.ledger = ledger;
    L.tables = tables;
    L.stats = stats;
    return L;
}

int dense_blocks(const vpmc_ctx *c, const vpmc_opts *o, unsigned long long items, int threads) {
    unsigned long long want = (items + threads - 1) / threads;
    const unsigned long long maxb = o->grid_blocks ? (unsigned long long)o->grid_blocks
                                    : (c->tuned_dense_blocks ? (unsigned long long)c->tuned_dense_blocks : 4096ull);
    return (int)std::min(want, maxb);
}

}  // namespace

extern "C" {

int vpmc_run_spots(vpmc_ctx *c, int field_id, const vpmc_spot *spots, int n_spots, const vpmc_scenario *scen,
                   int n_scen, const vpmc_opts *o, float *dose_gy, float *sigma_gy, double *ledger_mev,
                   int64_t *row_ptr) {
    double T = 0.0;
    int rc;
    if ((rc = validate_run(c, field_id, spots, n_spots, scen, n_scen, o, &T))) return rc;
    if (o->block_threads && o->block_threads != 256 && o->block_threads != 512 &&
        !(o->output == VPMC_OUT_CSR && (o->block_threads == 768 || o->block_threads == 1024)))
        return fail(VPMC_E_ARG, "block_threads must be 0, 256 or 512 (768 or 1024 also for CSR output)");
    if (o->grid_blocks < 0) return fail(VPMC_E_ARG, "grid_blocks < 0");
    if (o->hist_per_lane < 0 || o->hist_per_lane > 4096) return fail(VPMC_E_ARG, "hist_per_lane outside [0, 4096]");
    if (o->max_slots < 0) return fail(VPMC_E_ARG, "max_slots < 0");
    if (o->flags & ~(VPMC_DEVICE_PTRS | VPMC_GRAPH | VPMC_SURROGATE | VPMC_LET))
        return fail(VPMC_E_ARG, "unknown flags");
    if ((o->flags & VPMC_LET) && o->output != VPMC_OUT_DOSE)
        return fail(VPMC_E_ARG, "VPMC_LET is a dense-dose option");
    const bool use_sur = (o->flags & VPMC_SURROGATE) != 0;
    if (use_sur) {
        if (o->flags & VPMC_GRAPH) return fail(VPMC_E_ARG, "VPMC_SURROGATE cannot be combined with VPMC_GRAPH");
        if (!c->mlp_ready) return fail(VPMC_E_STATE, "VPMC_SURROGATE needs surrogate weights");
    }
    if (o->output == VPMC_OUT_CSR) {
        if (!row_ptr) return fail(VPMC_E_ARG, "CSR output needs row_ptr");
        if (sigma_gy) return fail(VPMC_E_ARG, "sigma_gy is not produced in CSR mode");
        int k = 0;
        if ((rc = pick_k(o, T, &k))) return rc;
        if (o->max_device_bytes && o->max_device_bytes / 2 < csr_slot_bytes(c->nvox))
            return fail(VPMC_E_OOM, "one influence-matrix row slot needs %zu bytes; max_device_bytes=%zu",
                        csr_slot_bytes(c->nvox), o->max_device_bytes);
        if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
        HIP_TRY(hipSetDevice(c->device));
        std::vector<BatchField> bf{{field_id, spots, n_spots}};
        return run_csr(c, bf, scen, n_scen, o, k, dose_gy, ledger_mev, row_ptr);
    } else if (o->output != VPMC_OUT_DOSE) {
        return fail(VPMC_E_ARG, "unknown output mode %d", o->output);
    }
    const int B = o->n_batches >= 2 ? o->n_batches : 1;
    if (sigma_gy && B < 2) return fail(VPMC_E_ARG, "sigma_gy needs n_batches >= 2");
    if (!dose_gy && !sigma_gy && !ledger_mev) return fail(VPMC_E_ARG, "no output requested");
    int k = 0;
    if ((rc = pick_k(o, T, &k))) return rc;
    {
        const size_t need = dense_bytes(c->nvox, n_scen, n_spots, B, (o->flags & VPMC_LET) != 0,
                                        (o->flags & VPMC_DEVICE_PTRS) != 0, dose_gy != nullptr, sigma_gy != nullptr);
        if (o->max_device_bytes && need > o->max_device_bytes)
            return fail(VPMC_E_OOM, "the dense run needs %zu bytes of device scratch; max_device_bytes=%zu", need,
                        o->max_device_bytes);
    }
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");

    const size_t nvox = c->nvox;
    const bool dev_out = (o->flags & VPMC_DEVICE_PTRS) != 0;
    const size_t cap = o->max_device_bytes;
    hipStream_t st = (hipStream_t)o->hip_stream;
    HIP_TRY(hipSetDevice(c->device));
    if ((rc = ensure(c, c->tallies, (size_t)n_scen * nvox * sizeof(long long), cap))) return rc;
    const bool want_let = (o->flags & VPMC_LET) != 0;
    if (want_let && (rc = ensure(c, c->let_tallies, (size_t)n_scen * nvox * sizeof(long long), cap))) return rc;
    c->last_let = false;
    if (B > 1) {
        if ((rc = ensure(c, c->qbatch, nvox * sizeof(unsigned long long), cap))) return rc;
        if ((rc = ensure(c, c->s2, nvox * sizeof(double), cap))) return rc;
    }
    if ((rc = ensure(c, c->ledger, (size_t)n_scen * NLEDGER * sizeof(unsigned long long), cap))) return rc;
    if ((rc = ensure(c, c->spots, std::max(1, n_spots) * sizeof(SpotDev), cap))) return rc;
    if ((rc = ensure(c, c->stats, 2 * sizeof(unsigned long long), cap))) return rc;
    if ((rc = ensure(c, c->offsets, (size_t)B * (n_spots + 1) * sizeof(unsigned long long), cap))) return rc;
    if (!dev_out) {
        if (dose_gy && (rc = ensure(c, c->stage_dose, nvox * sizeof(float), cap))) return rc;
        if (sigma_gy && (rc = ensure(c, c->stage_sigma, nvox * sizeof(float), cap))) return rc;
    }
    // surrogate queue: records of one batch launch (VPs beyond it cross the
    // block with the plain transport)
    const FieldDev &fd = c->fields[field_id].dev;
    const bool sur_on = use_sur && fd.has_block;
    unsigned long long sur_cap = 0;
    if (sur_on) {
        unsigned long long per_batch = 0;
        for (int i = 0; i < n_spots; ++i) per_batch += (spots[i].n_histories + B - 1) / B;
        sur_cap = std::max(1ull, std::min(per_batch, kSurMaxRecords));
        if ((rc = ensure(c, c->sur_rec, sur_cap * sizeof(DeferRec), cap))) return rc;
        if ((rc = ensure(c, c->sur_out, sur_cap * MLP_OUT * sizeof(float), cap))) return rc;
        if ((rc = ensure(c, c->sur_cnt, sizeof(unsigned long long), cap))) return rc;
    }

    // spots and per-batch work offsets
    std::vector<SpotDev> sd;
    std::vector<unsigned long long> off;
    dense_spot_tables(spots, n_spots, k, B, sd, off);
    HIP_TRY(hipMemcpyAsync(c->spots.ptr, sd.data(), sd.size() * sizeof(SpotDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->offsets.ptr, off.data(), off.size() * sizeof(unsigned long long),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(c->ledger.ptr, 0, (size_t)n_scen * NLEDGER * sizeof(unsigned long long), st));
    HIP_TRY(hipMemsetAsync(c->stats.ptr, 0, 2 * sizeof(unsigned long long), st));
    const size_t n_launch_max = (size_t)n_scen * B;
    while (c->events.size() < 2 * n_launch_max + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->events.push_back(e);
    }
    size_t n_launch = 0;
    HIP_TRY(hipEventRecord(c->events[0], st));

    const int threads = o->block_threads ? o->block_threads : (c->tuned_dense_threads ? c->tuned_dense_threads : 256);
    const double mev_scale = ldexp(MEV_TO_J, -k);
    unsigned long long deferred = 0;
    for (int sc = 0; sc < n_scen; ++sc) {
        long long *tally = (long long *)c->tallies.ptr + (size_t)sc * nvox;
        HIP_TRY(hipMemsetAsync(tally, 0, nvox * sizeof(long long), st));
        unsigned long long *let_tally =
            want_let ? (unsigned long long *)c->let_tallies.ptr + (size_t)sc * nvox : nullptr;
        if (let_tally) HIP_TRY(hipMemsetAsync(let_tally, 0, nvox * sizeof(long long), st));
        if (B > 1) HIP_TRY(hipMemsetAsync(c->s2.ptr, 0, nvox * sizeof(double), st));
        if (B > 1) HIP_TRY(hipMemsetAsync(c->qbatch.ptr, 0, nvox * sizeof(unsigned long long), st));
        for (int b = 0; b < B; ++b) {
            const unsigned long long *ob = (const unsigned long long *)c->offsets.ptr + (size_t)b * (n_spots + 1);
            const unsigned long long items = off[(size_t)b * (n_spots + 1) + n_spots];
            if (items == 0) continue;
            // every batch adds to the scenario's LET numerator
            LaunchDev L = dense_launch(o, field_id, scen[sc], (const SpotDev *)c->spots.ptr, ob, n_spots, items, b, B,
                                       B > 1 ? (unsigned long long *)c->qbatch.ptr : (unsigned long long *)tally,
                                       let_tally, (unsigned long long *)c->ledger.ptr + (size_t)sc * NLEDGER,
                                       (unsigned long long *)c->stats.ptr, c->d_tables);
            const int blocks = dense_blocks(c, o, items, threads);
            if (sur_on) {
                HIP_TRY(hipMemsetAsync(c->sur_cnt.ptr, 0, sizeof(unsigned long long), st));
                L.sur.enabled = 1;
                L.sur.d_fallback = c->sur_dfb;
                L.sur.count = (unsigned long long *)c->sur_cnt.ptr;
                L.sur.capacity = sur_cap;
                L.sur.rec = (DeferRec *)c->sur_rec.ptr;
            }
            HIP_TRY(hipEventRecord(c->events[2 + 2 * n_launch], st));
            HIP_TRY(launch_transport(c->geom, fd, L, blocks, threads, st));
            if (sur_on) {
                // the queue's length decides the network's launch shapes
                unsigned long long cnt = 0;
                HIP_TRY(hipMemcpyAsync(&cnt, c->sur_cnt.ptr, sizeof cnt, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                const unsigned long long nq = std::min(cnt, sur_cap);
                deferred += nq;
                const DeferRec *rec = (const DeferRec *)c->sur_rec.ptr;
                float *sout = (float *)c->sur_out.ptr;
                if (nq) {
                    HIP_TRY(mlp_infer(nullptr, rec, (int)nq, (const __bf16 *)c->mlp_wb.ptr, (const float *)c->mlp_w.ptr,
                                      sout, st));
                    HIP_TRY(launch_sur_resume(c->geom, fd, L, rec, sout, nq, c->sur_plo, c->sur_phi, st));
                }
            }
            HIP_TRY(hipEventRecord(c->events[3 + 2 * n_launch], st));
            ++n_launch;
            if (B > 1)
                HIP_TRY(launch_fold_batch((unsigned long long *)c->qbatch.ptr, tally, (double *)c->s2.ptr, nvox, st));
        }
        float *dd = dose_gy ? (dev_out ? dose_gy + (size_t)sc * nvox : (float *)c->stage_dose.ptr) : nullptr;
        float *ss = sigma_gy ? (dev_out ? sigma_gy + (size_t)sc * nvox : (float *)c->stage_sigma.ptr) : nullptr;
        if (dd || ss)
            HIP_TRY(launch_dose(tally, B > 1 ? (const double *)c->s2.ptr : nullptr, B, c->geom, mev_scale, dd, ss,
                                nvox, st));
        if (!dev_out) {
            if (dd) HIP_TRY(hipMemcpyAsync(dose_gy + (size_t)sc * nvox, dd, nvox * sizeof(float), hipMemcpyDeviceToHost, st));
            if (ss) HIP_TRY(hipMemcpyAsync(sigma_gy + (size_t)sc * nvox, ss, nvox * sizeof(float), hipMemcpyDeviceToHost, st));
        }
    }
    std::vector<long long> led((size_t)n_scen * NLEDGER);
    unsigned long long stv[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(led.data(), c->ledger.ptr, led.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(stv, c->stats.ptr, sizeof stv, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(c->events[1], st));
    HIP_TRY(hipStreamSynchronize(st));
    vpmc_stats S{};
    float ms = 0.0f;
    for (size_t i = 0; i < n_launch; ++i) {
        HIP_TRY(hipEventElapsedTime(&ms, c->events[2 + 2 * i], c->events[3 + 2 * i]));
        S.transport_ms += ms;
    }
    HIP_TRY(hipEventElapsedTime(&ms, c->events[0], c->events[1]));
    S.total_ms = ms;
    S.steps = stv[0];
    S.histories = stv[1];
    S.launches = n_launch;
    S.deferred = deferred;
    c->last_stats = S;
    if (ledger_mev)
        for (size_t i = 0; i < led.size(); ++i) ledger_mev[i] = ldexp((double)led[i], -k);
    c->last_k = k;
    c->last_let = want_let;
    c->last_nscen = n_scen;
    return VPMC_OK;
}

int vpmc_run_spots_noalloc(vpmc_ctx *c, int field_id, const vpmc_spot *spots, int n_spots,
                           const vpmc_scenario *scen, int n_scen, const vpmc_opts *o, float *dose_gy,
                           float *sigma_gy, double *ledger_mev) {
    double T = 0.0;
    int rc;
    if ((rc = validate_run(c, field_id, spots, n_spots, scen, n_scen, o, &T))) return rc;
    if (o->output != VPMC_OUT_DOSE) return fail(VPMC_E_ARG, "the allocation-free run writes dense dose only");
    if (o->flags != VPMC_DEVICE_PTRS)
        return fail(VPMC_E_ARG, "the allocation-free run takes flags == VPMC_DEVICE_PTRS (device dose/sigma)");
    if (o->block_threads && o->block_threads != 256 && o->block_threads != 512)
        return fail(VPMC_E_ARG, "block_threads must be 0, 256 or 512");
    if (o->grid_blocks < 0) return fail(VPMC_E_ARG, "grid_blocks < 0");
    const int B = o->n_batches >= 2 ? o->n_batches : 1;
    if (sigma_gy && B < 2) return fail(VPMC_E_ARG, "sigma_gy needs n_batches >= 2");
    if (!dose_gy && !sigma_gy && !ledger_mev) return fail(VPMC_E_ARG, "no output requested");
    int k = 0;
    if ((rc = pick_k(o, T, &k))) return rc;
    // scratch layout (256-byte aligned pieces): ledger [n_scen][6], stats [2],
    // spots, batch offsets [B][n_spots + 1], tally [nvox], and with batches
    // the batch tally [nvox] and the FP64 sum of squares [nvox]
    const size_t nvox = c->nvox;
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_led = 0;
    const size_t o_stats = o_led + a256((size_t)n_scen * NLEDGER * 8);
    const size_t o_spots = o_stats + a256(2 * 8);
    const size_t o_off = o_spots + a256((size_t)std::max(1, n_spots) * sizeof(SpotDev));
    const size_t o_tally = o_off + a256((size_t)B * (n_spots + 1) * 8);
    const size_t o_qb = o_tally + a256(nvox * 8);
    const size_t o_s2 = o_qb + (B > 1 ? a256(nvox * 8) : 0);
    const size_t need = o_s2 + (B > 1 ? a256(nvox * 8) : 0);
    if (need > kScratchBytes)
        return fail(VPMC_E_OOM, "the run needs %zu bytes of scratch; the static scratch holds %zu "
                    "(8 B per voxel, 24 B with batches, plus spots and ledgers)", need, kScratchBytes);
    if (c->device < 0 || !c->scratch) return fail(VPMC_E_STATE, "validation-only context has no device");

    hipStream_t st = (hipStream_t)o->hip_stream;
    HIP_TRY(hipSetDevice(c->device));
    unsigned char *base = (unsigned char *)c->scratch;
    unsigned long long *led_d = (unsigned long long *)(base + o_led);
    unsigned long long *stats_d = (unsigned long long *)(base + o_stats);
    SpotDev *spots_d = (SpotDev *)(base + o_spots);
    unsigned long long *off_d = (unsigned long long *)(base + o_off);
    long long *tally = (long long *)(base + o_tally);
    unsigned long long *qb = B > 1 ? (unsigned long long *)(base + o_qb) : nullptr;
    double *s2 = B > 1 ? (double *)(base + o_s2) : nullptr;

    std::vector<SpotDev> sd;
    std::vector<unsigned long long> off;
    dense_spot_tables(spots, n_spots, k, B, sd, off);
    HIP_TRY(hipMemcpyAsync(spots_d, sd.data(), sd.size() * sizeof(SpotDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(off_d, off.data(), off.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    // the scratch keeps the previous call's contents: clear with fill kernels
    HIP_TRY(launch_fill_u64(led_d, (size_t)n_scen * NLEDGER, 0ull, st));
    HIP_TRY(launch_fill_u64(stats_d, 2, 0ull, st));

    const FieldDev &fd = c->fields[field_id].dev;
    const int threads = o->block_threads ? o->block_threads : (c->tuned_dense_threads ? c->tuned_dense_threads : 256);
    const double mev_scale = ldexp(MEV_TO_J, -k);
    for (int sc = 0; sc < n_scen; ++sc) {
        HIP_TRY(launch_fill_u64((unsigned long long *)tally, nvox, 0ull, st));
        if (B > 1) {
            HIP_TRY(launch_fill_u64(qb, nvox, 0ull, st));
            HIP_TRY(launch_fill_u64((unsigned long long *)s2, nvox, 0ull, st));   // all-zero bits = 0.0
        }
        for (int b = 0; b < B; ++b) {
            const unsigned long long items = off[(size_t)b * (n_spots + 1) + n_spots];
            if (items == 0) continue;
            LaunchDev L = dense_launch(o, field_id, scen[sc], spots_d, off_d + (size_t)b * (n_spots + 1), n_spots,
                                       items, b, B, B > 1 ? qb : (unsigned long long *)tally, nullptr,
                                       led_d + (size_t)sc * NLEDGER, stats_d, c->d_tables);
            HIP_TRY(launch_transport(c->geom, fd, L, dense_blocks(c, o, items, threads), threads, st));
            if (B > 1) HIP_TRY(launch_fold_batch(qb, tally, s2, nvox, st));
        }
        float *dd = dose_gy ? dose_gy + (size_t)sc * nvox : nullptr;
        float *ss = sigma_gy ? sigma_gy + (size_t)sc * nvox : nullptr;
        if (dd || ss) HIP_TRY(launch_dose(tally, s2, B, c->geom, mev_scale, dd, ss, nvox, st));
    }
    if (ledger_mev) {
        std::vector<long long> led((size_t)n_scen * NLEDGER);
        HIP_TRY(hipMemcpyAsync(led.data(), led_d, led.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (size_t i = 0; i < led.size(); ++i) ledger_mev[i] = ldexp((double)led[i], -k);
    }
    return VPMC_OK;
}

int vpmc_last_stats(const vpmc_ctx *c, vpmc_stats *out) {
    if (!c || !out) return fail(VPMC_E_ARG, "ctx/out is NULL");
    *out = c->last_stats;
    return VPMC_OK;
}

int vpmc_run_batched(vpmc_ctx *c, const int *field_ids, const vpmc_spot *const *spots, const int *n_spots,
                     int n_fields, const vpmc_scenario *scen, int n_scen, const vpmc_opts *o, float *dose_gy,
                     double *ledger_mev, int64_t *row_ptr) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!o) return fail(VPMC_E_ARG, "opts is NULL");
    if (!c->has_geom) return fail(VPMC_E_STATE, "no geometry loaded");
    if (n_fields < 1 || n_fields > VPMC_MAX_FIELDS || !field_ids || !spots || !n_spots)
        return fail(VPMC_E_ARG, "need 1..%d fields with their spot arrays", VPMC_MAX_FIELDS);
    if (!row_ptr) return fail(VPMC_E_ARG, "row_ptr is NULL");
    int rc;
    double T = 0.0;
    std::vector<BatchField> bf;
    for (int f = 0; f < n_fields; ++f) {
        const int id = field_ids[f];
        if (id < 0 || id >= VPMC_MAX_FIELDS) return fail(VPMC_E_ARG, "field id %d out of range", id);
        if (!c->fields[id].set) return fail(VPMC_E_STATE, "field %d has no aperture/beam set", id);
        for (int g = 0; g < f; ++g)
            if (field_ids[g] == id) return fail(VPMC_E_ARG, "field id %d repeated", id);
        double Tf = 0.0;
        if ((rc = validate_spots(spots[f], n_spots[f], &Tf))) return rc;
        T += Tf;
        bf.push_back({id, spots[f], n_spots[f]});
    }
    if ((rc = validate_scen(scen, n_scen))) return rc;
    if (o->physics & ~VPMC_PHYS_ALL) return fail(VPMC_E_ARG, "unknown physics bits");
    if (o->flags & ~(VPMC_DEVICE_PTRS | VPMC_GRAPH | VPMC_SURROGATE)) return fail(VPMC_E_ARG, "unknown flags");
    if ((o->flags & VPMC_SURROGATE) && (o->flags & VPMC_GRAPH))
        return fail(VPMC_E_ARG, "VPMC_SURROGATE cannot be combined with VPMC_GRAPH");
    if ((o->flags & VPMC_SURROGATE) && !c->mlp_ready) return fail(VPMC_E_STATE, "VPMC_SURROGATE needs surrogate weights");
    if (o->hist_per_lane < 0 || o->hist_per_lane > 4096) return fail(VPMC_E_ARG, "hist_per_lane outside [0, 4096]");
    if (o->max_slots < 0 || o->grid_blocks < 0) return fail(VPMC_E_ARG, "negative tuning value");
    if (o->block_threads && o->block_threads != 256 && o->block_threads != 512 &&
        o->block_threads != 768 && o->block_threads != 1024)
        return fail(VPMC_E_ARG, "block_threads must be 0, 256, 512, 768 or 1024");
    int k = 0;
    if ((rc = pick_k(o, T, &k))) return rc;
    if (o->max_device_bytes && o->max_device_bytes / 2 < csr_slot_bytes(c->nvox))
        return fail(VPMC_E_OOM, "one influence-matrix row slot needs %zu bytes; max_device_bytes=%zu",
                    csr_slot_bytes(c->nvox), o->max_device_bytes);
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    return run_csr(c, bf, scen, n_scen, o, k, dose_gy, ledger_mev, row_ptr);
}

int vpmc_autotune(vpmc_ctx *c, int field_id, const vpmc_spot *spots, int n_spots, const vpmc_scenario *scen,
                  const vpmc_opts *base, uint64_t sample_histories, vpmc_opts *best) {
    if (!c || !base || !best || !spots || n_spots < 1 || !scen) return fail(VPMC_E_ARG, "bad autotune arguments");
    if (sample_histories < 64) return fail(VPMC_E_ARG, "sample_histories must be >= 64");
    if (!c->has_geom) return fail(VPMC_E_STATE, "no geometry loaded");
    if (field_id < 0 || field_id >= VPMC_MAX_FIELDS || !c->fields[field_id].set)
        return fail(VPMC_E_STATE, "field %d not set", field_id);
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    double tot = 0.0;
    for (int i = 0; i < n_spots; ++i) tot += spots[i].n_histories;
    if (tot <= 0) return fail(VPMC_E_ARG, "spots hold no histories");
    // the sample keeps the real per-spot history counts (the chunking and
    // the tally footprint of a row depend on them) and takes every s-th spot
    const int stride = std::max(1, (int)std::floor(tot / (double)sample_histories));
    std::vector<vpmc_spot> sub;
    for (int i = 0; i < n_spots; i += stride) sub.push_back(spots[i]);
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) cus = prop.multiProcessorCount;
    const bool csr = base->output == VPMC_OUT_CSR;
    struct Cand { int hpl, blocks, threads; };
    std::vector<Cand> cand;
    if (csr) {
        // one resident set of workgroups: 16 waves per CU (12 in double-float mode)
        const int waves_cu = base->physics == 0 ? 12 : 16;
        for (int h : {1, 2, 3, 4, 6, 8})
            for (int t : {1024, 512}) {
                const int tt = queue_threads(base->physics, t);
                cand.push_back({h, std::max(1, cus * waves_cu / (tt / 64)), tt});
            }
    } else {
        for (int m : {4, 8, 16, 32})
            for (int t : {256, 512}) cand.push_back({0, m * cus * 256 / t, t});
    }
    const int n_sub = (int)sub.size();
    const size_t R = (size_t)n_sub;
    std::vector<int64_t> rp(R + 1);
    std::vector<double> led(NLEDGER);
    // every candidate is timed twice (two passes over the list, the faster
    // time counts): shapes a few per cent apart are told apart reliably
    std::vector<double> cand_t(cand.size(), 1e300);
    for (size_t ci = 0; ci <= 2 * cand.size(); ++ci) {
        // the first run warms up the buffers and is not scored
        const size_t cix = ci == 0 ? 0 : (ci - 1) % cand.size();
        const Cand cd = cand[cix];
        vpmc_opts o = *base;
        o.flags &= ~(unsigned)VPMC_DEVICE_PTRS;
        o.flags &= ~(unsigned)VPMC_GRAPH;
        o.n_batches = 0;
        o.hist_per_lane = cd.hpl;
        o.grid_blocks = cd.blocks;
        o.block_threads = cd.threads;
        const int rc = csr ? vpmc_run_spots(c, field_id, sub.data(), n_sub, scen, 1, &o, nullptr, nullptr,
                                            led.data(), rp.data())
                           : vpmc_run_spots(c, field_id, sub.data(), n_sub, scen, 1, &o, nullptr, nullptr,
                                            led.data(), nullptr);
        if (rc) return rc;
        if (ci == 0) continue;
        const double t = c->last_stats.transport_ms / std::max<double>(1.0, (double)c->last_stats.histories);
        cand_t[cix] = std::min(cand_t[cix], t);
    }
    size_t bi = 0;
    for (size_t i = 1; i < cand.size(); ++i)
        if (cand_t[i] < cand_t[bi]) bi = i;
    vpmc_opts pick = *base;
    pick.hist_per_lane = cand[bi].hpl;
    pick.grid_blocks = cand[bi].blocks;
    pick.block_threads = cand[bi].threads;
    if (csr) {
        c->tuned_csr_hpl = pick.hist_per_lane;
        c->tuned_csr_hpl_field[field_id] = pick.hist_per_lane;
        c->tuned_csr_blocks = pick.grid_blocks;
        c->tuned_csr_threads = pick.block_threads;
    } else {
        c->tuned_dense_blocks = pick.grid_blocks;
        c->tuned_dense_threads = pick.block_threads;
    }
    *best = pick;
    return VPMC_OK;
}

int vpmc_copy_csr(vpmc_ctx *c, int32_t *col, float *val, int64_t *q_raw) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!c->csr_valid) return fail(VPMC_E_STATE, "no CSR run to copy");
    if (!col && !val && !q_raw) return fail(VPMC_E_ARG, "no output");
    const size_t n = c->csr_total;
    if (n == 0) return VPMC_OK;
    const bool dev = (c->csr_flags & VPMC_DEVICE_PTRS) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIP_TRY(hipSetDevice(c->device));
    if (col) HIP_TRY(hipMemcpy(col, c->csr_col.ptr, n * 4, kind));
    if (q_raw) HIP_TRY(hipMemcpy(q_raw, c->csr_q.ptr, n * 8, kind));
    if (val) {
        float *dst = val;
        if (!dev) {
            int rc = ensure(c, c->stage_dose, n * sizeof(float), 0);
            if (rc) return rc;
            dst = (float *)c->stage_dose.ptr;
        }
        HIP_TRY(launch_csr_values((const int32_t *)c->csr_col.ptr, (const long long *)c->csr_q.ptr, n, c->geom,
                                  ldexp(MEV_TO_J, -c->last_k), dst, nullptr));
        HIP_TRY(hipDeviceSynchronize());
        if (!dev) HIP_TRY(hipMemcpy(val, dst, n * 4, hipMemcpyDeviceToHost));
    }
    return VPMC_OK;
}

int vpmc_last_let(vpmc_ctx *c, int scen_index, int64_t *ql_out, int *shift_out, unsigned flags) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!ql_out && !shift_out) return fail(VPMC_E_ARG, "no output");
    if (flags & ~VPMC_DEVICE_PTRS) return fail(VPMC_E_ARG, "unknown flags");
    if (c->last_nscen == 0 || !c->last_let) return fail(VPMC_E_STATE, "the last dense run did not tally LET");
    if (scen_index < 0 || scen_index >= c->last_nscen) return fail(VPMC_E_ARG, "scenario index out of range");
    if (shift_out) *shift_out = kLetShift;
    if (ql_out) {
        HIP_TRY(hipSetDevice(c->device));
        HIP_TRY(hipMemcpy(ql_out, (long long *)c->let_tallies.ptr + (size_t)scen_index * c->nvox,
                          c->nvox * sizeof(long long),
                          (flags & VPMC_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
    return VPMC_OK;
}

int vpmc_last_tally(vpmc_ctx *c, int scen_index, int64_t *q_out, int *k_out, unsigned flags) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!q_out && !k_out) return fail(VPMC_E_ARG, "no output");
    if (!q_out && scen_index == -1 && (c->last_nscen || c->csr_valid)) {   // exponent only
        *k_out = c->last_k;
        return VPMC_OK;
    }
    if (c->last_nscen == 0) return fail(VPMC_E_STATE, "no dense run to copy");
    if (scen_index < 0 || scen_index >= c->last_nscen) return fail(VPMC_E_ARG, "scenario index out of range");
    if (k_out) *k_out = c->last_k;
    if (q_out) {
        HIP_TRY(hipSetDevice(c->device));
        HIP_TRY(hipMemcpy(q_out, (long long *)c->tallies.ptr + (size_t)scen_index * c->nvox,
                          c->nvox * sizeof(long long),
                          (flags & VPMC_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
    return VPMC_OK;
}

}  // extern "C"

int vpmc_optimize(vpmc_ctx *c, const int64_t *row_ptr, const int32_t *col, const float *val, int n_scen,
                  int n_spots, int nvox, const uint8_t *roi, const vpmc_opt_params *p, double *x, double *obj_hist,
                  double *step_L, float *dose_gy) {
    if (!c || !p) return fail(VPMC_E_ARG, "ctx and params are required");
    if (!row_ptr || !roi || !x) return fail(VPMC_E_ARG, "row_ptr, roi and x are required");
    if (n_scen < 1 || n_spots < 1 || nvox < 1) return fail(VPMC_E_ARG, "n_scen, n_spots and nvox must be >= 1");
    if (p->flags & ~(VPMC_DEVICE_PTRS | VPMC_OPT_REUSE)) return fail(VPMC_E_ARG, "unknown flags");
    if (!std::isfinite(p->d_presc) || !std::isfinite(p->d_max) || !std::isfinite(p->w_target) ||
        !std::isfinite(p->w_oar) || p->w_target < 0.0 || p->w_oar < 0.0)
        return fail(VPMC_E_ARG, "d_presc and d_max must be finite, the weights finite and >= 0");
    if (p->iters < 0 || p->iters > 100000) return fail(VPMC_E_ARG, "iters outside [0, 100000]");
    if (p->n_power < 1 || p->n_power > 1000) return fail(VPMC_E_ARG, "n_power outside [1, 1000]");
    const int stride = p->row_stride ? p->row_stride : n_spots;
    if (p->row_offset < 0 || stride < 1 || (long long)p->row_offset + n_spots > stride)
        return fail(VPMC_E_ARG, "need 0 <= row_offset and row_offset + n_spots <= row_stride");
    const long long n_layout = (long long)n_scen * stride;
    const long long n_rows = (long long)n_scen * n_spots;
    if (n_layout >= (1ll << 31) || n_rows * 64 >= (1ll << 31)) return fail(VPMC_E_ARG, "too many rows");
    if (n_spots > (1 << 20)) return fail(VPMC_E_ARG, "n_spots above 2^20");
    const bool dev = (p->flags & VPMC_DEVICE_PTRS) != 0;
    const bool reuse = (p->flags & VPMC_OPT_REUSE) != 0;
    // host copy of the row pointer for validation (host arrays are checked
    // here, before the device is touched)
    std::vector<int64_t> rp((size_t)n_layout + 1);
    if (!dev) {
        memcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t));
    } else {
        if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
        HIP_TRY(hipSetDevice(c->device));
        HIP_TRY(hipMemcpy(rp.data(), row_ptr, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    }
    if (rp[0] < 0) return fail(VPMC_E_ARG, "row_ptr[0] < 0");
    for (size_t r = 0; r + 1 < rp.size(); ++r)
        if (rp[r + 1] < rp[r]) return fail(VPMC_E_ARG, "row_ptr decreases at row %zu", r);
    const long long nnz = rp.back();
    if (nnz > 0 && (!col || !val)) return fail(VPMC_E_ARG, "col and val are required");
    if (!dev) {
        for (long long i = 0; i < nnz; ++i) {
            if ((unsigned)col[i] >= (unsigned)nvox) return fail(VPMC_E_ARG, "column %lld out of range", i);
            if (!std::isfinite(val[i])) return fail(VPMC_E_ARG, "value %lld not finite", i);
        }
    }
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)p->hip_stream;
    const int nchunks = (int)((nvox + (long long)kOptChunk - 1) / kOptChunk);
    const size_t nlist = (size_t)n_scen * nchunks;
    const int dims[5] = {n_scen, n_spots, stride, p->row_offset, nvox};
    const bool same = c->opt_valid && memcmp(dims, c->opt_dims, sizeof dims) == 0 && c->opt_rp_host == rp &&
                      (!dev || (c->opt_col_src == col && c->opt_val_src == val));
    // structure masks on the host (chunks that hold structure voxels; reuse check)
    std::vector<uint8_t> roi_h((size_t)nvox);
    HIP_TRY(hipMemcpy(roi_h.data(), roi, (size_t)nvox, dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    if (reuse && (!same || roi_h != c->opt_roi_host))
        return fail(VPMC_E_STATE, "VPMC_OPT_REUSE without a matching index (rows, columns or structures changed)");
    int rc;
    // CSR on the device: the library's own row pointer (validated), caller's or copied arrays
    if ((rc = ensure(c, c->opt_rp, rp.size() * 8, 0))) return rc;
    const int32_t *d_col = col;
    const float *d_val = val;
    const uint8_t *d_roi = roi;
    if (!dev) {
        if ((rc = ensure(c, c->opt_col, (size_t)std::max(nnz, 1ll) * 4, 0))) return rc;
        if ((rc = ensure(c, c->opt_val, (size_t)std::max(nnz, 1ll) * 4, 0))) return rc;
        if ((rc = ensure(c, c->opt_roi, (size_t)nvox, 0))) return rc;
        if (!reuse) {
            HIP_TRY(hipMemcpyAsync(c->opt_col.ptr, col, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(c->opt_val.ptr, val, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
        }
        HIP_TRY(hipMemcpyAsync(c->opt_roi.ptr, roi, (size_t)nvox, hipMemcpyHostToDevice, st));
        d_col = (const int32_t *)c->opt_col.ptr;
        d_val = (const float *)c->opt_val.ptr;
        d_roi = (const uint8_t *)c->opt_roi.ptr;
    }
    if ((rc = ensure(c, c->opt_amax, (size_t)n_rows * 4, 0))) return rc;
    if ((rc = ensure(c, c->opt_cnt, nlist * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_rcnt, (size_t)n_rows * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_crp, ((size_t)n_rows + 1) * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_poff, ((size_t)n_rows + 1) * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_resid, (size_t)n_scen * nvox * 4, 0))) return rc;
    if ((rc = ensure(c, c->opt_fpart, nlist * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_vec, (size_t)n_spots * 4 * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_scal, ((size_t)2 * n_scen + 2) * 8, 0))) return rc;
    if ((rc = ensure(c, c->opt_err, 4, 0))) return rc;
    if ((rc = ensure(c, c->opt_hist, ((size_t)p->iters + 1) * 8, 0))) return rc;
    // the whole layout (validation, bound of every row, dose output) ...
    OptDev F{};
    F.row_ptr = (const long long *)c->opt_rp.ptr;
    F.col = d_col;
    F.val = d_val;
    F.roi = d_roi;
    F.n_scen = n_scen;
    F.n_spots = n_spots;
    F.row_stride = stride;
    F.row_offset = p->row_offset;
    F.nvox = nvox;
    F.nchunks = nchunks;
    F.d_presc = p->d_presc;
    F.w_target = p->w_target;
    F.d_max = p->d_max;
    F.w_oar = p->w_oar;
    F.amax = (float *)c->opt_amax.ptr;
    F.resid = (float *)c->opt_resid.ptr;
    F.fpart = (double *)c->opt_fpart.ptr;
    double *vec = (double *)c->opt_vec.ptr;
    F.x = vec;
    F.y = vec + n_spots;
    F.z = vec + 2 * (size_t)n_spots;
    F.gvec = vec + 3 * (size_t)n_spots;
    F.scale = (double *)c->opt_scal.ptr;
    F.scal = F.scale + 2 * (size_t)n_scen;
    F.piece_off = (const long long *)c->opt_poff.ptr;
    // ... and its rows restricted to the structure voxels (the iterations)
    OptDev O = F;
    O.row_ptr = (const long long *)c->opt_crp.ptr;
    O.row_stride = n_spots;
    O.row_offset = 0;
    auto set_buckets = [](OptDev &D, const vpmc_ctx::OptBuckets &B) {
        D.boff = (const unsigned long long *)B.off.ptr;
        D.bkey = (const uint32_t *)B.key.ptr;
        D.bval = (const float *)B.val.ptr;
        D.work = (const uint32_t *)B.work.ptr;
        D.n_work = B.n_work;
    };
    // bucketed copy of the rows of D: lists (scenario, chunk) over the chunks
    // with keep[chunk] (all when keep is empty), heaviest first in the work list
    auto build_buckets = [&](OptDev &D, vpmc_ctx::OptBuckets &B, const std::vector<char> &keep,
                             long long expect) -> int {
        B.valid = false;
        int rc2;
        if ((rc2 = ensure(c, B.off, (nlist + 1) * 8, 0))) return rc2;
        if ((rc2 = ensure(c, B.work, std::max<size_t>(nlist, 1) * 4, 0))) return rc2;
        HIP_TRY(hipMemsetAsync(c->opt_cnt.ptr, 0, nlist * 8, st));
        HIP_TRY(hipMemsetAsync(c->opt_err.ptr, 0, 4, st));
        HIP_TRY(opt_build_count(D, (unsigned long long *)c->opt_cnt.ptr, (unsigned *)c->opt_err.ptr, st));
        HIP_TRY(opt_build_scan((unsigned long long *)c->opt_cnt.ptr, (unsigned long long *)B.off.ptr, nlist, st));
        std::vector<unsigned long long> boff(nlist + 1);
        HIP_TRY(hipMemcpyAsync(boff.data(), B.off.ptr, (nlist + 1) * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if ((long long)boff[nlist] != expect)
            return fail(VPMC_E_DEVICE, "entry count %llu of the chunk lists differs from the rows' %lld", boff[nlist],
                        expect);
        std::vector<uint32_t> work;
        for (size_t k = 0; k < nlist; ++k)
            if (keep.empty() || keep[k % (size_t)nchunks]) work.push_back((uint32_t)k);
        std::stable_sort(work.begin(), work.end(), [&](uint32_t a, uint32_t b) {
            return boff[a + 1] - boff[a] > boff[b + 1] - boff[b];
        });
        if (!work.empty())
            HIP_TRY(hipMemcpyAsync(B.work.ptr, work.data(), work.size() * 4, hipMemcpyHostToDevice, st));
        if ((rc2 = ensure(c, B.key, (size_t)std::max(expect, 1ll) * 4, 0))) return rc2;
        if ((rc2 = ensure(c, B.val, (size_t)std::max(expect, 1ll) * 4, 0))) return rc2;
        HIP_TRY(opt_build_emit(D, (const unsigned long long *)B.off.ptr, (unsigned long long *)c->opt_cnt.ptr,
                               (uint32_t *)B.key.ptr, (float *)B.val.ptr, st));
        HIP_TRY(hipStreamSynchronize(st));   // the host vectors outlive the copies
        B.n_work = (long long)work.size();
        B.valid = true;
        return VPMC_OK;
    };
    if (!reuse) {
        c->opt_valid = false;
        c->opt_bfull.valid = false;
        HIP_TRY(hipMemcpyAsync(c->opt_rp.ptr, rp.data(), rp.size() * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(c->opt_err.ptr, 0, 4, st));
        HIP_TRY(opt_roi_count(F, (unsigned long long *)c->opt_rcnt.ptr, (unsigned *)c->opt_err.ptr, st));
        std::vector<unsigned long long> rcnt((size_t)n_rows);
        unsigned err = 0;
        HIP_TRY(hipMemcpyAsync(rcnt.data(), c->opt_rcnt.ptr, (size_t)n_rows * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&err, c->opt_err.ptr, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (err & 1u) return fail(VPMC_E_ARG, "a column index is outside [0, nvox)");
        if (err & 2u) return fail(VPMC_E_ARG, "a value is not finite");
        // structure-restricted CSR and its gradient pieces of at most kOptPiece entries
        std::vector<long long> crp((size_t)n_rows + 1), poff((size_t)n_rows + 1);
        std::vector<OptPiece> pieces;
        crp[0] = 0;
        for (long long r = 0; r < n_rows; ++r) {
            crp[(size_t)r + 1] = crp[(size_t)r] + (long long)rcnt[(size_t)r];
            poff[(size_t)r] = (long long)pieces.size();
            for (long long q = crp[(size_t)r]; q < crp[(size_t)r + 1]; q += kOptPiece)
                pieces.push_back(OptPiece{q, (int)std::min<long long>(kOptPiece, crp[(size_t)r + 1] - q), (int)r});
        }
        poff[(size_t)n_rows] = (long long)pieces.size();
        const long long kept = crp[(size_t)n_rows];
        if ((rc = ensure(c, c->opt_ccol, (size_t)std::max(kept, 1ll) * 4, 0))) return rc;
        if ((rc = ensure(c, c->opt_cval, (size_t)std::max(kept, 1ll) * 4, 0))) return rc;
        if ((rc = ensure(c, c->opt_piece, std::max<size_t>(pieces.size(), 1) * sizeof(OptPiece), 0))) return rc;
        if ((rc = ensure(c, c->opt_gpart, std::max<size_t>(pieces.size(), 1) * 8, 0))) return rc;
        HIP_TRY(hipMemcpyAsync(c->opt_crp.ptr, crp.data(), crp.size() * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(c->opt_poff.ptr, poff.data(), poff.size() * 8, hipMemcpyHostToDevice, st));
        if (!pieces.empty())
            HIP_TRY(hipMemcpyAsync(c->opt_piece.ptr, pieces.data(), pieces.size() * sizeof(OptPiece),
                                   hipMemcpyHostToDevice, st));
        HIP_TRY(opt_roi_copy(F, (const long long *)c->opt_crp.ptr, (int32_t *)c->opt_ccol.ptr,
                             (float *)c->opt_cval.ptr, st));
        c->opt_npieces = (long long)pieces.size();
        O.col = (const int32_t *)c->opt_ccol.ptr;
        O.val = (const float *)c->opt_cval.ptr;
        std::vector<char> keep((size_t)nchunks, 0);
        for (int v = 0; v < nvox; ++v)
            if (roi_h[(size_t)v]) keep[(size_t)(v / kOptChunk)] = 1;
        if ((rc = build_buckets(O, c->opt_broi, keep, kept))) return rc;
        // the buckets hold voxel keys; the gradient's columns become indices
        // among the structure voxels, its residual a compact array
        std::vector<int32_t> sidx((size_t)nvox, -1);
        int ns = 0;
        for (int v = 0; v < nvox; ++v)
            if (roi_h[(size_t)v]) sidx[(size_t)v] = ns++;
        if ((rc = ensure(c, c->opt_sidx, (size_t)nvox * 4, 0))) return rc;
        if ((rc = ensure(c, c->opt_rstruct, (size_t)n_scen * std::max(ns, 1) * 4, 0))) return rc;
        HIP_TRY(hipMemcpyAsync(c->opt_sidx.ptr, sidx.data(), (size_t)nvox * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(opt_renumber((int32_t *)c->opt_ccol.ptr, kept, (const int32_t *)c->opt_sidx.ptr, nvox, st));
        HIP_TRY(hipStreamSynchronize(st));   // the host vector outlives the copy
        c->opt_nstruct = ns;
        memcpy(c->opt_dims, dims, sizeof dims);
        c->opt_rp_host.swap(rp);
        c->opt_roi_host.swap(roi_h);
        c->opt_col_src = dev ? (const void *)col : nullptr;
        c->opt_val_src = dev ? (const void *)val : nullptr;
        c->opt_valid = true;
    }
    O.col = (const int32_t *)c->opt_ccol.ptr;
    O.val = (const float *)c->opt_cval.ptr;
    O.piece = (const OptPiece *)c->opt_piece.ptr;
    O.n_pieces = c->opt_npieces;
    O.gpart = (double *)c->opt_gpart.ptr;
    O.rstruct = (float *)c->opt_rstruct.ptr;
    O.sidx = (const int32_t *)c->opt_sidx.ptr;
    O.nstruct = c->opt_nstruct;
    F.piece = O.piece;
    F.n_pieces = O.n_pieces;
    F.gpart = O.gpart;
    set_buckets(O, c->opt_broi);
    if (dose_gy && !c->opt_bfull.valid) {
        long long used = 0;
        for (long long r = 0; r < n_rows; ++r) {
            const long long crow = (r / n_spots) * stride + p->row_offset + r % n_spots;
            used += c->opt_rp_host[(size_t)crow + 1] - c->opt_rp_host[(size_t)crow];
        }
        if ((rc = build_buckets(F, c->opt_bfull, std::vector<char>(), used))) return rc;
    }
    HIP_TRY(hipMemcpyAsync(O.x, x, (size_t)n_spots * 8, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    double *hist = (double *)c->opt_hist.ptr;
    HIP_TRY(opt_update(O, kOptPowerInit, 0.0, 0, hist, st));
    for (int k = 0; k < p->n_power; ++k) {
        HIP_TRY(opt_forward(O, O.z, 1, nullptr, st));
        HIP_TRY(opt_gradient(O, st));
        HIP_TRY(opt_update(O, kOptPower, 0.0, 0, hist, st));
    }
    HIP_TRY(opt_update(O, kOptFistaInit, 0.0, 0, hist, st));
    double t = 1.0;
    for (int it = 0; it < p->iters; ++it) {
        HIP_TRY(opt_forward(O, O.y, 0, nullptr, st));
        HIP_TRY(opt_gradient(O, st));
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        HIP_TRY(opt_update(O, kOptFista, (t - 1.0) / tn, it, hist, st));
        t = tn;
    }
    HIP_TRY(opt_update(O, kOptFinalPrep, 0.0, 0, hist, st));
    float *dose_dev = nullptr;
    if (dose_gy) {
        if (dev) {
            dose_dev = dose_gy;
        } else {
            if ((rc = ensure(c, c->opt_dose, (size_t)n_scen * nvox * 4, 0))) return rc;
            dose_dev = (float *)c->opt_dose.ptr;
        }
    }
    if (dose_dev) {
        // the dose everywhere: the whole rows (objective from the same dose)
        set_buckets(F, c->opt_bfull);
        HIP_TRY(opt_forward(F, F.x, 2, dose_dev, st));
        HIP_TRY(opt_update(F, kOptFinal, 0.0, p->iters, hist, st));
    } else {
        HIP_TRY(opt_forward(O, O.x, 0, nullptr, st));
        HIP_TRY(opt_update(O, kOptFinal, 0.0, p->iters, hist, st));
    }
    const hipMemcpyKind out_kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIP_TRY(hipMemcpyAsync(x, O.x, (size_t)n_spots * 8, out_kind, st));
    if (obj_hist) HIP_TRY(hipMemcpyAsync(obj_hist, hist, ((size_t)p->iters + 1) * 8, out_kind, st));
    if (dose_gy && !dev)
        HIP_TRY(hipMemcpyAsync(dose_gy, dose_dev, (size_t)n_scen * nvox * 4, hipMemcpyDeviceToHost, st));
    double L = 0.0;
    HIP_TRY(hipMemcpyAsync(&L, O.scal + kOptL, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (step_L) *step_L = L;
    return VPMC_OK;
}

int vpmc_csr_cells(vpmc_ctx *c, const int64_t *row_ptr, int n_rows, const int32_t *col, const int64_t *q, int k,
                   const int32_t *cell_of_voxel, int n_cells, int64_t *row_ptr_out, int32_t *cell_out,
                   int64_t *q_out, float *val_out, unsigned flags) {
    if (!c) return fail(VPMC_E_ARG, "ctx is NULL");
    if (!row_ptr || !cell_of_voxel || !row_ptr_out) return fail(VPMC_E_ARG, "row_ptr, cell_of_voxel and row_ptr_out are required");
    if (n_rows < 0 || (long long)n_rows * 64 >= (1ll << 31)) return fail(VPMC_E_ARG, "n_rows outside [0, 2^25)");
    if (k < 0 || k > 62) return fail(VPMC_E_ARG, "k outside [0, 62]");
    if (n_cells < 1) return fail(VPMC_E_ARG, "n_cells must be >= 1");
    if (flags & ~VPMC_DEVICE_PTRS) return fail(VPMC_E_ARG, "unknown flags");
    if (!c->has_geom) return fail(VPMC_E_STATE, "no geometry loaded");
    const bool dev = (flags & VPMC_DEVICE_PTRS) != 0;
    const int nvox = (int)c->nvox;
    std::vector<int64_t> rp((size_t)n_rows + 1);
    std::vector<int32_t> cmap((size_t)nvox);
    if (dev) {
        if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
        HIP_TRY(hipSetDevice(c->device));
        HIP_TRY(hipMemcpy(rp.data(), row_ptr, rp.size() * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(cmap.data(), cell_of_voxel, cmap.size() * 4, hipMemcpyDeviceToHost));
    } else {
        memcpy(rp.data(), row_ptr, rp.size() * 8);
        memcpy(cmap.data(), cell_of_voxel, cmap.size() * 4);
    }
    if (rp[0] < 0) return fail(VPMC_E_ARG, "row_ptr[0] < 0");
    for (size_t r = 0; r + 1 < rp.size(); ++r)
        if (rp[r + 1] < rp[r]) return fail(VPMC_E_ARG, "row_ptr decreases at row %zu", r);
    // cells: runs of consecutive voxels, numbered 0 .. n_cells-1 in order
    if (cmap[0] != 0 || cmap[(size_t)nvox - 1] != n_cells - 1)
        return fail(VPMC_E_ARG, "cell map must start at 0 and end at n_cells - 1");
    std::vector<int32_t> cstart((size_t)n_cells + 1);
    cstart[0] = 0;
    for (int v = 1; v < nvox; ++v) {
        const int d = cmap[(size_t)v] - cmap[(size_t)v - 1];
        if (d != 0 && d != 1) return fail(VPMC_E_ARG, "cell map must grow by 0 or 1 from voxel to voxel (voxel %d)", v);
        if (d == 1) cstart[(size_t)cmap[(size_t)v]] = v;
    }
    cstart[(size_t)n_cells] = nvox;
    const long long nnz = rp[(size_t)n_rows] - rp[0];
    if (nnz > 0 && (!col || !q)) return fail(VPMC_E_ARG, "col and q are required");
    if (!dev && nnz > 0) {
        for (long long i = rp[0]; i < rp[(size_t)n_rows]; ++i)
            if ((unsigned)col[i] >= (unsigned)nvox) return fail(VPMC_E_ARG, "column %lld out of range", i);
    }
    if (c->device < 0) return fail(VPMC_E_STATE, "validation-only context has no device");
    HIP_TRY(hipSetDevice(c->device));
    int rc;
    const size_t R = (size_t)n_rows;
    if ((rc = ensure(c, c->cl_rp, (R + 1) * 8, 0))) return rc;
    if ((rc = ensure(c, c->cl_map, (size_t)nvox * 4, 0))) return rc;
    if ((rc = ensure(c, c->cl_start, ((size_t)n_cells + 1) * 4, 0))) return rc;
    if ((rc = ensure(c, c->cl_mass, (size_t)n_cells * 8, 0))) return rc;
    // pieces of at most kCellPiece entries, row by row
    std::vector<CellPiece> pcs;
    std::vector<size_t> first_piece(R + 1);
    for (size_t r = 0; r < R; ++r) {
        first_piece[r] = pcs.size();
        for (long long q0 = rp[r]; q0 < rp[r + 1]; q0 += kCellPiece)
            pcs.push_back(CellPiece{q0, (int)std::min<long long>(kCellPiece, rp[r + 1] - q0), (int)r});
    }
    first_piece[R] = pcs.size();
    const size_t NP = pcs.size();
    if ((rc = ensure(c, c->cl_piece, std::max<size_t>(NP, 1) * sizeof(CellPiece), 0))) return rc;
    if ((rc = ensure(c, c->cl_cnt, std::max<size_t>(NP, 1) * 8, 0))) return rc;
    if ((rc = ensure(c, c->cl_out, (NP + 1) * 8, 0))) return rc;
    if ((rc = ensure(c, c->flags, 4, 0))) return rc;
    HIP_TRY(hipMemcpy(c->cl_rp.ptr, rp.data(), rp.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->cl_map.ptr, cmap.data(), cmap.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->cl_start.ptr, cstart.data(), cstart.size() * 4, hipMemcpyHostToDevice));
    if (NP) HIP_TRY(hipMemcpy(c->cl_piece.ptr, pcs.data(), NP * sizeof(CellPiece), hipMemcpyHostToDevice));
    const int32_t *d_col = col;
    const long long *d_q = (const long long *)q;
    if (!dev && nnz > 0) {
        // host rows: the used range [rp[0], rp[n_rows]) is staged; offsets stay as given
        if ((rc = ensure(c, c->cl_col, (size_t)rp[R] * 4, 0))) return rc;
        if ((rc = ensure(c, c->cl_q, (size_t)rp[R] * 8, 0))) return rc;
        HIP_TRY(hipMemcpy(c->cl_col.ptr, col, (size_t)rp[R] * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->cl_q.ptr, q, (size_t)rp[R] * 8, hipMemcpyHostToDevice));
        d_col = (const int32_t *)c->cl_col.ptr;
        d_q = (const long long *)c->cl_q.ptr;
    }
    HIP_TRY(hipMemset(c->flags.ptr, 0, 4));
    HIP_TRY(launch_cell_count((const long long *)c->cl_rp.ptr, (const CellPiece *)c->cl_piece.ptr, (long long)NP,
                              d_col, (const int32_t *)c->cl_map.ptr, nvox, (unsigned long long *)c->cl_cnt.ptr,
                              (unsigned *)c->flags.ptr, nullptr));
    std::vector<unsigned long long> cnt(std::max<size_t>(NP, 1));
    unsigned err = 0;
    if (NP) HIP_TRY(hipMemcpy(cnt.data(), c->cl_cnt.ptr, NP * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&err, c->flags.ptr, 4, hipMemcpyDeviceToHost));
    if (err & 1u) return fail(VPMC_E_ARG, "a column index is outside [0, nvox)");
    if (err & 2u) return fail(VPMC_E_ARG, "columns are not ascending within a row");
    // output offsets: per piece (its own runs) and per row
    std::vector<int64_t> pout(NP + 1), op(R + 1);
    pout[0] = 0;
    for (size_t k = 0; k < NP; ++k) pout[k + 1] = pout[k] + (int64_t)cnt[k];
    for (size_t r = 0; r <= R; ++r) op[r] = pout[first_piece[r]];
    HIP_TRY(hipMemcpy(row_ptr_out, op.data(), op.size() * 8, dev ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    const long long nout = op[R];
    if (!cell_out && !q_out && !val_out) return VPMC_OK;
    HIP_TRY(hipMemcpy(c->cl_out.ptr, pout.data(), pout.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(launch_cell_mass(c->geom, (const int32_t *)c->cl_start.ptr, n_cells, (double *)c->cl_mass.ptr, nullptr));
    int32_t *ocell = cell_out;
    long long *oq = (long long *)q_out;
    float *oval = val_out;
    if (!dev) {
        const size_t n1 = (size_t)std::max(nout, 1ll);
        if (cell_out && (rc = ensure(c, c->cl_ocell, n1 * 4, 0))) return rc;
        if (q_out && (rc = ensure(c, c->cl_oq, n1 * 8, 0))) return rc;
        if (val_out && (rc = ensure(c, c->cl_oval, n1 * 4, 0))) return rc;
        ocell = cell_out ? (int32_t *)c->cl_ocell.ptr : nullptr;
        oq = q_out ? (long long *)c->cl_oq.ptr : nullptr;
        oval = val_out ? (float *)c->cl_oval.ptr : nullptr;
    }
    HIP_TRY(launch_cell_emit((const long long *)c->cl_rp.ptr, (const CellPiece *)c->cl_piece.ptr, (long long)NP, d_col,
                             d_q, (const int32_t *)c->cl_map.ptr, (const long long *)c->cl_out.ptr,
                             (const double *)c->cl_mass.ptr, ldexp(MEV_TO_J, -k),
                             ocell, oq, oval, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    if (!dev && nout > 0) {
        if (cell_out) HIP_TRY(hipMemcpy(cell_out, ocell, (size_t)nout * 4, hipMemcpyDeviceToHost));
        if (q_out) HIP_TRY(hipMemcpy(q_out, oq, (size_t)nout * 8, hipMemcpyDeviceToHost));
        if (val_out) HIP_TRY(hipMemcpy(val_out, oval, (size_t)nout * 4, hipMemcpyDeviceToHost));
    }
    return VPMC_OK;
}
