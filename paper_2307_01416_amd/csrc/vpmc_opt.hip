// Spot-weight optimisation on influence matrices (the plan-optimisation
// step that consumes the 13-scenario matrices, Methods E).  Per iteration two
// HBM-bound sweeps over the CSR rows:
//   forward  D_s = A_s^T w : one workgroup per (voxel chunk, scenario) sums
//            the row segments that fall in its chunk into int64 fixed-point
//            LDS accumulators (order-independent, so bit-reproducible), then
//            turns the chunk's dose into the objective residual;
//   gradient g_j = sum_s A_s[j,:] r_s : one wavefront per row, FP64 sums in a
//            fixed order;
// and a one-workgroup update (power iteration for the step size, projected
// FISTA, the fixed-point scale of the next forward sweep).
#include <hip/hip_runtime.h>

#include <math.h>

#include "vpmc_internal.hpp"

namespace vpmc {

namespace {

constexpr int kOptThreads = 256;
static_assert(kOptChunk % kOptThreads == 0, "chunk tiles the workgroup");
constexpr int kUpdThreads = 1024;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ void set_err(unsigned *err, unsigned bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// CSR row of (scenario s, spot j)
__device__ __forceinline__ long long csr_row(const OptDev &O, int s, int j) {
    return (long long)s * O.row_stride + O.row_offset + j;
}

// Pass 1 over the rows: segments per (scenario, chunk), validation of the
// columns and values, largest |a| per row.  A segment is a maximal run of a
// row's entries inside one voxel chunk; it starts at every entry whose chunk
// differs from its predecessor's.
__global__ void __launch_bounds__(kOptThreads) opt_count_kernel(OptDev O, unsigned *cnt, unsigned *err) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const int lane = lane_id();
    int carry = -1;
    float amax = 0.0f;
    for (long long i0 = b; i0 < e; i0 += 64) {
        const long long i = i0 + lane;
        const bool valid = i < e;
        int ck = -2;
        if (valid) {
            const int c = O.col[i];
            const float a = O.val[i];
            if ((unsigned)c >= (unsigned)O.nvox) set_err(err, 1u);
            else ck = c / kOptChunk;
            if (!isfinite(a)) set_err(err, 2u);
            else amax = fmaxf(amax, fabsf(a));
        }
        int prev = __shfl_up(ck, 1);
        if (lane == 0) prev = carry;
        if (valid && ck >= 0 && ck != prev) atomicAdd(&cnt[(size_t)s * O.nchunks + ck], 1u);
        carry = __shfl(ck, 63);
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    if (lane == 0) O.amax[r] = amax;
}

// Exclusive scan of n counts into off[0..n] by one workgroup; the counts are
// cleared (they serve next as the emit pass's cursors).
__global__ void __launch_bounds__(kUpdThreads) opt_scan_kernel(unsigned *cnt, unsigned long long *off, size_t n) {
    __shared__ unsigned long long part[kUpdThreads];
    const size_t per = (n + kUpdThreads - 1) / kUpdThreads;
    const size_t lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    unsigned long long sum = 0;
    for (size_t k = lo; k < hi; ++k) sum += cnt[k];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kUpdThreads; d <<= 1) {
        const unsigned long long v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long run = part[threadIdx.x] - sum;
    for (size_t k = lo; k < hi; ++k) {
        off[k] = run;
        run += cnt[k];
        cnt[k] = 0u;
    }
    if (threadIdx.x == kUpdThreads - 1) off[n] = part[kUpdThreads - 1];
}

// Pass 2 over the rows: every segment start after the row's first entry
// closes the segment before it, which is written to its (scenario, chunk)
// list; lane 0 closes the row's last segment.  The order inside a list does
// not matter (the forward sums are integers).
__global__ void __launch_bounds__(kOptThreads) opt_emit_kernel(OptDev O, const unsigned long long *off,
                                                               unsigned *cur, OptSeg *seg, unsigned long long cap) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const int lane = lane_id();
    int carry_ck = -1;
    long long carry_start = b;
    auto put = [&](int ck, long long start, long long end) {
        const size_t list = (size_t)s * O.nchunks + ck;
        const unsigned long long pos = off[list] + atomicAdd(&cur[list], 1u);
        if (pos < cap && pos < off[list + 1]) {
            OptSeg q;
            q.begin = start;
            q.len = (int)(end - start);
            q.spot = j;
            seg[pos] = q;
        }
    };
    for (long long i0 = b; i0 < e; i0 += 64) {
        const long long i = i0 + lane;
        const bool valid = i < e;
        int ck = -2;
        if (valid) {
            const int c = O.col[i];
            if ((unsigned)c < (unsigned)O.nvox) ck = c / kOptChunk;
        }
        int prev = __shfl_up(ck, 1);
        if (lane == 0) prev = carry_ck;
        const bool start = valid && ck >= 0 && ck != prev;
        const unsigned long long m = __ballot(start);
        if (start && i > b) {
            // previous start: the highest start below this lane, else the carry
            const unsigned long long below = m & ((1ull << lane) - 1ull);
            const long long ps = below ? i0 + (63 - __clzll((long long)below)) : carry_start;
            if (prev >= 0) put(prev, ps, i);
        }
        if (m) carry_start = i0 + (63 - __clzll((long long)m));
        carry_ck = __shfl(ck, 63);
        if (i0 + 64 >= e) carry_ck = __shfl(ck, (int)(e - 1 - i0));
    }
    if (lane == 0 && e > b && carry_ck >= 0) put(carry_ck, carry_start, e);
}

// Forward sweep of one (chunk, scenario).  mode 0: objective residual and
// objective partial; mode 1: residual M D of the power iteration (M = the
// target and organ weights); mode 2: as mode 0 and the dose into dose_out.
__global__ void __launch_bounds__(kOptThreads) opt_forward_kernel(OptDev O, const double *w, int mode, float *dose_out) {
    __shared__ unsigned long long acc[kOptChunk];
    __shared__ double red[kOptThreads / 64];
    const int c = blockIdx.x, s = blockIdx.y;
    const long long base = (long long)c * kOptChunk;
    const int nv = (int)(O.nvox - base < kOptChunk ? O.nvox - base : kOptChunk);
    for (int v = threadIdx.x; v < kOptChunk; v += kOptThreads) acc[v] = 0ull;
    __syncthreads();
    const double sc = O.scale[s], isc = O.scale[O.n_scen + s];
    const size_t list = (size_t)s * O.nchunks + c;
    const unsigned long long k0 = O.seg_off[list], k1 = O.seg_off[list + 1];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    for (unsigned long long k = k0 + wave; k < k1; k += kOptThreads / 64) {
        const OptSeg q = O.seg[k];
        const double ws = w[q.spot] * sc;
        const long long end = q.begin + q.len;
        for (long long i = q.begin + lane; i < end; i += 64) {
            const int v = O.col[i] - (int)base;
            const double t = rint(ws * (double)O.val[i]);
            if ((unsigned)v < (unsigned)nv) atomicAdd(&acc[v], (unsigned long long)(long long)t);
        }
    }
    __syncthreads();
    double f = 0.0;
    float *res = O.resid + (size_t)s * O.nvox + base;
    const unsigned char *roi = O.roi + base;
    for (int v = threadIdx.x; v < nv; v += kOptThreads) {
        const double D = (double)(long long)acc[v] * isc;
        const unsigned m = roi[v];
        double r = 0.0;
        if (mode == 1) {
            const double mw = ((m & 1u) ? O.w_target : 0.0) + ((m & 2u) ? O.w_oar : 0.0);
            r = mw * D;
        } else {
            if (m & 1u) {
                const double d = D - O.d_presc;
                r += O.w_target * d;
                f += O.w_target * d * d;
            }
            if (m & 2u) {
                const double d = D > O.d_max ? D - O.d_max : 0.0;
                r += O.w_oar * d;
                f += O.w_oar * d * d;
            }
            if (mode == 2 && dose_out) dose_out[(size_t)s * O.nvox + base + v] = (float)D;
        }
        res[v] = (float)r;
    }
    if (mode == 1) return;
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if (lane == 0) red[threadIdx.x >> 6] = f;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kOptThreads / 64; ++q) t += red[q];
        O.fpart[list] = t;
    }
}

// Gradient sweep: wavefront per row, FP64 products of FP32 values (exact),
// summed per lane in entry order then over lanes by a fixed butterfly.
__global__ void __launch_bounds__(kOptThreads) opt_grad_kernel(OptDev O) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const float *res = O.resid + (size_t)s * O.nvox;
    const int lane = lane_id();
    double a0 = 0.0, a1 = 0.0;
    long long i = b + lane;
    for (; i + 64 < e; i += 128) {
        const int c0 = O.col[i], c1 = O.col[i + 64];
        const float v0 = O.val[i], v1 = O.val[i + 64];
        const float r0 = (unsigned)c0 < (unsigned)O.nvox ? res[c0] : 0.0f;
        const float r1 = (unsigned)c1 < (unsigned)O.nvox ? res[c1] : 0.0f;
        a0 = fma((double)v0, (double)r0, a0);
        a1 = fma((double)v1, (double)r1, a1);
    }
    if (i < e) {
        const int c0 = O.col[i];
        const float r0 = (unsigned)c0 < (unsigned)O.nvox ? res[c0] : 0.0f;
        a0 = fma((double)O.val[i], (double)r0, a0);
    }
    double a = a0 + a1;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) O.gpart[r] = a;
}

__device__ double block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < kUpdThreads / 64; ++q) t += red[q];
    return t;
}

// fixed-point scale of the next forward sweep over vector w: 2^m with
// sum_j |w_j| max|A_s[j,:]| < 2^60, so every int64 sum stays in range
__device__ void set_scales(const OptDev &O, const double *w, double *red) {
    for (int s = 0; s < O.n_scen; ++s) {
        double bnd = 0.0;
        for (int j = threadIdx.x; j < O.n_spots; j += kUpdThreads)
            bnd += fabs(w[j]) * (double)O.amax[(size_t)s * O.n_spots + j];
        bnd = block_sum(bnd, red);
        if (threadIdx.x == 0) {
            int ex = 0;
            if (bnd > 0.0) (void)frexp(bnd, &ex);
            const int m = bnd > 0.0 ? 60 - ex : 0;
            O.scale[s] = ldexp(1.0, m);
            O.scale[O.n_scen + s] = ldexp(1.0, -m);
        }
    }
}

// Objective over the forward sweep's partials, fixed order.
__device__ double objective(const OptDev &O, double *red) {
    const size_t n = (size_t)O.n_scen * O.nchunks;
    double f = 0.0;
    for (size_t k = threadIdx.x; k < n; k += kUpdThreads) f += O.fpart[k];
    return block_sum(f, red) / (double)O.n_scen;
}

// One workgroup.  Modes: kOptPowerInit (z = 1), kOptPower (lam = |g|/|z|,
// z = g/|g|), kOptFistaInit (L = 1.05 lam, x = max(x, 0), y = x), kOptFista
// (objective of the sweep into hist[it]; x+ = P(y - g/L), y = x+ + beta (x+ - x)),
// kOptFinalPrep (scale for x), kOptFinal (objective at x into hist[it]).
__global__ void __launch_bounds__(kUpdThreads) opt_update_kernel(OptDev O, int mode, double beta, int it,
                                                                 double *hist) {
    __shared__ double red[kUpdThreads / 64];
    const int n = O.n_spots;
    const double g_scale = 2.0 / (double)O.n_scen;
    if (mode == kOptPowerInit) {
        for (int j = threadIdx.x; j < n; j += kUpdThreads) O.z[j] = 1.0;
        __syncthreads();
        set_scales(O, O.z, red);
        return;
    }
    if (mode == kOptPower) {
        double gg = 0.0, zz = 0.0;
        for (int j = threadIdx.x; j < n; j += kUpdThreads) {
            double g = 0.0;
            for (int s = 0; s < O.n_scen; ++s) g += O.gpart[(size_t)s * n + j];
            g *= g_scale;
            O.gvec[j] = g;
            gg += g * g;
            zz += O.z[j] * O.z[j];
        }
        gg = block_sum(gg, red);
        zz = block_sum(zz, red);
        const double gn = sqrt(gg), zn = sqrt(zz);
        if (threadIdx.x == 0) O.scal[kOptLam] = zn > 0.0 ? gn / zn : 0.0;
        if (gn > 0.0)
            for (int j = threadIdx.x; j < n; j += kUpdThreads) O.z[j] = O.gvec[j] / gn;
        __syncthreads();
        set_scales(O, O.z, red);
        return;
    }
    if (mode == kOptFistaInit) {
        if (threadIdx.x == 0) O.scal[kOptL] = 1.05 * O.scal[kOptLam];
        for (int j = threadIdx.x; j < n; j += kUpdThreads) {
            const double x = O.x[j] > 0.0 ? O.x[j] : 0.0;
            O.x[j] = x;
            O.y[j] = x;
        }
        __syncthreads();
        set_scales(O, O.y, red);
        return;
    }
    if (mode == kOptFista) {
        const double F = objective(O, red);
        if (threadIdx.x == 0 && hist) hist[it] = F;
        const double L = O.scal[kOptL];
        for (int j = threadIdx.x; j < n; j += kUpdThreads) {
            double g = 0.0;
            for (int s = 0; s < O.n_scen; ++s) g += O.gpart[(size_t)s * n + j];
            g *= g_scale;
            double xn = L > 0.0 ? O.y[j] - g / L : O.y[j];
            xn = xn > 0.0 ? xn : 0.0;
            O.y[j] = xn + beta * (xn - O.x[j]);
            O.x[j] = xn;
        }
        __syncthreads();
        set_scales(O, O.y, red);
        return;
    }
    if (mode == kOptFinalPrep) {
        set_scales(O, O.x, red);
        return;
    }
    // kOptFinal
    const double F = objective(O, red);
    if (threadIdx.x == 0 && hist) hist[it] = F;
}

}  // namespace

hipError_t opt_build_count(const OptDev &O, unsigned *cnt, unsigned *err, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_count_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, cnt, err);
    return hipGetLastError();
}

hipError_t opt_build_scan(unsigned *cnt, unsigned long long *off, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(opt_scan_kernel, dim3(1), dim3(kUpdThreads), 0, st, cnt, off, n);
    return hipGetLastError();
}

hipError_t opt_build_emit(const OptDev &O, const unsigned long long *off, unsigned *cur, OptSeg *seg,
                          unsigned long long cap, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_emit_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, off, cur, seg, cap);
    return hipGetLastError();
}

hipError_t opt_forward(const OptDev &O, const double *w, int mode, float *dose_out, hipStream_t st) {
    hipLaunchKernelGGL(opt_forward_kernel, dim3((unsigned)O.nchunks, (unsigned)O.n_scen), dim3(kOptThreads), 0, st,
                       O, w, mode, dose_out);
    return hipGetLastError();
}

hipError_t opt_gradient(const OptDev &O, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_grad_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O);
    return hipGetLastError();
}

hipError_t opt_update(const OptDev &O, int mode, double beta, int it, double *hist, hipStream_t st) {
    hipLaunchKernelGGL(opt_update_kernel, dim3(1), dim3(kUpdThreads), 0, st, O, mode, beta, it, hist);
    return hipGetLastError();
}

}  // namespace vpmc
