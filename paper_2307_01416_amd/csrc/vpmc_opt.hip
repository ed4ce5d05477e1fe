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
constexpr int kUpdThreads = 1024;
constexpr int kFwdThreads = 512;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ void set_err(unsigned *err, unsigned bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// CSR row of (scenario s, spot j)
__device__ __forceinline__ long long csr_row(const OptDev &O, int s, int j) {
    return (long long)s * O.row_stride + O.row_offset + j;
}

// Pass 1 over the rows: entries per (scenario, chunk), validation of the
// columns and values.  A segment is a maximal run of a
// row's entries inside one voxel chunk; it starts at every entry whose chunk
// differs from its predecessor's.
__global__ void __launch_bounds__(kOptThreads) opt_count_kernel(OptDev O, unsigned long long *cnt, unsigned *err) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const int lane = lane_id();
    int carry = -1;
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
        }
        int prev = __shfl_up(ck, 1);
        if (lane == 0) prev = carry;
        // entries per (scenario, chunk): one add per segment start, of the
        // segment's entry count inside this window; continuing segments add
        // the rest at the next window's lane 0
        const bool start = valid && ck >= 0 && (ck != prev || lane == 0);
        const unsigned long long m = __ballot(start);
        if (start) {
            const unsigned long long above = m & ~((2ull << lane) - 1ull);
            const long long stop = above ? i0 + (__ffsll((long long)above) - 1) : (i0 + 64 < e ? i0 + 64 : e);
            atomicAdd(&cnt[(size_t)s * O.nchunks + ck], (unsigned long long)(stop - i));
        }
        carry = __shfl(ck, 63);
    }
}

// Exclusive scan of n counts into off[0..n] by one workgroup; the counts are
// cleared (they serve next as the emit pass's cursors).
__global__ void __launch_bounds__(kUpdThreads) opt_scan_kernel(unsigned long long *cnt, unsigned long long *off, size_t n) {
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
        cnt[k] = 0ull;
    }
    if (threadIdx.x == kUpdThreads - 1) off[n] = part[kUpdThreads - 1];
}

// Restriction to the structures: the objective and its gradient involve only
// voxels with a structure bit, so the iterations run on the rows' entries in
// those voxels.  Count pass (also validates every entry and takes the
// largest |a| of each whole row) and copy pass (entries kept in row order).
__global__ void __launch_bounds__(kOptThreads) opt_roi_count_kernel(OptDev O, unsigned long long *rcnt,
                                                                    unsigned *err) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const int lane = lane_id();
    float amax = 0.0f;
    unsigned long long kept = 0;
    for (long long i = b + lane; i < e; i += 64) {
        const int c = O.col[i];
        const float a = O.val[i];
        if ((unsigned)c >= (unsigned)O.nvox) set_err(err, 1u);
        else if (O.roi[c]) ++kept;
        if (!isfinite(a)) set_err(err, 2u);
        else amax = fmaxf(amax, fabsf(a));
    }
    for (int o = 32; o > 0; o >>= 1) {
        amax = fmaxf(amax, __shfl_xor(amax, o));
        kept += __shfl_xor(kept, o);
    }
    if (lane == 0) {
        O.amax[r] = amax;
        rcnt[r] = kept;
    }
}

__global__ void __launch_bounds__(kOptThreads) opt_roi_copy_kernel(OptDev O, const long long *rptr, int32_t *ccol,
                                                                   float *cval) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const long long o0 = rptr[r], o1 = rptr[r + 1];
    const int lane = lane_id();
    long long out = o0;
    for (long long i0 = b; i0 < e; i0 += 64) {
        const long long i = i0 + lane;
        int c = -1;
        if (i < e) c = O.col[i];
        const bool keep = (unsigned)c < (unsigned)O.nvox && O.roi[c] != 0;
        const unsigned long long m = __ballot(keep);
        const long long pos = out + __popcll(m & ((1ull << lane) - 1ull));
        if (keep && pos < o1) {
            ccol[pos] = c;
            cval[pos] = O.val[i];
        }
        out += __popcll(m);
    }
}

// Column renumbering of the structure-restricted rows: voxel -> its index
// among the structure voxels (-1 for any other, which the gradient skips).
__global__ void __launch_bounds__(kOptThreads) opt_renumber_kernel(int32_t *ccol, long long n, const int32_t *sidx,
                                                                   int nvox) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int c = ccol[i];
        ccol[i] = (unsigned)c < (unsigned)nvox ? sidx[c] : -1;
    }
}

// Pass 2 over the rows: the entries of every segment are copied, as one
// block, into the entry range of its (scenario, chunk) list: key (spot <<
// kOptChunkBits | voxel - chunk base) and value.  A segment closes at the next segment
// start of the row or at the row's end; the whole wavefront copies it.  The
// order of blocks inside a list does not matter (the dose sums are integers).
__global__ void __launch_bounds__(kOptThreads) opt_emit_kernel(OptDev O, const unsigned long long *off,
                                                               unsigned long long *cur, uint32_t *bkey, float *bval) {
    const int r = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (r >= O.n_scen * O.n_spots) return;
    const int s = r / O.n_spots, j = r - s * O.n_spots;
    const long long crow = csr_row(O, s, j);
    const long long b = O.row_ptr[crow], e = O.row_ptr[crow + 1];
    const int lane = lane_id();
    int carry_ck = -1;
    long long carry_start = b;
    auto copy = [&](int ck, long long start, long long end) {
        const size_t list = (size_t)s * O.nchunks + ck;
        const long long len = end - start;
        unsigned long long pos = 0;
        if (lane == 0) pos = off[list] + atomicAdd(&cur[list], (unsigned long long)len);
        pos = __shfl(pos, 0);
        if (pos + len > off[list + 1]) return;   // cannot happen after a consistent count pass
        const uint32_t hi = (uint32_t)j << kOptChunkBits;
        const int base = ck * kOptChunk;
        for (long long t = lane; t < len; t += 64) {
            bkey[pos + t] = hi | (uint32_t)(O.col[start + t] - base);
            bval[pos + t] = O.val[start + t];
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
        // closes in lane order: the start at lane l closes [previous start, i0 + l)
        long long ps = carry_start;
        for (unsigned long long mm = m; mm; mm &= mm - 1ull) {
            const int l = __ffsll((long long)mm) - 1;
            const int pck = __shfl(prev, l);
            if (i0 + l > b && pck >= 0) copy(pck, ps, i0 + l);
            ps = i0 + l;
        }
        carry_start = ps;
        carry_ck = __shfl(ck, 63);
        if (i0 + 64 >= e) carry_ck = __shfl(ck, (int)(e - 1 - i0));
    }
    if (e > b && carry_ck >= 0) copy(carry_ck, carry_start, e);
}

// Forward sweep of one (scenario, chunk) item of the work list (items in
// decreasing entry count).  mode 0: objective residual and objective partial;
// mode 1: residual M D of the power iteration (M = the target and organ
// weights); mode 2: as mode 0 and the dose into dose_out.
__global__ void __launch_bounds__(kFwdThreads) opt_forward_kernel(OptDev O, const double *w, int mode, float *dose_out) {
    __shared__ unsigned long long acc[kOptChunk];
    __shared__ double red[kFwdThreads / 64];
    const unsigned item = O.work[blockIdx.x];
    const int s = (int)(item / (unsigned)O.nchunks), c = (int)(item - (unsigned)s * O.nchunks);
    const long long base = (long long)c * kOptChunk;
    const int nv = (int)(O.nvox - base < kOptChunk ? O.nvox - base : kOptChunk);
    for (int v = threadIdx.x; v < kOptChunk; v += kFwdThreads) acc[v] = 0ull;
    __syncthreads();
    const double sc = O.scale[s], isc = O.scale[O.n_scen + s];
    const size_t list = (size_t)s * O.nchunks + c;
    const long long e0 = (long long)O.boff[list], e1 = (long long)O.boff[list + 1];
    const uint32_t *bk = O.bkey;
    const float *bv = O.bval;
    long long e = e0 + threadIdx.x;
    for (; e + 3 * kFwdThreads < e1; e += 4 * kFwdThreads) {
        uint32_t k[4];
        float a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            k[u] = bk[e + u * kFwdThreads];
            a[u] = bv[e + u * kFwdThreads];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t j = k[u] >> kOptChunkBits;
            if (j < (uint32_t)O.n_spots) {
                const double t = rint(w[j] * sc * (double)a[u]);
                atomicAdd(&acc[k[u] & (kOptChunk - 1)], (unsigned long long)(long long)t);
            }
        }
    }
    for (; e < e1; e += kFwdThreads) {
        const uint32_t k = bk[e], j = k >> kOptChunkBits;
        if (j < (uint32_t)O.n_spots) {
            const double t = rint(w[j] * sc * (double)bv[e]);
            atomicAdd(&acc[k & (kOptChunk - 1)], (unsigned long long)(long long)t);
        }
    }
    __syncthreads();
    double f = 0.0;
    float *res = O.resid + (size_t)s * O.nvox + base;
    const unsigned char *roi = O.roi + base;
    for (int v = threadIdx.x; v < nv; v += kFwdThreads) {
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
        if (O.rstruct && m) {
            // the structure voxels' residual, compact: what the gradient gathers
            const int si = O.sidx[base + v];
            if ((unsigned)si < (unsigned)O.nstruct) O.rstruct[(size_t)s * O.nstruct + si] = (float)r;
        }
    }
    if (mode == 1) return;
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = f;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kFwdThreads / 64; ++q) t += red[q];
        O.fpart[blockIdx.x] = t;
    }
}

// Gradient sweep: a wavefront per piece (at most kOptPiece consecutive
// entries of one row), FP64 products of FP32 values (exact) summed per lane
// in entry order, then over lanes by a fixed butterfly; pieces of a row are
// summed in order by the update.
__global__ void __launch_bounds__(kOptThreads) opt_grad_kernel(OptDev O) {
    const long long p = (long long)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
    if (p >= O.n_pieces) return;
    const OptPiece q = O.piece[p];
    const int r = __builtin_amdgcn_readfirstlane(q.row);
    const int s = r / O.n_spots;
    // columns renumbered to structure voxels: the residual gathered is the
    // compact one (n_scen x nstruct floats, cache-resident)
    const float *res = O.rstruct + (size_t)s * O.nstruct;
    const int lane = lane_id();
    const long long e = q.begin + q.len;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    long long i = q.begin + lane;
    for (; i + 192 < e; i += 256) {
        int c[4];
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = O.col[i + 64 * u];
            v[u] = O.val[i + 64 * u];
        }
        float rr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) rr[u] = (unsigned)c[u] < (unsigned)O.nstruct ? res[c[u]] : 0.0f;
        a0 = fma((double)v[0], (double)rr[0], a0);
        a1 = fma((double)v[1], (double)rr[1], a1);
        a2 = fma((double)v[2], (double)rr[2], a2);
        a3 = fma((double)v[3], (double)rr[3], a3);
    }
    for (; i < e; i += 64) {
        const int c0 = O.col[i];
        const float r0 = (unsigned)c0 < (unsigned)O.nstruct ? res[c0] : 0.0f;
        a0 = fma((double)O.val[i], (double)r0, a0);
    }
    double a = (a0 + a1) + (a2 + a3);
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) O.gpart[p] = a;
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

// sum over scenarios of A_s[j,:] r_s: the row pieces in order
__device__ double row_gradient(const OptDev &O, int j) {
    double g = 0.0;
    for (int s = 0; s < O.n_scen; ++s) {
        const size_t r = (size_t)s * O.n_spots + j;
        for (long long p = O.piece_off[r]; p < O.piece_off[r + 1]; ++p) g += O.gpart[p];
    }
    return g;
}

// Objective over the forward sweep's partials, fixed order.
__device__ double objective(const OptDev &O, double *red) {
    const size_t n = (size_t)O.n_work;
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
            const double g = row_gradient(O, j) * g_scale;
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
            const double g = row_gradient(O, j) * g_scale;
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

hipError_t opt_build_count(const OptDev &O, unsigned long long *cnt, unsigned *err, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_count_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, cnt, err);
    return hipGetLastError();
}

hipError_t opt_roi_count(const OptDev &O, unsigned long long *rcnt, unsigned *err, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_roi_count_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, rcnt, err);
    return hipGetLastError();
}

hipError_t opt_renumber(int32_t *ccol, long long n, const int32_t *sidx, int nvox, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n + kOptThreads - 1) / kOptThreads, 65536);
    hipLaunchKernelGGL(opt_renumber_kernel, dim3((unsigned)blocks), dim3(kOptThreads), 0, st, ccol, n, sidx, nvox);
    return hipGetLastError();
}

hipError_t opt_roi_copy(const OptDev &O, const long long *rptr, int32_t *ccol, float *cval, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_roi_copy_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, rptr, ccol, cval);
    return hipGetLastError();
}

hipError_t opt_build_scan(unsigned long long *cnt, unsigned long long *off, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(opt_scan_kernel, dim3(1), dim3(kUpdThreads), 0, st, cnt, off, n);
    return hipGetLastError();
}

hipError_t opt_build_emit(const OptDev &O, const unsigned long long *off, unsigned long long *cur, uint32_t *bkey,
                          float *bval, hipStream_t st) {
    const long long rows = (long long)O.n_scen * O.n_spots;
    const int blocks = (int)((rows * 64 + kOptThreads - 1) / kOptThreads);
    hipLaunchKernelGGL(opt_emit_kernel, dim3(blocks), dim3(kOptThreads), 0, st, O, off, cur, bkey, bval);
    return hipGetLastError();
}

hipError_t opt_forward(const OptDev &O, const double *w, int mode, float *dose_out, hipStream_t st) {
    if (O.n_work == 0) return hipSuccess;
    hipLaunchKernelGGL(opt_forward_kernel, dim3((unsigned)O.n_work), dim3(kFwdThreads), 0, st, O, w, mode, dose_out);
    return hipGetLastError();
}

hipError_t opt_gradient(const OptDev &O, hipStream_t st) {
    if (O.n_pieces == 0) return hipSuccess;
    const long long blocks = (O.n_pieces * 64 + kOptThreads - 1) / kOptThreads;
    hipLaunchKernelGGL(opt_grad_kernel, dim3((unsigned)blocks), dim3(kOptThreads), 0, st, O);
    return hipGetLastError();
}

hipError_t opt_update(const OptDev &O, int mode, double beta, int it, double *hist, hipStream_t st) {
    hipLaunchKernelGGL(opt_update_kernel, dim3(1), dim3(kUpdThreads), 0, st, O, mode, beta, it, hist);
    return hipGetLastError();
}

}  // namespace vpmc
