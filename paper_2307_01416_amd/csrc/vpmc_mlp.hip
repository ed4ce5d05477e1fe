// gfx950 kernels of the learned aperture surrogate: a multilayer perceptron
// 8 -> 256 -> 256 -> 256 -> 256 -> 29 (SiLU) with BF16 weights and
// activations and FP32 accumulation on the matrix cores, its loss and
// gradients (transmission cross-entropy + 4-component Gaussian mixture over
// outgoing energy loss / angle / offset) and an Adam optimiser with FP32
// master weights.
#include <math.h>

#include "vpmc_internal.hpp"

namespace vpmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C[m][n] = sum_k A(m,k) B(k,n) + bias[n], A(m,k) = AT ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = BT ? B[n*ldb+k] : B[k*ldb+n].  C (FP32) and/or Cb (BF16 of the
// activation, SiLU when ACT) are written.  Workgroup tile 64x64, four waves
// each own a 32x32 block computed with v_mfma_f32_32x32x16_bf16; K advances
// 16 at a time through LDS (B stored transposed so each lane's eight K values
// are contiguous).  Tails in M, N, K are zero-filled / masked.
template <bool AT, bool BT, bool ACT>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const __bf16 *__restrict__ A, int lda,
                                                        const __bf16 *__restrict__ B, int ldb,
                                                        const float *__restrict__ bias, float *C, int ldc,
                                                        __bf16 *Cb, int ldcb, int M, int N, int K) {
    __shared__ __attribute__((aligned(16))) __bf16 As[64][24];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[64][24];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    const __bf16 zero = (__bf16)0.0f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        {
            const int r = t >> 2, kk = (t & 3) * 4, m = m0 + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + kk + j;
                __bf16 val = zero;
                if (m < M && k < K) val = AT ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
                As[r][kk + j] = val;
            }
        }
        {
            const int c = t >> 2, kk = (t & 3) * 4, n = n0 + c;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + kk + j;
                __bf16 val = zero;
                if (n < N && k < K) val = BT ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
                Bs[c][kk + j] = val;
            }
        }
        __syncthreads();
        bf16x8 a, b;
        const int kb = 8 * (lane >> 5);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = As[wr + (lane & 31)][kb + j];
            b[j] = Bs[wc + (lane & 31)][kb + j];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        __syncthreads();
    }
    const int n = n0 + wc + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + wr + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (m < M && n < N) {
            const float z = acc[i] + (bias ? bias[n] : 0.0f);
            if (C) C[(size_t)m * ldc + n] = z;
            if (Cb) Cb[(size_t)m * ldcb + n] = (__bf16)(ACT ? silu_f(z) : z);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused inference: one workgroup (4 waves) carries 64 samples through all
// five layers.  The activations stay in LDS (two BF16 buffers of 64 x 256,
// rows padded to 264 to spread the banks); each wave computes 64 output
// columns of a hidden layer as 2 x 2 tiles of v_mfma_f32_32x32x16_bf16, its B
// fragments (eight consecutive K of one output unit, W[out][in] row-major)
// read straight from the L2-resident BF16 weights.  The K order and the
// instruction are those of gemm_bf16_kernel, so the outputs equal the
// layer-by-layer forward pass bit for bit.  REC: the inputs are computed from
// the deferred-VP records (same encoding as the training data) instead of
// read as FP32 rows of 8.
constexpr int kInfRows = 64;
constexpr int kInfLd = 264;

template <bool REC>
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float *__restrict__ x, const DeferRec *__restrict__ rec,
                                                        int n, const __bf16 *__restrict__ wb,
                                                        const float *__restrict__ wf, float *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) __bf16 H[2][kInfRows][kInfLd];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int row0 = blockIdx.x * kInfRows;
    const __bf16 zero = (__bf16)0.0f;
    if (t < kInfRows) {
        float in[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int r = row0 + t;
        if (r < n) {
            if (REC) {
                const DeferRec q = rec[r];
                in[0] = q.x / 20.0f;
                in[1] = q.y / 20.0f;
                in[2] = q.u / 0.05f;
                in[3] = q.v / 0.05f;
                in[4] = (q.E + q.Elo - 150.0f) / 50.0f;
                in[5] = fminf(q.d_edge, 100.0f) / 10.0f;
                in[6] = q.thick / 30.0f;
                in[7] = 0.0f;   // brass
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) in[j] = x[(size_t)r * 8 + j];
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            H[0][t][j] = (__bf16)in[j];
            H[0][t][8 + j] = zero;
        }
    }
    __syncthreads();
    int off = 0;   // parameter offset of the layer
#pragma unroll 1
    for (int l = 0; l < MLP_LAYERS; ++l) {
        const int ni = l == 0 ? MLP_IN : MLP_HIDDEN;
        const int no = l == MLP_LAYERS - 1 ? MLP_OUT : MLP_HIDDEN;
        const int K = l == 0 ? 16 : MLP_HIDDEN;
        const __bf16 *W = wb + off;
        const float *bias = wf + off + no * ni;
        const bool last = l == MLP_LAYERS - 1;
        // hidden layers: wave w owns columns 64w .. 64w+63 (2 x 2 tiles);
        // output layer: waves 0 and 1 each own one 32 x 32 tile (rows 32w)
        const int ntile = last ? 1 : 2, mtile = last ? 1 : 2;
        const int n0 = last ? 0 : 64 * w, m0 = last ? 32 * w : 0;
        if (!last || w < 2) {
            f32x16 acc[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
            const __bf16(*in)[kInfLd] = H[l & 1];
            const int kb = 8 * (lane >> 5);
            for (int k0 = 0; k0 < K; k0 += 16) {
                bf16x8 af[2], bfr[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    if (a < mtile) af[a] = *reinterpret_cast<const bf16x8 *>(&in[m0 + 32 * a + (lane & 31)][k0 + kb]);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if (b >= ntile) continue;
                    const int col = n0 + 32 * b + (lane & 31);
                    const int k = k0 + kb;
                    if (col < no && k < ni) {
                        bfr[b] = *reinterpret_cast<const bf16x8 *>(W + (size_t)col * ni + k);
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j) bfr[b][j] = zero;
                    }
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        if (a < mtile && b < ntile)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
            }
            __bf16(*ob)[kInfLd] = H[(l + 1) & 1];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if (a >= mtile || b >= ntile) continue;
                    const int col = n0 + 32 * b + (lane & 31);
                    const float bc = col < no ? bias[col] : 0.0f;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int r = m0 + 32 * a + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                        const float z = acc[a][b][i] + bc;
                        if (!last) {
                            ob[r][col] = (__bf16)silu_f(z);
                        } else if (col < no && row0 + r < n) {
                            out[(size_t)(row0 + r) * MLP_OUT + col] = z;
                        }
                    }
                }
        }
        off += no * ni + no;
        __syncthreads();
    }
}

__global__ void to_bf16_kernel(const float *__restrict__ x, __bf16 *__restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (__bf16)x[i];
}

// gather rows of x (n_cols wide) by index, converting to BF16
__global__ void gather_rows_kernel(const float *__restrict__ x, const int *__restrict__ idx, int n, int cols,
                                   __bf16 *xb, float *xf) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * cols; i += gridDim.x * blockDim.x) {
        const int r = i / cols, c = i - r * cols;
        const float v = x[(size_t)idx[r] * cols + c];
        if (xb) xb[i] = (__bf16)v;
        if (xf) xf[i] = v;
    }
}

// Per-sample loss and its gradient with respect to the 29 outputs (scaled
// by 1/n for the batch mean), written as FP32 and BF16.
__global__ void loss_head_kernel(const float *__restrict__ out, const float *__restrict__ y,
                                 const float *__restrict__ trans, int n, float inv_n, float *dout,
                                 __bf16 *dout_b, float *loss) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float *o = out + (size_t)s * 29;
    float g[29];
#pragma unroll
    for (int j = 0; j < 29; ++j) g[j] = 0.0f;
    const float lt = o[0], tr = trans[s];
    float L = fmaxf(lt, 0.0f) - lt * tr + log1pf(__expf(-fabsf(lt)));
    g[0] = 1.0f / (1.0f + __expf(-lt)) - tr;
    if (tr > 0.5f) {
        float mw = o[1];
#pragma unroll
        for (int c = 1; c < 4; ++c) mw = fmaxf(mw, o[1 + c]);
        float zs = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) zs += __expf(o[1 + c] - mw);
        const float lz = __logf(zs);
        float lw[4], lp[4], m = -INFINITY;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            lw[c] = o[1 + c] - mw - lz;
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float mu = o[5 + 3 * c + j], ls = o[17 + 3 * c + j];
                const float r = (y[(size_t)s * 3 + j] - mu) * __expf(-ls);
                acc += -0.5f * r * r - ls - 0.91893853320467274f;
            }
            lp[c] = lw[c] + acc;
            m = fmaxf(m, lp[c]);
        }
        float tot = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) tot += __expf(lp[c] - m);
        const float lse = m + __logf(tot);
        L -= lse;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float gam = __expf(lp[c] - lse), pic = __expf(lw[c]);
            g[1 + c] += pic - gam;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float mu = o[5 + 3 * c + j], ls = o[17 + 3 * c + j];
                const float iv = __expf(-2.0f * ls), d = y[(size_t)s * 3 + j] - mu;
                g[5 + 3 * c + j] += -gam * d * iv;
                g[17 + 3 * c + j] += -gam * (d * d * iv - 1.0f);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 29; ++j) {
        dout[(size_t)s * 29 + j] = g[j] * inv_n;
        dout_b[(size_t)s * 29 + j] = (__bf16)(g[j] * inv_n);
    }
    loss[s] = L;
}

// dZ = dH * silu'(Z), FP32 and BF16 copies
__global__ void silu_back_kernel(const float *__restrict__ dh, const float *__restrict__ z, float *dz,
                                 __bf16 *dz_b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float v = dh[i] * dsilu_f(z[i]);
        dz[i] = v;
        dz_b[i] = (__bf16)v;
    }
}

// bias gradient: column sums of dZ [n x cols]
__global__ void colsum_kernel(const float *__restrict__ dz, int n, int cols, float *gb) {
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < n; r += blockDim.x) s += dz[(size_t)r * cols + c];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[c] = red[0];
}

// Adam (Kingma and Ba) on FP32 master weights, refreshing the BF16 copy
__global__ void adam_kernel(float *p, const float *__restrict__ g, float *m, float *v, __bf16 *pb, int np,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        pb[i] = (__bf16)pi;
    }
}

__global__ void reduce_sum_kernel(const float *__restrict__ x, int n, float *out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

}  // namespace

// ------------------------------------------------------------------ host side
static const int kDims[MLP_LAYERS + 1] = {8, 256, 256, 256, 256, 29};

int mlp_param_count() {
    int n = 0;
    for (int l = 0; l < MLP_LAYERS; ++l) n += kDims[l + 1] * kDims[l] + kDims[l + 1];
    return n;
}

int mlp_param_offset(int layer) {
    int n = 0;
    for (int l = 0; l < layer; ++l) n += kDims[l + 1] * kDims[l] + kDims[l + 1];
    return n;
}

int mlp_dim(int i) { return kDims[i]; }

hipError_t mlp_gemm(bool at, bool bt, bool act, const __bf16 *A, int lda, const __bf16 *B, int ldb,
                    const float *bias, float *C, int ldc, __bf16 *Cb, int ldcb, int M, int N, int K, hipStream_t s) {
    dim3 grid((N + 63) / 64, (M + 63) / 64), block(256);
#define VPMC_GEMM(AT_, BT_, ACT_) \
    hipLaunchKernelGGL((gemm_bf16_kernel<AT_, BT_, ACT_>), grid, block, 0, s, A, lda, B, ldb, bias, C, ldc, Cb, ldcb, M, N, K)
    if (!at && bt && act) VPMC_GEMM(false, true, true);
    else if (!at && bt && !act) VPMC_GEMM(false, true, false);
    else if (!at && !bt) VPMC_GEMM(false, false, false);
    else if (at && !bt) VPMC_GEMM(true, false, false);
    else return hipErrorInvalidValue;
#undef VPMC_GEMM
    return hipGetLastError();
}

hipError_t mlp_forward(const MlpBuffers &b, int n, hipStream_t s) {
    // layer inputs: X (BF16 n x 8), H1..H4 (BF16 n x 256); pre-activations Z1..Z4 and OUT (FP32)
    hipError_t e = hipSuccess;
    for (int l = 0; l < MLP_LAYERS && e == hipSuccess; ++l) {
        const int ni = kDims[l], no = kDims[l + 1];
        const __bf16 *in = l == 0 ? b.x : b.h[l - 1];
        const __bf16 *W = b.wb + mlp_param_offset(l);
        const float *bias = b.w + mlp_param_offset(l) + no * ni;
        const bool last = l == MLP_LAYERS - 1;
        e = mlp_gemm(false, true, !last, in, ni, W, ni, bias, last ? b.out : b.z[l], no, last ? nullptr : b.h[l], no,
                     n, no, ni, s);
    }
    return e;
}

hipError_t mlp_loss_grad(const MlpBuffers &b, const float *y, const float *trans, int n, float *grad, float *loss,
                         hipStream_t s) {
    hipError_t e = mlp_forward(b, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_head_kernel, dim3((n + 255) / 256), dim3(256), 0, s, b.out, y, trans, n, 1.0f / n,
                       b.dout, b.dout_b, b.loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, b.loss, n, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // backward through the layers; dZ of the current layer in (dcur FP32, dcur_b BF16)
    const float *dcur = b.dout;
    const __bf16 *dcur_b = b.dout_b;
    for (int l = MLP_LAYERS - 1; l >= 0; --l) {
        const int ni = kDims[l], no = kDims[l + 1];
        const __bf16 *in = l == 0 ? b.x : b.h[l - 1];
        float *gW = grad + mlp_param_offset(l), *gb = gW + no * ni;
        // dW = dZ^T . H_in   (M = no, N = ni, K = n)
        if ((e = mlp_gemm(true, false, false, dcur_b, no, in, ni, nullptr, gW, ni, nullptr, 0, no, ni, n, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(colsum_kernel, dim3(no), dim3(256), 0, s, dcur, n, no, gb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l == 0) break;
        // dH_in = dZ . W   (M = n, N = ni, K = no), then dZ_in = dH_in * silu'(Z_in)
        const __bf16 *W = b.wb + mlp_param_offset(l);
        if ((e = mlp_gemm(false, false, false, dcur_b, no, W, ni, nullptr, b.dh, ni, nullptr, 0, n, ni, no, s)) != hipSuccess)
            return e;
        float *dz = (l & 1) ? b.dz_a : b.dz_b;
        __bf16 *dzb = (l & 1) ? b.dzb_a : b.dzb_b;
        hipLaunchKernelGGL(silu_back_kernel, dim3(grid_for((size_t)n * ni)), dim3(256), 0, s, b.dh, b.z[l - 1], dz, dzb,
                           (size_t)n * ni);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        dcur = dz;
        dcur_b = dzb;
    }
    return hipSuccess;
}

hipError_t mlp_infer(const float *x, const DeferRec *rec, int n, const __bf16 *wb, const float *wf, float *out,
                     hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + kInfRows - 1) / kInfRows), block(256);
    if (rec) hipLaunchKernelGGL(mlp_infer_kernel<true>, grid, block, 0, s, x, rec, n, wb, wf, out);
    else hipLaunchKernelGGL(mlp_infer_kernel<false>, grid, block, 0, s, x, rec, n, wb, wf, out);
    return hipGetLastError();
}

hipError_t mlp_gather(const float *x, const int *idx, int n, int cols, __bf16 *xb, float *xf, hipStream_t s) {
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((size_t)n * cols)), dim3(256), 0, s, x, idx, n, cols, xb, xf);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *x, __bf16 *y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t mlp_adam(float *p, const float *g, float *m, float *v, __bf16 *pb, int np, float lr, int step,
                    hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for((size_t)np)), dim3(256), 0, s, p, g, m, v, pb, np, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace vpmc
