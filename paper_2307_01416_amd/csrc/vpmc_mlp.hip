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

// C[m][n] = sum_k A(m,k) B(k,n) over one K range, A(m,k) = AT ? A[k*lda+m] :
// A[m*lda+k], B(k,n) = BT ? B[n*ldb+k] : B[k*ldb+n].  Workgroup tile 64x64,
// four waves each own a 32x32 block computed with v_mfma_f32_32x32x16_bf16,
// K advancing 64 per LDS stage (next stage's 16-byte global loads in flight
// in registers during the current stage's MFMAs).  The operand whose
// contiguous dimension is K is copied to LDS as is; the other is transposed
// on the way in, so each lane's eight K values are contiguous in LDS.  Loads
// are 8 elements wide: pitches and pointers are multiples of 8 elements and
// the contiguous dimension of each operand is readable up to the next
// multiple of 8 (elements past M or N only reach masked outputs; elements
// past K are zeroed).  blockIdx.z selects the K range [z*kchunk, ...) for a
// split-K product; its partial goes to C + z*czs.
//   EPI_F32:   C = acc (+ bias[n])                                   (FP32)
//   EPI_SILU:  C = z = acc + bias[n], Cb = bf16(silu(z))             (forward)
//   EPI_DSILU: d = acc * silu'(aux[m*ldc+n]), Cb = bf16(d), and the sum of d
//              over each 32-row block into C[(m/32)*ldc + n]          (backward)
// For a given element the k16 MFMAs run in ascending K order into one
// accumulator, as in the fused inference kernel below.
enum { EPI_F32 = 0, EPI_SILU = 1, EPI_DSILU = 2 };
constexpr int kGT = 64, kGK = 64, kGLd = kGK + 8;

template <bool AT>
__device__ __forceinline__ void gemm_fetch(const __bf16 *__restrict__ P, int ld, int rows, int r0, int k0, int kend,
                                           int t, uint4 (&r)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = t + 256 * h, outer = c >> 3, inner = (c & 7) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (!AT) {   // rows of the tile, K contiguous
            const int row = r0 + outer, k = k0 + inner;
            if (row < rows && k < kend) {
                v = *(const uint4 *)(P + (size_t)row * ld + k);
                if (k + 8 > kend) {   // zero the elements past K
                    unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (k + j >= kend) w[j >> 1] &= (j & 1) ? 0x0000FFFFu : 0xFFFF0000u;
                    v = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        } else {     // K rows, tile rows contiguous
            const int k = k0 + outer, row = r0 + inner;
            if (k < kend && row < rows) v = *(const uint4 *)(P + (size_t)k * ld + row);
        }
        r[h] = v;
    }
}

template <bool AT>
__device__ __forceinline__ void gemm_stash(unsigned short *L, int t, const uint4 (&r)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = t + 256 * h, outer = c >> 3, inner = (c & 7) * 8;
        if (!AT) {
            *(uint4 *)(L + outer * kGLd + inner) = r[h];
        } else {
            const unsigned int w[4] = {r[h].x, r[h].y, r[h].z, r[h].w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                L[(inner + j) * kGLd + outer] = (unsigned short)(w[j >> 1] >> (16 * (j & 1)));
        }
    }
}

template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const __bf16 *__restrict__ A, int lda,
                                                        const __bf16 *__restrict__ B, int ldb,
                                                        const float *__restrict__ bias, const float *__restrict__ aux,
                                                        float *C, int ldc, size_t czs, __bf16 *Cb, int ldcb, int M,
                                                        int N, int K, int kchunk) {
    __shared__ __attribute__((aligned(16))) unsigned short As[kGT * kGLd];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[kGT * kGLd];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    uint4 ra[2], rb[2];
    gemm_fetch<AT>(A, lda, M, m0, kbeg, kend, t, ra);
    gemm_fetch<!BT>(B, ldb, N, n0, kbeg, kend, t, rb);
    const int kb = 8 * (lane >> 5);
    for (int k0 = kbeg; k0 < kend; k0 += kGK) {
        gemm_stash<AT>(As, t, ra);
        gemm_stash<!BT>(Bs, t, rb);
        __syncthreads();
        if (k0 + kGK < kend) {
            gemm_fetch<AT>(A, lda, M, m0, k0 + kGK, kend, t, ra);
            gemm_fetch<!BT>(B, ldb, N, n0, k0 + kGK, kend, t, rb);
        }
#pragma unroll
        for (int kk = 0; kk < kGK / 16; ++kk) {
            if (k0 + 16 * kk >= kend) break;
            const uint4 av = *(const uint4 *)(As + (wr + (lane & 31)) * kGLd + 16 * kk + kb);
            const uint4 bv = *(const uint4 *)(Bs + (wc + (lane & 31)) * kGLd + 16 * kk + kb);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                          __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int n = n0 + wc + (lane & 31);
    float csum = 0.0f;
    C += (size_t)blockIdx.z * czs;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + wr + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (m < M && n < N) {
            if (EPI == EPI_F32) {
                C[(size_t)m * ldc + n] = acc[i] + (bias ? bias[n] : 0.0f);
            } else if (EPI == EPI_SILU) {
                const float z = acc[i] + bias[n];
                C[(size_t)m * ldc + n] = z;
                Cb[(size_t)m * ldcb + n] = (__bf16)silu_f(z);
            } else {
                const float d = acc[i] * dsilu_f(aux[(size_t)m * ldc + n]);
                Cb[(size_t)m * ldcb + n] = (__bf16)d;
                csum += d;
            }
        }
    }
    if (EPI == EPI_DSILU) {
        csum += __shfl_xor(csum, 32, 64);
        const int mb = (m0 + wr) >> 5;
        if (lane < 32 && n < N && m0 + wr < M) C[(size_t)mb * ldc + n] = csum;
    }
}

// out[i] = sum over p < parts of in[p*stride + i], in order of p
__global__ void sum_parts_kernel(const float *__restrict__ in, int parts, size_t stride, size_t n, float *out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int p = 0; p < parts; ++p) s += in[(size_t)p * stride + i];
        out[i] = s;
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
// by 1/n for the batch mean), written as FP32 [n][29] and as BF16 rows of
// MLP_OUT_LD with zero padding.
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
        dout_b[(size_t)s * MLP_OUT_LD + j] = (__bf16)(g[j] * inv_n);
    }
#pragma unroll
    for (int j = 29; j < MLP_OUT_LD; ++j) dout_b[(size_t)s * MLP_OUT_LD + j] = (__bf16)0.0f;
    loss[s] = L;
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

// *out += (sum of x[0..n)) * scale, in FP64
__global__ void reduce_sum_kernel(const float *__restrict__ x, int n, double scale, double *out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += (double)red[0] * scale;
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

// C = A.B over the whole K range.  With `part` (room for kMlpSplit products
// of M x N) and a product too small to fill the chip, K is split over up to
// kMlpSplit workgroup layers whose partials are then summed in order.
static hipError_t mlp_gemm(bool at, bool bt, int epi, const __bf16 *A, int lda, const __bf16 *B, int ldb,
                           const float *bias, const float *aux, float *C, int ldc, __bf16 *Cb, int ldcb, int M, int N,
                           int K, float *part, hipStream_t s) {
    const int tiles = ((N + kGT - 1) / kGT) * ((M + kGT - 1) / kGT);
    int split = 1;
    if (part && epi == EPI_F32 && !bias && ldc == N && K >= 4 * kGK)
        split = std::max(1, std::min({kMlpSplit, 256 / tiles, K / (2 * kGK)}));
    const int kchunk = split > 1 ? ((K + split - 1) / split + kGK - 1) / kGK * kGK : K;
    split = (K + kchunk - 1) / kchunk;
    float *dst = split > 1 ? part : C;
    const int ldd = split > 1 ? N : ldc;
    const size_t czs = (size_t)M * N;
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, split), block(256);
#define VPMC_GEMM(AT_, BT_, E_)                                                                                   \
    hipLaunchKernelGGL((gemm_bf16_kernel<AT_, BT_, E_>), grid, block, 0, s, A, lda, B, ldb, bias, aux, dst, ldd, \
                       czs, Cb, ldcb, M, N, K, kchunk)
    if (!at && bt && epi == EPI_SILU) VPMC_GEMM(false, true, EPI_SILU);
    else if (!at && bt && epi == EPI_F32) VPMC_GEMM(false, true, EPI_F32);
    else if (!at && !bt && epi == EPI_DSILU) VPMC_GEMM(false, false, EPI_DSILU);
    else if (at && !bt && epi == EPI_F32) VPMC_GEMM(true, false, EPI_F32);
    else return hipErrorInvalidValue;
#undef VPMC_GEMM
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || split == 1) return e;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(czs)), dim3(256), 0, s, part, split, czs, czs, C);
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
        e = mlp_gemm(false, true, last ? EPI_F32 : EPI_SILU, in, ni, W, ni, bias, nullptr, last ? b.out : b.z[l], no,
                     last ? nullptr : b.h[l], no, n, no, ni, nullptr, s);
    }
    return e;
}

hipError_t mlp_loss_grad(const MlpBuffers &b, const float *y, const float *trans, int n, float *grad,
                         double *loss_acc, hipStream_t s) {
    hipError_t e = mlp_forward(b, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_head_kernel, dim3((n + 255) / 256), dim3(256), 0, s, b.out, y, trans, n, 1.0f / n,
                       b.dout, b.dout_b, b.loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, b.loss, n, 1.0 / n, loss_acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // backward through the layers; dZ of the current layer in BF16 (dcur, row
    // pitch ldd) and its bias gradient from FP32 values
    const __bf16 *dcur = b.dout_b;
    int ldd = MLP_OUT_LD;
    for (int l = MLP_LAYERS - 1; l >= 0; --l) {
        const int ni = kDims[l], no = kDims[l + 1];
        const __bf16 *in = l == 0 ? b.x : b.h[l - 1];
        float *gW = grad + mlp_param_offset(l), *gb = gW + no * ni;
        // dW = dZ^T . H_in   (M = no, N = ni, K = n)
        if ((e = mlp_gemm(true, false, EPI_F32, dcur, ldd, in, ni, nullptr, nullptr, gW, ni, nullptr, 0, no, ni, n,
                          b.wpart, s)) != hipSuccess)
            return e;
        if (l == MLP_LAYERS - 1)   // output layer: column sums of the FP32 dOUT
            hipLaunchKernelGGL(colsum_kernel, dim3(no), dim3(256), 0, s, b.dout, n, no, gb);
        else                       // 32-row partial sums left by the dZ epilogue
            hipLaunchKernelGGL(colsum_kernel, dim3(no), dim3(256), 0, s, b.bpart, (n + 31) / 32, no, gb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l == 0) break;
        // dZ_in = (dZ . W) * silu'(Z_in)   (M = n, N = ni, K = no)
        const __bf16 *W = b.wb + mlp_param_offset(l);
        __bf16 *dzb = (l & 1) ? b.dzb_a : b.dzb_b;
        if ((e = mlp_gemm(false, false, EPI_DSILU, dcur, ldd, W, ni, nullptr, b.z[l - 1], b.bpart, ni, dzb, ni, n,
                          ni, no, nullptr, s)) != hipSuccess)
            return e;
        dcur = dzb;
        ldd = ni;
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
