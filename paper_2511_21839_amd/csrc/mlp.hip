// Emittance surrogate on the matrix cores: a BF16 MFMA GEMM with fused
// epilogues for the forward pass with tangent columns, the Sobolev loss and
// its reverse sweep, and Adam. The C ABI is declared in include/dmlp.h.
//
// Layouts. Activations are column-major [columns][features] in BF16: sample
// s owns columns 16 s .. 16 s + 15 (value, 13 tangents, 2 zero columns), so
// a 16 x 16 MFMA result block holds 16 features of exactly one sample and
// the value column sits in the first lane of every 16-lane row group.
// Feature counts are padded to 32 at the input and output layers.
//
// Forward, layer l:   Z_l = W_l A_{l-1}  (+ b_l on value columns)
//   hidden:  A_l = silu(Z_l) on value columns, silu'(z_value) Z_l on tangents
//   output:  OUT = Z_5 (FP32)
// Backward, from Zbar_5 (the loss head):
//   Abar_{l-1} = W_l^T Zbar_l
//   Zbar_{l-1} = silu'(z) Abar on tangents; on values
//                silu'(z) Abar_v + silu''(z) sum_t Abar_t Z_t
//   Wbar_l = Zbar_l A_{l-1}^T (split over the columns), bbar_l = sum of value columns
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dmlp.h"

namespace dmlp {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NIN = DMLP_NIN, NOUT = DMLP_NOUT, H = DMLP_HIDDEN, NL = DMLP_LAYERS;
constexpr int CPS = 16;     // columns per sample
constexpr int FPAD = 32;    // padded input / output feature count
constexpr int BM = 128, BN = 128, BK = 32, LDS_LD = BK + 8;
constexpr int GEMM_THREADS = 256;

// layer l (0-based): in/out features, padded, and parameter offsets
constexpr int fin(int l) { return l == 0 ? NIN : H; }
constexpr int fout(int l) { return l == NL - 1 ? NOUT : H; }
constexpr int fin_pad(int l) { return l == 0 ? FPAD : H; }
constexpr int fout_pad(int l) { return l == NL - 1 ? FPAD : H; }
constexpr int64_t w_off(int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)fout(i) * fin(i) + fout(i);
    return o;
}
constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)fout(l) * fin(l); }
constexpr int64_t NPARAM = w_off(NL);
constexpr int64_t wpad_off(int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)fout_pad(i) * fin_pad(i);
    return o;
}
constexpr int64_t NWPAD = wpad_off(NL);

__device__ __forceinline__ float sig(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sig(z); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = sig(z);
    return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ float d2silu_f(float z) {
    const float s = sig(z);
    return s * (1.0f - s) * (2.0f + z * (1.0f - 2.0f * s));
}

// ---------------------------------------------------------------- GEMM
enum { AM_ROW = 0, AM_COL = 1 };  // A stored [M][K] or [K][M]
enum { BN_COL = 0, BN_ROW = 1 };  // B stored [N][K] or [K][N]
enum { EPI_SILU = 0, EPI_LINEAR = 1, EPI_BWD = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    const bf16* A;
    int64_t lda;
    const bf16* B;
    int64_t ldb;
    int M, N, K, ksplit;
    const float* bias;  // added to value columns of rows < nbias
    int nbias;
    bf16* out_bf;       // [N][ldo]
    int64_t ldo;
    float* out_f;       // [N][ldf]; EPI_PARTIAL: [split][N][ldf]
    int64_t ldf;
    const float* zin;   // EPI_BWD: stored Z of the layer, [N][ldz]
    int64_t ldz;
};

union V8 {
    uint4 u;
    bf16 h[8];
};

// C[M x N] = A[M x K] B[K x N] on one 128 x 128 tile per workgroup; four
// wavefronts of 64 x 64, each a 4 x 4 grid of 16 x 16 x 32 MFMAs per K step.
// M and N must be multiples of 16, K (per split) of 32.
template <int AM, int BMODE, int EPI>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm(GemmArgs g) {
    __shared__ __align__(16) bf16 As[BM * LDS_LD];  // [m][k]
    __shared__ __align__(16) bf16 Bs[BN * LDS_LD];  // [n][k]
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kb = blockIdx.z * g.ksplit;
    const int ke = kb + g.ksplit < g.K ? kb + g.ksplit : g.K;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = t + GEMM_THREADS * it;  // 512 chunks of 8 values per operand
            V8 v;
            v.u = make_uint4(0, 0, 0, 0);
            if (AM == AM_ROW) {
                const int r = idx >> 2, kc = (idx & 3) * 8;
                if (m0 + r < g.M) v.u = *reinterpret_cast<const uint4*>(g.A + (int64_t)(m0 + r) * g.lda + k0 + kc);
                *reinterpret_cast<uint4*>(&As[r * LDS_LD + kc]) = v.u;
            } else {
                const int kk = idx >> 4, mc = (idx & 15) * 8;
                if (m0 + mc < g.M) v.u = *reinterpret_cast<const uint4*>(g.A + (int64_t)(k0 + kk) * g.lda + m0 + mc);
#pragma unroll
                for (int j = 0; j < 8; ++j) As[(mc + j) * LDS_LD + kk] = v.h[j];
            }
            V8 w;
            w.u = make_uint4(0, 0, 0, 0);
            if (BMODE == BN_COL) {
                const int r = idx >> 2, kc = (idx & 3) * 8;
                if (n0 + r < g.N) w.u = *reinterpret_cast<const uint4*>(g.B + (int64_t)(n0 + r) * g.ldb + k0 + kc);
                *reinterpret_cast<uint4*>(&Bs[r * LDS_LD + kc]) = w.u;
            } else {
                const int kk = idx >> 4, nc = (idx & 15) * 8;
                if (n0 + nc < g.N) w.u = *reinterpret_cast<const uint4*>(g.B + (int64_t)(k0 + kk) * g.ldb + n0 + nc);
#pragma unroll
                for (int j = 0; j < 8; ++j) Bs[(nc + j) * LDS_LD + kk] = w.h[j];
            }
        }
        __syncthreads();
        bf16x8 af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * 64 + 16 * i + (lane & 15)) * LDS_LD + 8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * 64 + 16 * j + (lane & 15)) * LDS_LD + 8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // epilogue: lane holds rows mb .. mb + 3 of column n of every 16 x 16 block
    const int c = lane & 15;
    const int vsrc = lane & ~15;  // lane holding the value column of this row group
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mb = m0 + wm * 64 + 16 * i + 4 * (lane >> 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + 16 * j + c;
            const bool ok = mb < g.M && n < g.N;
            float z[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) z[r] = acc[i][j][r];
            if (EPI == EPI_PARTIAL) {
                if (ok) {
                    float* o = g.out_f + ((int64_t)blockIdx.z * g.N + n) * g.ldf + mb;
                    *reinterpret_cast<float4*>(o) = make_float4(z[0], z[1], z[2], z[3]);
                }
                continue;
            }
            if (EPI == EPI_SILU || EPI == EPI_LINEAR) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (c == 0 && mb + r < g.nbias) z[r] += g.bias[mb + r];
            }
            if (EPI == EPI_LINEAR) {
                if (ok) *reinterpret_cast<float4*>(g.out_f + (int64_t)n * g.ldf + mb) = make_float4(z[0], z[1], z[2], z[3]);
                continue;
            }
            float o[4];
            if (EPI == EPI_SILU) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float zv = __shfl(z[r], vsrc, 64);
                    o[r] = c == 0 ? silu_f(zv) : dsilu_f(zv) * z[r];
                }
                if (ok && g.out_f)
                    *reinterpret_cast<float4*>(g.out_f + (int64_t)n * g.ldf + mb) = make_float4(z[0], z[1], z[2], z[3]);
            } else {  // EPI_BWD: z holds Abar; the forward Z of this layer is stored
                float zl[4] = {0.f, 0.f, 0.f, 0.f}, zv[4] = {0.f, 0.f, 0.f, 0.f};
                if (ok) {
                    const float4 a = *reinterpret_cast<const float4*>(g.zin + (int64_t)n * g.ldz + mb);
                    const float4 b = *reinterpret_cast<const float4*>(g.zin + (int64_t)(n - c) * g.ldz + mb);
                    zl[0] = a.x; zl[1] = a.y; zl[2] = a.z; zl[3] = a.w;
                    zv[0] = b.x; zv[1] = b.y; zv[2] = b.z; zv[3] = b.w;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float av = __shfl(z[r], vsrc, 64);
                    float s = c == 0 ? 0.f : z[r] * zl[r];
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
                    o[r] = c == 0 ? dsilu_f(zv[r]) * av + d2silu_f(zv[r]) * s : dsilu_f(zv[r]) * z[r];
                }
            }
            if (ok) {
                V8 pk;
#pragma unroll
                for (int r = 0; r < 4; ++r) pk.h[r] = (bf16)o[r];
                *reinterpret_cast<uint2*>(g.out_bf + (int64_t)n * g.ldo + mb) = make_uint2(pk.u.x, pk.u.y);
            }
        }
    }
}

template <int AM, int BMODE, int EPI>
static hipError_t gemm(const GemmArgs& g, int splits, hipStream_t s) {
    if (g.M % 16 || g.N % 16 || g.K % BK || g.ksplit % BK) return hipErrorInvalidValue;
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, splits);
    hipLaunchKernelGGL((k_gemm<AM, BMODE, EPI>), grid, dim3(GEMM_THREADS), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- small kernels
struct Norm {
    double ic[NIN], is[NIN], oc[NOUT], os[NOUT];
};

// x [n][13] -> X0 [16 npad][32]: value column u = (x - ic) / is, tangent
// column 1 + t the unit vector e_t, zero padding (and zero padded samples)
__global__ void k_pack_inputs(const double* __restrict__ x, int n, int npad, Norm nm, bf16* __restrict__ X0) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)npad * CPS * FPAD) return;
    const int f = (int)(gid % FPAD);
    const int64_t col = gid / FPAD;
    const int s = (int)(col / CPS), c = (int)(col % CPS);
    float v = 0.f;
    if (s < n && f < NIN) {
        if (c == 0)
            v = (float)((x[(int64_t)s * NIN + f] - nm.ic[f]) / nm.is[f]);
        else if (c == 1 + f)
            v = 1.f;
    }
    X0[gid] = (bf16)v;
}

// Sobolev loss head: Zbar_5 [16 npad][32] (BF16) and per-block loss sums.
constexpr int HEAD_THREADS = 256;
__global__ __launch_bounds__(HEAD_THREADS) void k_loss_head(const float* __restrict__ out, int n, int npad, Norm nm,
                                                            const double* __restrict__ eps, const double* __restrict__ jac,
                                                            float wv, float wj, bf16* __restrict__ zbar,
                                                            float* __restrict__ part) {
    __shared__ float red[HEAD_THREADS];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (s < npad) {
        bf16* zb = zbar + (int64_t)s * CPS * FPAD;
        for (int i = 0; i < CPS * FPAD; ++i) zb[i] = (bf16)0.f;
        if (s < n) {
            const float* o = out + (int64_t)s * CPS * FPAD;
            const float inv = 1.0f / (float)n;
#pragma unroll
            for (int k = 0; k < NOUT; ++k) {
                const float y = (float)((eps[(int64_t)s * NOUT + k] - nm.oc[k]) / nm.os[k]);
                const float d = o[k] - y;
                l += wv * d * d;
                zb[k] = (bf16)(2.f * wv * d * inv);
                for (int t = 0; t < NIN; ++t) {
                    const float G = (float)(jac[((int64_t)s * NOUT + k) * NIN + t] * nm.is[t] / nm.os[k]);
                    const float e = o[(1 + t) * FPAD + k] - G;
                    l += wj * e * e;
                    zb[(1 + t) * FPAD + k] = (bf16)(2.f * wj * e * inv);
                }
            }
            l *= inv;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int off = HEAD_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum(const float* __restrict__ part, int m, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Wbar [fo][fi] (packed, row-major) = sum over splits of P[split][n][m] (n < fi, m < fo)
__global__ void k_reduce_wgrad(const float* __restrict__ P, int splits, int ldn, int ldm, int fo, int fi,
                               float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= fo * fi) return;
    const int m = i / fi, nn = i % fi;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += P[((int64_t)k * ldn + nn) * ldm + m];
    grad[i] = s;
}

// bbar[m] = sum over samples of Zbar[16 s][m]; grid.y splits the samples, atomics join them
__global__ void k_bias_grad(const bf16* __restrict__ zbar, int ld, int fo, int npad, float* __restrict__ grad) {
    const int m = threadIdx.x;
    if (m >= fo) return;
    const int per = (npad + gridDim.x - 1) / gridDim.x;
    const int s0 = blockIdx.x * per, s1 = s0 + per < npad ? s0 + per : npad;
    float s = 0.f;
    for (int q = s0; q < s1; ++q) s += (float)zbar[(int64_t)q * CPS * ld + m];
    atomicAdd(grad + m, s);
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// BF16 copies of the weights, zero-padded to [fout_pad][fin_pad] per layer
struct LayerTab {
    int64_t w[NL], wp[NL];
    int fo[NL], fi[NL], fop[NL], fip[NL];
};

__global__ void k_weights_bf16(const float* __restrict__ p, LayerTab tb, bf16* __restrict__ wb) {
    const int l = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)tb.fop[l] * tb.fip[l]) return;
    const int m = (int)(i / tb.fip[l]), k = (int)(i % tb.fip[l]);
    const float v = (m < tb.fo[l] && k < tb.fi[l]) ? p[tb.w[l] + (int64_t)m * tb.fi[l] + k] : 0.f;
    wb[tb.wp[l] + i] = (bf16)v;
}

// ---------------------------------------------------------------- fused inference
// One workgroup carries FT_COLS columns (FT_COLS / 16 samples) through the
// whole network with its activations in LDS. Per layer, Z = W A with the
// weights streamed from L2 in BK-wide chunks (double-buffered in LDS) and
// the accumulators in registers; the epilogue then writes the next layer's
// activations over the current ones. The MFMA sequence and the epilogue
// arithmetic are those of the layer-by-layer GEMM, and the outputs go
// straight to eps and the Jacobian (the unpack formulas).
constexpr int FT_COLS = 128;
constexpr int FT_LD = H + 8;  // activation row stride (BF16)
constexpr int FT_THREADS = 256;

// Weight fragments of one layer for this wave: rows r0 + 16 i + (lane & 15)
// (i < NI), k = BK ks + 8 (lane >> 4) (ks < KS), in MFMA A-operand order.
template <int KS, int NI>
__device__ __forceinline__ void ft_load_w(const bf16* __restrict__ W, int K, int r0, bf16x8 (&wa)[8][4]) {
    const int lane = threadIdx.x & 63;
    const bf16* wrow = W + (int64_t)(r0 + (lane & 15)) * K + 8 * (lane >> 4);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int i = 0; i < NI; ++i) wa[ks][i] = *reinterpret_cast<const bf16x8*>(wrow + (int64_t)16 * i * K + ks * BK);
}

// fragment ks of rows r0 + 16 i + (lane & 15), i < NI, of a [rows][K] matrix
template <int NI>
__device__ __forceinline__ void ft_load_frag(const bf16* __restrict__ W, int K, int r0, int ks, bf16x8 (&wa)[8][4]) {
    const int lane = threadIdx.x & 63;
    const bf16* wrow = W + (int64_t)(r0 + (lane & 15)) * K + 8 * (lane >> 4) + ks * BK;
#pragma unroll
    for (int i = 0; i < NI; ++i) wa[ks][i] = *reinterpret_cast<const bf16x8*>(wrow + (int64_t)16 * i * K);
}

// bias of this lane's rows r0 + 16 i + 4 (lane >> 4) + r
__device__ __forceinline__ void ft_load_b(const float* __restrict__ bias, int r0, float (&bv)[4][4]) {
    const int q = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[i][r] = bias[r0 + 16 * i + 4 * q + r];
}

// The next layer a hidden layer prefetches into its weight registers.
struct FtNext {
    const bf16* W;      // weights [rows][K]
    const float* bias;  // nullptr for the output layer (its bias is read at the end)
    int K, r0;          // inputs, this wave's first row
};

// One hidden layer of a fused tile (K inputs): wave owns rows 64 wave .. + 63
// and all 8 column blocks, with its weight fragments in registers, so the K
// loop reads only LDS activations (double-buffered per K step), with no
// weight staging and no barrier per K step. As soon as K step ks has issued
// its MFMAs, fragment ks of the next layer (KSN steps of NNI row blocks) is
// loaded into the same registers; the next biases load during the epilogue.
// Epilogue: silu on value columns, silu'(z_value) z on tangents. Only the
// value column's 16 rows per block are distinct arguments, so the wave
// writes its 512 of them to its LDS scratch `vs` ([2][512]), each lane
// evaluates 8 (silu into vs[0], silu' into vs[1]) and every lane reads its
// rows back: 8 sigmoid evaluations per lane, not 128.
template <int K, int KSN, int NNI>
__device__ __forceinline__ void ft_hidden(bf16x8 (&wa)[8][4], float (&bv)[4][4], FtNext nx, bf16* __restrict__ act,
                                          float* __restrict__ vs) {
    constexpr int KS = K / BK;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, q = lane >> 4;
    __syncthreads();  // the layer's input is in act
    floatx4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 bfr[2][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bfr[0][j] = *reinterpret_cast<const bf16x8*>(&act[(16 * j + c) * FT_LD + 8 * q]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                bfr[(ks + 1) & 1][j] =
                    *reinterpret_cast<const bf16x8*>(&act[(16 * j + c) * FT_LD + (ks + 1) * BK + 8 * q]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks][i], bfr[ks & 1][j], acc[i][j], 0, 0, 0);
        if (ks < KSN) ft_load_frag<NNI>(nx.W, nx.K, nx.r0, ks, wa);  // step ks is done with these registers
    }
#pragma unroll
    for (int ks = KS; ks < KSN; ++ks) ft_load_frag<NNI>(nx.W, nx.K, nx.r0, ks, wa);
    float* __restrict__ vz = vs;        // value-column pre-activations, then silu
    float* __restrict__ vd = vs + 512;  // silu'
    if (c == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                *reinterpret_cast<float4*>(&vz[(i * 8 + j) * 16 + 4 * q]) =
                    make_float4(acc[i][j][0] + bv[i][0], acc[i][j][1] + bv[i][1], acc[i][j][2] + bv[i][2],
                                acc[i][j][3] + bv[i][3]);
    }
    if (nx.bias) ft_load_b(nx.bias, nx.r0, bv);
    __syncthreads();  // every read of act is done; the scratch is written
    {
        const float4 z0 = *reinterpret_cast<const float4*>(&vz[lane * 8]);
        const float4 z1 = *reinterpret_cast<const float4*>(&vz[lane * 8 + 4]);
        const float z[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
        float sv[8], dv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            dv[k] = dsilu_f(z[k]);
            sv[k] = silu_f(z[k]);
        }
        *reinterpret_cast<float4*>(&vd[lane * 8]) = make_float4(dv[0], dv[1], dv[2], dv[3]);
        *reinterpret_cast<float4*>(&vd[lane * 8 + 4]) = make_float4(dv[4], dv[5], dv[6], dv[7]);
        *reinterpret_cast<float4*>(&vz[lane * 8]) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        *reinterpret_cast<float4*>(&vz[lane * 8 + 4]) = make_float4(sv[4], sv[5], sv[6], sv[7]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mb = wave * 64 + 16 * i + 4 * q;
        // this row block's factors for all 8 column blocks first, then the writes
        float4 sv[8], dv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sv[j] = *reinterpret_cast<const float4*>(&vz[(i * 8 + j) * 16 + 4 * q]);
            dv[j] = *reinterpret_cast<const float4*>(&vd[(i * 8 + j) * 16 + 4 * q]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float sa[4] = {sv[j].x, sv[j].y, sv[j].z, sv[j].w}, da[4] = {dv[j].x, dv[j].y, dv[j].z, dv[j].w};
            V8 pk;
#pragma unroll
            for (int r = 0; r < 4; ++r) pk.h[r] = (bf16)(c == 0 ? sa[r] : da[r] * acc[i][j][r]);
            *reinterpret_cast<uint2*>(&act[(16 * j + c) * FT_LD + mb]) = make_uint2(pk.u.x, pk.u.y);
        }
    }
}

// The output layer (FPAD padded rows, NOUT real): row block wave & 1 (its
// weight fragments in wa[ks][0]), column blocks 4 (wave >> 1) + j; rows 0, 1
// go to eps (value column) and the Jacobian (tangent columns).
__device__ __forceinline__ void ft_output(const bf16x8 (&wa)[8][4], const float* __restrict__ bias, const bf16* act,
                                          int s0, int n, const Norm& nm, double* __restrict__ eps,
                                          double* __restrict__ jac) {
    constexpr int KS = H / BK;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, q = lane >> 4;
    __syncthreads();  // the last hidden layer's output is in act
    floatx4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8 bfr =
                *reinterpret_cast<const bf16x8*>(&act[(16 * (4 * (wave >> 1) + j) + c) * FT_LD + ks * BK + 8 * q]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks][0], bfr, acc[j], 0, 0, 0);
        }
    if ((wave & 1) != 0 || q != 0) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int s = s0 + 4 * (wave >> 1) + j;
        if (s >= n) continue;
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
            float z = acc[j][k];
            if (c == 0) {
                z += bias[k];
                eps[(int64_t)s * NOUT + k] = nm.oc[k] + nm.os[k] * (double)z;
            } else if (jac && c <= NIN) {
                jac[((int64_t)s * NOUT + k) * NIN + c - 1] = nm.os[k] * (double)z / nm.is[c - 1];
            }
        }
    }
}

__global__ __launch_bounds__(FT_THREADS) void k_mlp_infer(const double* __restrict__ x, int n, Norm nm,
                                                          const bf16* __restrict__ wb, const float* __restrict__ params,
                                                          LayerTab tb, double* __restrict__ eps,
                                                          double* __restrict__ jac) {
    static_assert(NL == 5, "the layer sequence below is written out for 4 hidden layers");
    __shared__ __align__(16) bf16 act[FT_COLS * FT_LD];             // [column][feature]
    __shared__ __align__(16) float vsc[FT_THREADS / 64][2 * 512];  // per-wave epilogue scratch
    const int s0 = blockIdx.x * (FT_COLS / CPS);
    const int wave = threadIdx.x >> 6;
    auto bias = [&](int l) { return params + tb.w[l] + (int64_t)tb.fo[l] * tb.fi[l]; };
    bf16x8 wa[8][4];
    float bv[4][4];
    ft_load_w<FPAD / BK, 4>(wb + tb.wp[0], FPAD, 64 * wave, wa);
    ft_load_b(bias(0), 64 * wave, bv);
    // layer-0 input: value column u = (x - ic) / is, tangent column 1 + f the unit vector
    for (int i = threadIdx.x; i < FT_COLS * FPAD; i += FT_THREADS) {
        const int col = i / FPAD, f = i % FPAD, s = s0 + col / CPS, cc = col % CPS;
        float v = 0.f;
        if (s < n && f < NIN) {
            if (cc == 0)
                v = (float)((x[(int64_t)s * NIN + f] - nm.ic[f]) / nm.is[f]);
            else if (cc == 1 + f)
                v = 1.f;
        }
        act[col * FT_LD + f] = (bf16)v;
    }
    float* vs = vsc[wave];
    // each layer loads the next one's weights and biases while its epilogue runs
    ft_hidden<FPAD, H / BK, 4>(wa, bv, FtNext{wb + tb.wp[1], bias(1), H, 64 * wave}, act, vs);
    ft_hidden<H, H / BK, 4>(wa, bv, FtNext{wb + tb.wp[2], bias(2), H, 64 * wave}, act, vs);
    ft_hidden<H, H / BK, 4>(wa, bv, FtNext{wb + tb.wp[3], bias(3), H, 64 * wave}, act, vs);
    ft_hidden<H, H / BK, 1>(wa, bv, FtNext{wb + tb.wp[4], nullptr, H, 16 * (wave & 1)}, act, vs);
    ft_output(wa, bias(4), act, s0, n, nm, eps, jac);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

}  // namespace dmlp

// ---------------------------------------------------------------- context
struct dmlp_ctx {
    int nmax = 0, npmax = 0;
    hipStream_t stream = nullptr;
    std::string err;
    dmlp::Norm norm{};
    bool norm_set = false, params_set = false;
    double b1 = 0.9, b2 = 0.999, aeps = 1e-8;
    int64_t adam_t = 0;
    int splits = 1;
    // workspace
    float *params = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    dmlp::bf16* wb = nullptr;
    dmlp::bf16* X0 = nullptr;
    dmlp::bf16* A[dmlp::NL - 1] = {};
    float* Z[dmlp::NL - 1] = {};
    float* out = nullptr;
    dmlp::bf16* zb5 = nullptr;
    dmlp::bf16* zb[2] = {};
    float* part = nullptr;
    float* lpart = nullptr;
    double* loss = nullptr;
};

namespace {

using namespace dmlp;

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
int npad_of(int n) { return (n + 7) / 8 * 8; }  // whole 128-column tiles
constexpr int WSPLITS = 128;                    // column splits of the weight-gradient products
constexpr int HEAD_BLOCKS_MAX = 65536;

int fail(dmlp_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail((c), DPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t layout(int nmax, char* base, dmlp_ctx* c) {
    const size_t np = (size_t)npad_of(nmax);
    const size_t ncol = np * CPS;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return base ? base + o : nullptr;
    };
    dmlp_ctx t;
    t.params = (float*)take(NPARAM * 4);
    t.grad = (float*)take(NPARAM * 4);
    t.m1 = (float*)take(NPARAM * 4);
    t.m2 = (float*)take(NPARAM * 4);
    t.wb = (bf16*)take(NWPAD * 2);
    t.X0 = (bf16*)take(ncol * FPAD * 2);
    for (int l = 0; l < NL - 1; ++l) t.A[l] = (bf16*)take(ncol * H * 2);
    for (int l = 0; l < NL - 1; ++l) t.Z[l] = (float*)take(ncol * H * 4);
    t.out = (float*)take(ncol * FPAD * 4);
    t.zb5 = (bf16*)take(ncol * FPAD * 2);
    t.zb[0] = (bf16*)take(ncol * H * 2);
    t.zb[1] = (bf16*)take(ncol * H * 2);
    t.part = (float*)take((size_t)WSPLITS * H * H * 4);
    t.lpart = (float*)take((size_t)HEAD_BLOCKS_MAX * 4);
    t.loss = (double*)take(8);
    if (c) {
        c->params = t.params; c->grad = t.grad; c->m1 = t.m1; c->m2 = t.m2; c->wb = t.wb; c->X0 = t.X0;
        for (int l = 0; l < NL - 1; ++l) { c->A[l] = t.A[l]; c->Z[l] = t.Z[l]; }
        c->out = t.out; c->zb5 = t.zb5; c->zb[0] = t.zb[0]; c->zb[1] = t.zb[1];
        c->part = t.part; c->lpart = t.lpart; c->loss = t.loss;
    }
    return off;
}

LayerTab layer_tab() {
    LayerTab tb;
    for (int l = 0; l < NL; ++l) {
        tb.w[l] = w_off(l);
        tb.wp[l] = wpad_off(l);
        tb.fo[l] = fout(l);
        tb.fi[l] = fin(l);
        tb.fop[l] = fout_pad(l);
        tb.fip[l] = fin_pad(l);
    }
    return tb;
}

hipError_t sync_weights(dmlp_ctx* c) {
    const int64_t maxn = (int64_t)H * H;
    hipLaunchKernelGGL(k_weights_bf16, dim3((unsigned)((maxn + 255) / 256), NL), dim3(256), 0, c->stream, c->params,
                       layer_tab(), c->wb);
    return hipGetLastError();
}

// Forward over npad samples (columns 16 npad); keep Z for the backward when train.
hipError_t forward(dmlp_ctx* c, int n, const double* x, bool train) {
    const int np = npad_of(n);
    const int ncol = np * CPS;
    const int64_t tot = (int64_t)ncol * FPAD;
    hipLaunchKernelGGL(k_pack_inputs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, x, n, np, c->norm,
                       c->X0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bf16* in = c->X0;
    int ldin = FPAD;
    for (int l = 0; l < NL; ++l) {
        GemmArgs g{};
        g.A = c->wb + wpad_off(l);
        g.lda = fin_pad(l);
        g.B = in;
        g.ldb = ldin;
        g.M = fout_pad(l);
        g.N = ncol;
        g.K = fin_pad(l);
        g.ksplit = g.K;
        g.bias = c->params + b_off(l);
        g.nbias = fout(l);
        if (l < NL - 1) {
            g.out_bf = c->A[l];
            g.ldo = H;
            g.out_f = train ? c->Z[l] : nullptr;
            g.ldf = H;
            if ((e = gemm<AM_ROW, BN_COL, EPI_SILU>(g, 1, c->stream)) != hipSuccess) return e;
            in = c->A[l];
            ldin = H;
        } else {
            g.out_f = c->out;
            g.ldf = FPAD;
            if ((e = gemm<AM_ROW, BN_COL, EPI_LINEAR>(g, 1, c->stream)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Wbar_l and bbar_l from Zbar_l [ncol][ldz] and A_{l-1} [ncol][ldi]
hipError_t weight_grad(dmlp_ctx* c, int l, const bf16* zbar, int ldz, const bf16* ain, int ldi, int np) {
    const int ncol = np * CPS;
    GemmArgs g{};
    g.A = zbar;  // A-op (m, k) = Zbar[k][m]
    g.lda = ldz;
    g.B = ain;  // B-op (k, n) = A[k][n]
    g.ldb = ldi;
    g.M = fout_pad(l);
    g.N = fin_pad(l);
    g.K = ncol;
    int ks = (ncol + WSPLITS - 1) / WSPLITS;
    ks = (ks + BK - 1) / BK * BK;
    g.ksplit = ks;
    const int splits = (ncol + ks - 1) / ks;
    g.out_f = c->part;
    g.ldf = g.M;
    hipError_t e = gemm<AM_COL, BN_ROW, EPI_PARTIAL>(g, splits, c->stream);
    if (e != hipSuccess) return e;
    const int nw = fout(l) * fin(l);
    hipLaunchKernelGGL(k_reduce_wgrad, dim3((nw + 255) / 256), dim3(256), 0, c->stream, c->part, splits, g.N, g.M,
                       fout(l), fin(l), c->grad + w_off(l));
    hipLaunchKernelGGL(k_bias_grad, dim3(64), dim3(256), 0, c->stream, zbar, ldz, fout(l), np, c->grad + b_off(l));
    return hipGetLastError();
}

// loss head and the full reverse sweep into c->grad (zeroed biases first)
hipError_t backward(dmlp_ctx* c, int n, const double* eps, const double* jac, double wv, double wj) {
    const int np = npad_of(n);
    const int ncol = np * CPS;
    hipError_t e;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, c->stream, c->grad, NPARAM, 0.f);
    const int hb = (np + HEAD_THREADS - 1) / HEAD_THREADS;
    hipLaunchKernelGGL(k_loss_head, dim3(hb), dim3(HEAD_THREADS), 0, c->stream, c->out, n, np, c->norm, eps, jac,
                       (float)wv, (float)wj, c->zb5, c->lpart);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, c->stream, c->lpart, hb, c->loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const bf16* zcur = c->zb5;
    int ldzc = FPAD;
    for (int l = NL - 1; l >= 0; --l) {
        const bf16* ain = l == 0 ? c->X0 : c->A[l - 1];
        const int ldi = l == 0 ? FPAD : H;
        if ((e = weight_grad(c, l, zcur, ldzc, ain, ldi, np)) != hipSuccess) return e;
        if (l == 0) break;
        // Abar_{l-1} = W_l^T Zbar_l, epilogue -> Zbar_{l-1}
        GemmArgs g{};
        g.A = c->wb + wpad_off(l);  // A-op (m = in, k = out) = W[out][in]
        g.lda = fin_pad(l);
        g.B = zcur;  // B-op (k = out, n = col) = Zbar[col][out]
        g.ldb = ldzc;
        g.M = fin_pad(l);
        g.N = ncol;
        g.K = fout_pad(l);
        g.ksplit = g.K;
        bf16* znext = c->zb[l & 1];
        g.out_bf = znext;
        g.ldo = H;
        g.zin = c->Z[l - 1];
        g.ldz = H;
        if ((e = gemm<AM_COL, BN_COL, EPI_BWD>(g, 1, c->stream)) != hipSuccess) return e;
        zcur = znext;
        ldzc = H;
    }
    return hipSuccess;
}

int check_batch(dmlp_ctx* c, int n) {
    if (n < 1 || n > c->nmax) return fail(c, DPIC_EINVAL, "batch of %d samples outside 1..%d", n, c->nmax);
    if (!c->norm_set || !c->params_set) return fail(c, DPIC_ESTATE, "set the normalisation and the parameters first");
    if ((npad_of(n) + HEAD_THREADS - 1) / HEAD_THREADS > HEAD_BLOCKS_MAX) return fail(c, DPIC_EINVAL, "batch too large");
    return DPIC_OK;
}

}  // namespace

extern "C" {

int dmlp_param_count(void) { return (int)NPARAM; }

int dmlp_query_workspace(int nmax, size_t* bytes) {
    if (nmax < 1 || nmax > (1 << 22) || !bytes) return DPIC_EINVAL;
    *bytes = layout(nmax, nullptr, nullptr);
    return DPIC_OK;
}

int dmlp_create(int nmax, void* ws, size_t bytes, void* stream, dmlp_ctx** out) {
    if (nmax < 1 || nmax > (1 << 22) || !ws || !out) return DPIC_EINVAL;
    if ((uintptr_t)ws % ALIGN) return DPIC_EINVAL;
    if (bytes < layout(nmax, nullptr, nullptr)) return DPIC_EINVAL;
    dmlp_ctx* c = new (std::nothrow) dmlp_ctx();
    if (!c) return DPIC_EINVAL;
    c->nmax = nmax;
    c->npmax = npad_of(nmax);
    c->stream = (hipStream_t)stream;
    layout(nmax, (char*)ws, c);
    *out = c;
    return DPIC_OK;
}

int dmlp_destroy(dmlp_ctx* c) {
    if (!c) return DPIC_EINVAL;
    delete c;
    return DPIC_OK;
}

int dmlp_last_error(const dmlp_ctx* c, char* buf, size_t len) {
    if (!c || !buf || !len) return DPIC_EINVAL;
    snprintf(buf, len, "%s", c->err.c_str());
    return DPIC_OK;
}

int dmlp_set_normalization(dmlp_ctx* c, const double* ic, const double* is, const double* oc, const double* os) {
    if (!c || !ic || !is || !oc || !os) return DPIC_EINVAL;
    for (int i = 0; i < NIN; ++i) {
        if (!isfinite(ic[i]) || !(is[i] > 0) || !isfinite(is[i])) return fail(c, DPIC_EINVAL, "input %d: bad center/scale", i);
        c->norm.ic[i] = ic[i];
        c->norm.is[i] = is[i];
    }
    for (int k = 0; k < NOUT; ++k) {
        if (!isfinite(oc[k]) || !(os[k] > 0) || !isfinite(os[k])) return fail(c, DPIC_EINVAL, "output %d: bad center/scale", k);
        c->norm.oc[k] = oc[k];
        c->norm.os[k] = os[k];
    }
    c->norm_set = true;
    return DPIC_OK;
}

int dmlp_set_params(dmlp_ctx* c, const float* p) {
    if (!c || !p) return DPIC_EINVAL;
    for (int64_t i = 0; i < NPARAM; ++i)
        if (!isfinite(p[i])) return fail(c, DPIC_EINVAL, "parameter %lld not finite", (long long)i);
    HIPCHK(c, hipMemcpyAsync(c->params, p, NPARAM * 4, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, c->stream, c->m1, NPARAM, 0.f);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, c->stream, c->m2, NPARAM, 0.f);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, sync_weights(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    c->params_set = true;
    return DPIC_OK;
}

int dmlp_get_params(dmlp_ctx* c, float* p) {
    if (!c || !p) return DPIC_EINVAL;
    HIPCHK(c, hipMemcpyAsync(p, c->params, NPARAM * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

int dmlp_predict(dmlp_ctx* c, int n, const double* x, double* eps, double* jac) {
    if (!c || !x || !eps) return DPIC_EINVAL;
    int r = check_batch(c, n);
    if (r != DPIC_OK) return r;
    const int tiles = npad_of(n) * CPS / FT_COLS;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)tiles), dim3(FT_THREADS), 0, c->stream, x, n, c->norm, c->wb,
                       c->params, layer_tab(), eps, jac);
    HIPCHK(c, hipGetLastError());
    return DPIC_OK;
}

int dmlp_loss_grad(dmlp_ctx* c, int n, const double* x, const double* eps, const double* jac, double wv, double wj,
                   double* loss, float* grad) {
    if (!c || !x || !eps || !jac) return DPIC_EINVAL;
    int r = check_batch(c, n);
    if (r != DPIC_OK) return r;
    if (!isfinite(wv) || !isfinite(wj) || wv < 0 || wj < 0) return fail(c, DPIC_EINVAL, "loss weights must be >= 0");
    HIPCHK(c, forward(c, n, x, true));
    HIPCHK(c, backward(c, n, eps, jac, wv, wj));
    if (loss) HIPCHK(c, hipMemcpyAsync(loss, c->loss, 8, hipMemcpyDeviceToHost, c->stream));
    if (grad) HIPCHK(c, hipMemcpyAsync(grad, c->grad, NPARAM * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

int dmlp_train_step(dmlp_ctx* c, int n, const double* x, const double* eps, const double* jac, double wv, double wj,
                    double lr) {
    if (!c || !x || !eps || !jac) return DPIC_EINVAL;
    int r = check_batch(c, n);
    if (r != DPIC_OK) return r;
    if (!isfinite(wv) || !isfinite(wj) || wv < 0 || wj < 0 || !(lr > 0))
        return fail(c, DPIC_EINVAL, "loss weights must be >= 0 and lr > 0");
    HIPCHK(c, forward(c, n, x, true));
    HIPCHK(c, backward(c, n, eps, jac, wv, wj));
    c->adam_t += 1;
    const float c1 = (float)(1.0 - pow(c->b1, (double)c->adam_t)), c2 = (float)(1.0 - pow(c->b2, (double)c->adam_t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, c->stream, c->params, c->grad,
                       c->m1, c->m2, NPARAM, (float)lr, (float)c->b1, (float)c->b2, (float)c->aeps, c1, c2);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, sync_weights(c));
    return DPIC_OK;
}

int dmlp_set_adam(dmlp_ctx* c, double b1, double b2, double eps) {
    if (!c) return DPIC_EINVAL;
    if (!(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0)) return fail(c, DPIC_EINVAL, "bad Adam constants");
    c->b1 = b1;
    c->b2 = b2;
    c->aeps = eps;
    return DPIC_OK;
}

int dmlp_read_loss(dmlp_ctx* c, double* loss) {
    if (!c || !loss) return DPIC_EINVAL;
    HIPCHK(c, hipMemcpyAsync(loss, c->loss, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

}  // extern "C"
