// Open-boundary Poisson solve by Hockney's method on the doubled grid, and
// the central-difference field (Sec. 4: potential from the charge, field by
// central finite differences; here with open boundaries instead of the
// paper's conducting pipe).
//
// phi(i) = sum_j rho(j) G(i - j) for node indices i in -1..n (one exact ghost
// ring), j in 0..n-1. With rho zero-padded to M = 2n per dimension and G
// tabulated at offsets o = i (i <= n) or i - M (i > n), the circular
// convolution on the M^3 grid equals the aperiodic sum for those targets.
// G is even, so its transform Ghat is real; it is stored on the
// (n+1)^3 octant, [ky][kx][kz] with kz fastest, with the 1/(Mx My Mz)
// normalisation folded in.
//
// Channels: the NC real channels of a dual grid array are packed pairwise
// into NCC = NC/2 complex channels (c, c + NCC); since Ghat is real each
// complex channel carries two independent real convolutions.
//
// Passes (complex arrays, x fastest, NCC channels innermost):
//   1  rows:  rho[nz][ny][nx][NC]  -> A[nz][ny][Mx][NCC]  (x forward, clears rho)
//   2  cols:  A -> B[nz][My][Mx][NCC]                       (y forward)
//   3  cols:  B -> C[nz+2][My][Mx][NCC]                     (z forward, x Ghat, z inverse)
//   4  cols:  C -> D[nz+2][ny+2][Mx][NCC]                   (y inverse)
//   5  rows:  D -> phi[nz+2][ny+2][nx+2][NC]                 (x inverse)
// Forward transforms read only the n nonzero inputs; inverse transforms write
// only the n+2 outputs needed (positions M-1, 0, .., n).
//
// Every pass runs its M-point transforms as two register stages with one
// LDS exchange between them (ColCfg below); the x passes treat channel j of
// a row, its values interleaved with the row's other channels, as a column.
#include "context.hpp"

namespace dpic {

// ---------------------------------------------------------------- passes 2-4
struct ColArgs {
    int W;            // columns per outer index
    int64_t bstride;  // element stride between neighbouring columns
    int64_t in_outer, in_stride;
    int n_in;         // nonzero input rows
    int64_t out_outer, out_stride;
    int n_out;        // output rows; row t holds transform row (t - out_shift) mod M
    int out_shift;
    int64_t in_batch, out_batch;  // strides between settings (grid dimension y)
    // Ghat multiply (mode 1): column w is (kx = w / ncc), outer index is ky
    const double* ghat;
    int ncc, gnx1, Mx, My;
};

// Column transforms (passes 2-4 and the Green's function) as two register
// stages: M = R1 R2, n = R2 n1 + n2, k = k1 + R1 k2,
//   X[k1 + R1 k2] = sum_n2 W_M^(n2 k1) W_R2^(n2 k2) sum_n1 x[R2 n1 + n2] W_R1^(n1 k1).
// A thread owns one column b and one n2 (stage A, an R1-point DFT on values
// loaded straight from global memory), then R1/R2 groups k1 (stage B, R2-point
// DFTs) after one LDS exchange. The inverse runs the same split transposed:
// per k1 over k2 first (the groups a thread holds after a forward), then per
// n2 over k1 after one exchange, x[n2 + R2 n1] = sum_k1 W_R1^(-n1 k1) W_M^(-n2 k1)
// sum_k2 X[k1 + R1 k2] W_R2^(-n2 k2). Forward-Ghat-inverse therefore needs
// two exchanges and no global round trip in between.
template <int M>
struct ColCfg {
    static constexpr int R1 = M >= 128 ? 16 : (M >= 32 ? 8 : 4);
    static constexpr int R2 = M / R1;
    static constexpr int NG = R1 / R2;    // stage-B groups per thread
    static constexpr int BC = (M >= 128 ? 4096 : 2048) / M;   // columns per block
    static constexpr int NT = BC * R2;    // threads per block
};

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }
constexpr int bitrev(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r = (r << 1) | ((i >> b) & 1);
    return r;
}

// cos and sin of 2 pi j / 16: the twiddles inside the register DFTs (R <= 16)
// are compile-time constants, so they cost neither LDS reads nor registers.
struct Tw16 {
    static constexpr double c[16] = {1.0,  0.9238795325112867,  0.7071067811865476,  0.3826834323650898,
                                     0.0,  -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
                                     -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898,
                                     0.0,  0.3826834323650898,  0.7071067811865476,  0.9238795325112867};
    static constexpr double s[16] = {0.0,  0.3826834323650898,  0.7071067811865476,  0.9238795325112867,
                                     1.0,  0.9238795325112867,  0.7071067811865476,  0.3826834323650898,
                                     0.0,  -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
                                     -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};
};

// (vr, vi) *= exp(-2 pi i J / 16), conjugated for INV; J = 4 (a quarter turn)
// is a swap with a sign
template <int J, bool INV>
__device__ __forceinline__ void mul_w16(double& vr, double& vi) {
    if constexpr (J == 0) {
        return;
    } else if constexpr (J == 4) {
        const double t = vr;
        if constexpr (INV) {
            vr = -vi;
            vi = t;
        } else {
            vr = vi;
            vi = -t;
        }
    } else {
        constexpr double wr = Tw16::c[J], wi = INV ? Tw16::s[J] : -Tw16::s[J];
        const double tr = vr * wr - vi * wi;
        vi = vr * wi + vi * wr;
        vr = tr;
    }
}

// R-point DFT in registers (radix-2 decimation in time, bit-reversed input
// order, natural output order), R in {2, 4, 8, 16}; the butterfly twiddle
// of stage len, index j is W_len^j = W_16^(16 j / len).
template <int R, bool INV, int LEN, int J>
__device__ __forceinline__ void butterflies(double (&ar)[R], double (&ai)[R], int s0) {
    constexpr int half = LEN / 2;
    double vr = ar[s0 + J + half], vi = ai[s0 + J + half];
    mul_w16<J * (16 / LEN), INV>(vr, vi);
    ar[s0 + J + half] = ar[s0 + J] - vr;
    ai[s0 + J + half] = ai[s0 + J] - vi;
    ar[s0 + J] += vr;
    ai[s0 + J] += vi;
    if constexpr (J + 1 < half) butterflies<R, INV, LEN, J + 1>(ar, ai, s0);
}

template <int R, bool INV, int LEN = 2>
__device__ __forceinline__ void dft_stages(double (&ar)[R], double (&ai)[R]) {
    if constexpr (LEN <= R) {
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += LEN) butterflies<R, INV, LEN, 0>(ar, ai, s0);
        dft_stages<R, INV, LEN * 2>(ar, ai);
    }
}

template <int M, int R, bool INV>
__device__ __forceinline__ void dft_reg(double (&re)[R], double (&im)[R]) {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "register DFT of 2, 4, 8 or 16 points");
    constexpr int LOG = ilog2c(R);
    double ar[R], ai[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        ar[bitrev(i, LOG)] = re[i];
        ai[bitrev(i, LOG)] = im[i];
    }
    dft_stages<R, INV>(ar, ai);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        re[i] = ar[i];
        im[i] = ai[i];
    }
}

// multiply by W_M^(e) (conjugate for INV), e taken mod M
template <int M, bool INV>
__device__ __forceinline__ void twiddle(double& re, double& im, int e, const double* twr, const double* twi) {
    const int m = e & (M - 1);
    const double wr = twr[m], wi = INV ? -twi[m] : twi[m];
    const double t = re * wr - im * wi;
    im = re * wi + im * wr;
    re = t;
}

template <int M, int MODE>  // 0: forward, 1: forward * Ghat * inverse, 2: inverse
__global__ __launch_bounds__(ColCfg<M>::NT) void k_fft_cols(const double2* __restrict__ in, double2* __restrict__ out,
                                                            ColArgs a, const double2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int R1 = C::R1, R2 = C::R2, NG = C::NG, BC = C::BC;
    constexpr int GZ = M / 2 + 1;  // kz octant rows
    __shared__ double ex[M * BC], twr[M], twi[M];  // exchange buffer: real parts, then imaginary parts
    for (int m = threadIdx.x; m < M; m += C::NT) {
        const double2 w = tw[m];
        twr[m] = w.x;
        twi[m] = w.y;
    }
    const int b = threadIdx.x % BC;
    const int r = threadIdx.x / BC;  // n2 in stage A / inverse stage 2; group base in the others
    const int tiles = (a.W + BC - 1) / BC;
    const int outer = blockIdx.x / tiles;
    const int col = (blockIdx.x - outer * tiles) * BC + b;
    const bool valid = col < a.W;
    // mode 1: this thread's Ghat values, issued first so that their latency
    // overlaps the transform (ky = outer, kx = col / ncc, one contiguous kz row)
    double gv[MODE == 1 ? NG : 1][R2];
    if (MODE == 1) {
        const int ky = outer, kx = col / a.ncc;
        const int gy = ky <= a.My - ky ? ky : a.My - ky;
        const int gx = kx <= a.Mx - kx ? kx : a.Mx - kx;
        const double* grow = a.ghat + ((int64_t)gy * a.gnx1 + gx) * GZ;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int kz = r + R2 * g + R1 * k2;
                const int gz = kz <= M - kz ? kz : M - kz;
                gv[g][k2] = valid ? grow[gz] : 0.0;
            }
        }
    }
    const double2* src = in + (int64_t)blockIdx.y * a.in_batch + (int64_t)outer * a.in_outer + (int64_t)col * a.bstride;
    double2* dst = out + (int64_t)blockIdx.y * a.out_batch + (int64_t)outer * a.out_outer + (int64_t)col * a.bstride;
    double hr[NG][R2], hi[NG][R2];  // groups k1 = r + R2 g, values over k2
    if (MODE != 2) {
        double xr[R1], xi[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) {
            const int row = R2 * n1 + r;
            double2 v = make_double2(0.0, 0.0);
            if (valid && row < a.n_in) v = src[(int64_t)row * a.in_stride];
            xr[n1] = v.x;
            xi[n1] = v.y;
        }
        __syncthreads();  // twiddle table
        dft_reg<M, R1, false>(xr, xi);
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) twiddle<M, false>(xr[k1], xi[k1], r * k1, twr, twi);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) ex[(k1 * R2 + r) * BC + b] = xr[k1];
        __syncthreads();
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) hr[g][n2] = ex[((r + R2 * g) * R2 + n2) * BC + b];
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) ex[(k1 * R2 + r) * BC + b] = xi[k1];
        __syncthreads();
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) hi[g][n2] = ex[((r + R2 * g) * R2 + n2) * BC + b];
            dft_reg<M, R2, false>(hr[g], hi[g]);
        }
        if (MODE == 0) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int t = (r + R2 * g + R1 * k2 + a.out_shift) & (M - 1);
                    if (valid && t < a.n_out) dst[(int64_t)t * a.out_stride] = make_double2(hr[g][k2], hi[g][k2]);
                }
            }
            return;
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                hr[g][k2] *= gv[g][k2];
                hi[g][k2] *= gv[g][k2];
            }
        }
        __syncthreads();  // every stage-B read of the exchange buffer is done
    } else {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int row = r + R2 * g + R1 * k2;
                double2 v = make_double2(0.0, 0.0);
                if (valid && row < a.n_in) v = src[(int64_t)row * a.in_stride];
                hr[g][k2] = v.x;
                hi[g][k2] = v.y;
            }
        }
        __syncthreads();  // twiddle table
    }
    // inverse: per k1 over k2, twiddle, exchange, per n2 over k1
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int k1 = r + R2 * g;
        dft_reg<M, R2, true>(hr[g], hi[g]);
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            twiddle<M, true>(hr[g][n2], hi[g][n2], n2 * k1, twr, twi);
            ex[(n2 * R1 + k1) * BC + b] = hr[g][n2];
        }
    }
    __syncthreads();
    double xr[R1], xi[R1];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) xr[k1] = ex[(r * R1 + k1) * BC + b];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) ex[(n2 * R1 + r + R2 * g) * BC + b] = hi[g][n2];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) xi[k1] = ex[(r * R1 + k1) * BC + b];
    dft_reg<M, R1, true>(xr, xi);
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
        const int t = (r + R2 * n1 + a.out_shift) & (M - 1);
        if (valid && t < a.n_out) dst[(int64_t)t * a.out_stride] = make_double2(xr[n1], xi[n1]);
    }
}

// ---------------------------------------------------------------- passes 2-4 fused
// With M-point y and z transforms, M = 128 or 64 (64 or 32 nodes), passes
// 2-4 of the forward solve run as one kernel: a workgroup takes one complex
// column (kx, channel) of one setting and keeps its (z, y) plane in LDS,
// (M/2 + 2) x M values, so the two intermediates of passes 2 and 3 never
// reach HBM (at 64^3 the solve's pass traffic falls from ~470 to ~200 MB).
// With n = M/2 nonzero inputs per dimension and RA = M/8:
//   y forward: each of the n input rows z, an M-point transform of its n
//     nonzero values, as RA- and 8-point register DFTs around one in-place
//     exchange in its plane row. Row slot 8 k1 + k2 ends up holding
//     ky = k1 + RA k2.
//   z: each ky column, forward over its n nonzero z, times Ghat, inverse to
//     the n + 2 needed z. The column has n + 2 slots, not M, so the M-point
//     transform is split by the parity of kz. The even kz are the n-point
//     transform of x, the odd kz that of x W_M^z. Each half is an
//     (n/8)-point and an 8-point register stage around an exchange in the
//     column's first n slots, and so is its inverse. The inverse M-point
//     transform at z is e(z mod n) + W_M^-z o(z mod n), with e and o the
//     two inverse halves.
//   y inverse: each of the n + 2 output rows, 8- and RA-point stages around
//     an exchange in the row, written to global memory at the n + 2 needed y.
// All transforms are unnormalised; 1/(Mx My Mz) is in Ghat. In global memory
// each column's input (z, y) and output (zo, yo) values are contiguous
// ("column planes"), which passes 1 and 5 write and read with strides.
// A thread's twiddles are powers of W_M^lo (lo, its place in its group of
// 8, is fixed) times compile-time powers of W_16, formed in registers.
template <int M>
struct YzCfg {
    static constexpr int N = M / 2, NO = N + 2;
    static constexpr int PS = M + 1;        // plane row stride (complex values), padded against bank conflicts
    static constexpr int RA = M / 8;        // row transforms: RA-point then 8-point stages
    static constexpr int HA = M / 16;       // z halves (N points): HA-point then 8-point stages
    static constexpr int NT = 8 * M;        // threads: 8 per column in the z transforms
    static constexpr int W16 = 128 / M;     // W_M^8 = W_16^W16
};

struct YzArgs {
    int W;                        // complex columns (Mx * NCC)
    int64_t cp_in, cp_out;        // column plane lengths: n n, and (n + 2)^2 padded to 8
    int64_t in_batch, out_batch;  // strides between settings (W cp_in, W cp_out)
    const double* ghat;
    int ncc, gnx1, Mx;
};

// (re, im) *= (wr, wi)
__device__ __forceinline__ void cmul_by(double& re, double& im, double wr, double wi) {
    const double t = re * wr - im * wi;
    im = re * wi + im * wr;
    re = t;
}

// (re, im) *= W_16^j (conjugated for inv), j a constant once the caller's loop is unrolled
__device__ __forceinline__ void mul_w16_at(double& re, double& im, int j, bool inv) {
#define DPIC_W16(J)                                        \
    case J:                                                \
        if (inv) mul_w16<J, true>(re, im);                 \
        else mul_w16<J, false>(re, im);                    \
        break;
    switch (j & 15) {
        DPIC_W16(0) DPIC_W16(1) DPIC_W16(2) DPIC_W16(3) DPIC_W16(4) DPIC_W16(5) DPIC_W16(6) DPIC_W16(7)
        DPIC_W16(8) DPIC_W16(9) DPIC_W16(10) DPIC_W16(11) DPIC_W16(12) DPIC_W16(13) DPIC_W16(14) DPIC_W16(15)
    }
#undef DPIC_W16
}

// Inside the y row transforms and the z column transforms, the lanes that
// exchange values through the plane are the 8 lanes of one row or column,
// which are always in one wavefront. A wavefront performs its LDS operations
// in issue order, so there a fence that keeps the compiler from moving LDS
// accesses across it replaces the workgroup barrier; barriers remain only
// where the data crosses wavefronts (the twiddle table, rows to columns and
// back).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int M>
__global__ __launch_bounds__(YzCfg<M>::NT) void k_fft_yz(const double2* __restrict__ in, double2* __restrict__ out,
                                                         YzArgs a, const double2* __restrict__ tw) {
    using C = YzCfg<M>;
    constexpr int N = C::N, NO = C::NO, PS = C::PS, RA = C::RA, HA = C::HA, NT = C::NT, W16 = C::W16;
    constexpr int GZ = M / 2 + 1;
    __shared__ double2 P[NO * PS];
    __shared__ double twr[M], twi[M];
    const int t = threadIdx.x;
    for (int m = t; m < M; m += NT) {
        const double2 w = tw[m];
        twr[m] = w.x;
        twi[m] = w.y;
    }
    // column of this workgroup: each XCD (workgroups round-robin over 8)
    // takes a contiguous eighth of the columns, so the NCC columns of one kx,
    // which read the same Ghat rows, go through one L2
    const int wpx = a.W / 8;
    const int col = (blockIdx.x % 8) * wpx + blockIdx.x / 8;
    const double2* src = in + (int64_t)blockIdx.y * a.in_batch + col * a.cp_in;
    double2* dst = out + (int64_t)blockIdx.y * a.out_batch + col * a.cp_out;
    const int lo = t & 7;  // n2 or r: the thread's place in its group of 8
    // the Ghat row (kx, ky) of this thread's z column p = t >> 3 (kz fastest)
    const double* grow;
    {
        const int p = t >> 3, ky = (p >> 3) + RA * (p & 7), kx = col / a.ncc;
        const int gy = ky <= M - ky ? ky : M - ky;
        const int gx = kx <= a.Mx - kx ? kx : a.Mx - kx;
        grow = a.ghat + ((int64_t)gy * a.gnx1 + gx) * GZ;
    }
    // y forward, rows z < n: stage A (thread (z, n2)), exchange, stage B (thread (z, r))
    const bool rowt = t < N * 8;
    const int zr = t >> 3;
    double xr[RA], xi[RA];
    if (rowt) {
#pragma unroll
        for (int n1 = 0; n1 < RA; ++n1) {
            xr[n1] = 0.0;
            xi[n1] = 0.0;
        }
#pragma unroll
        for (int n1 = 0; n1 < RA / 2; ++n1) {
            const double2 v = src[zr * N + 8 * n1 + lo];
            xr[n1] = v.x;
            xi[n1] = v.y;
        }
    }
    __syncthreads();  // twiddle table
    if (rowt) {
        const double w1r = twr[lo], w1i = twi[lo];
        dft_reg<M, RA, false>(xr, xi);
        double wr = w1r, wi = w1i;  // W^(lo k1)
#pragma unroll
        for (int k1 = 0; k1 < RA; ++k1) {
            if (k1 > 0) {
                cmul_by(xr[k1], xi[k1], wr, wi);
                cmul_by(wr, wi, w1r, w1i);
            }
            P[zr * PS + 8 * k1 + lo] = make_double2(xr[k1], xi[k1]);
        }
    }
    wave_sync();  // the row's 8 lanes
    if (rowt) {
#pragma unroll
        for (int g = 0; g < RA / 8; ++g) {
            const int k1 = lo + 8 * g;
            double hr[8], hi[8];
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) {
                const double2 v = P[zr * PS + 8 * k1 + n2];
                hr[n2] = v.x;
                hi[n2] = v.y;
            }
            dft_reg<M, 8, false>(hr, hi);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) P[zr * PS + 8 * k1 + k2] = make_double2(hr[k2], hi[k2]);
        }
    }
    __syncthreads();
    // z, column p = t >> 3 (slot p of every row): the thread holds x at z = 8 n1 + n2 (n2 = lo)
    const int p = t >> 3;
    double x0r[HA], x0i[HA];
#pragma unroll
    for (int n1 = 0; n1 < HA; ++n1) {
        const double2 v = P[(8 * n1 + lo) * PS + p];
        x0r[n1] = v.x;
        x0i[n1] = v.y;
    }
    double er[HA], ei[HA];
    const bool bt = lo < HA;  // stage-B role r = lo: the HA groups k1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        // Ghat at kz = 2 (r + HA k2) + h for role r = lo, issued before the stage that needs it
        double gv[8];
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            const int kz = 2 * (lo + HA * k2) + h;
            gv[k2] = bt ? grow[kz <= M - kz ? kz : M - kz] : 0.0;
        }
        wave_sync();  // every read of the column's slots before is done
        // stage A: HA-point DFT over n1 of x (x W_M^z for the odd kz), twiddle W_n^(n2 k1)
        double ar[HA], ai[HA];
        {
            const double w1r = twr[lo], w1i = twi[lo];
#pragma unroll
            for (int n1 = 0; n1 < HA; ++n1) {
                ar[n1] = x0r[n1];
                ai[n1] = x0i[n1];
                if (h == 1) {  // W_M^(8 n1 + lo)
                    cmul_by(ar[n1], ai[n1], w1r, w1i);
                    mul_w16_at(ar[n1], ai[n1], W16 * n1, false);
                }
            }
        }
        dft_reg<M, HA, false>(ar, ai);
        {
            const double w2r = twr[2 * lo], w2i = twi[2 * lo];  // W_M^(2 lo) = W_n^lo
            double wr = w2r, wi = w2i;
#pragma unroll
            for (int k1 = 0; k1 < HA; ++k1) {
                if (k1 > 0) {
                    cmul_by(ar[k1], ai[k1], wr, wi);
                    cmul_by(wr, wi, w2r, w2i);
                }
                P[(8 * k1 + lo) * PS + p] = make_double2(ar[k1], ai[k1]);
            }
        }
        wave_sync();
        // stage B (r = lo < HA): 8-point DFT over n2 gives kk = r + HA k2; times Ghat;
        // inverse 8-point DFT over k2, twiddle W_n^(-r n2)
        double br[8], bi[8];
        if (bt) {
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) {
                const double2 v = P[(8 * lo + n2) * PS + p];
                br[n2] = v.x;
                bi[n2] = v.y;
            }
            dft_reg<M, 8, false>(br, bi);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) {
                br[k2] *= gv[k2];
                bi[k2] *= gv[k2];
            }
            dft_reg<M, 8, true>(br, bi);
            const double w2r = twr[2 * lo], w2i = twi[2 * lo];
            double wr = w2r, wi = -w2i;  // W^(-2 lo n2)
#pragma unroll
            for (int n2 = 1; n2 < 8; ++n2) {
                cmul_by(br[n2], bi[n2], wr, wi);
                cmul_by(wr, wi, w2r, -w2i);
            }
        }
        wave_sync();  // every stage-B read is done
        if (bt)
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) P[(HA * n2 + lo) * PS + p] = make_double2(br[n2], bi[n2]);
        wave_sync();
        // stage A' (n2 = lo): inverse HA-point DFT over r gives z = n2 + 8 n1
#pragma unroll
        for (int r = 0; r < HA; ++r) {
            const double2 v = P[(HA * lo + r) * PS + p];
            ar[r] = v.x;
            ai[r] = v.y;
        }
        dft_reg<M, HA, true>(ar, ai);
        if (h == 0) {
#pragma unroll
            for (int n1 = 0; n1 < HA; ++n1) {
                er[n1] = ar[n1];
                ei[n1] = ai[n1];
            }
        } else {
            // combine at z = n2 + 8 n1 (slot z + 1); z = -1 and z = n reuse z mod n
            wave_sync();  // every stage-A' read is done
            const double w1r = twr[lo], w1i = twi[lo];
#pragma unroll
            for (int n1 = 0; n1 < HA; ++n1) {
                const int z = lo + 8 * n1;
                double orr = ar[n1], oi = ai[n1];  // times W_M^-z = W_M^-lo W_16^-(W16 n1)
                cmul_by(orr, oi, w1r, -w1i);
                mul_w16_at(orr, oi, W16 * n1, true);
                P[(z + 1) * PS + p] = make_double2(er[n1] + orr, ei[n1] + oi);
            }
            if (lo == 7) {  // z = -1 from z mod n = n - 1 (n1 = HA - 1)
                double orr = ar[HA - 1], oi = ai[HA - 1];
                twiddle<M, true>(orr, oi, M - 1, twr, twi);
                P[p] = make_double2(er[HA - 1] + orr, ei[HA - 1] + oi);
            }
            if (lo == 0) {  // z = n from z mod n = 0: W_M^-n = -1
                P[(N + 1) * PS + p] = make_double2(er[0] - ar[0], ei[0] - ai[0]);
            }
        }
    }
    __syncthreads();
    // y inverse, rows zo < n + 2: stage 1 (thread (zo, r)), exchange, stage 2 (thread (zo, n2))
    const bool outt = t < NO * 8;
    double cr[RA / 8][8], ci[RA / 8][8];
    if (outt) {
        const double w1r = twr[lo], w1i = twi[lo];
#pragma unroll
        for (int g = 0; g < RA / 8; ++g) {
            const int k1 = lo + 8 * g;
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) {
                const double2 v = P[zr * PS + 8 * k1 + k2];
                cr[g][k2] = v.x;
                ci[g][k2] = v.y;
            }
            dft_reg<M, 8, true>(cr[g], ci[g]);
            double wr = w1r, wi = -w1i;  // W^(-n2 lo); k1 = lo + 8 g adds W_M^(-8 n2 g)
#pragma unroll
            for (int n2 = 1; n2 < 8; ++n2) {
                cmul_by(cr[g][n2], ci[g][n2], wr, wi);
                if (g > 0) mul_w16_at(cr[g][n2], ci[g][n2], W16 * n2 * g, true);
                cmul_by(wr, wi, w1r, -w1i);
            }
        }
    }
    wave_sync();
    if (outt) {
#pragma unroll
        for (int g = 0; g < RA / 8; ++g)
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) P[zr * PS + RA * n2 + lo + 8 * g] = make_double2(cr[g][n2], ci[g][n2]);
    }
    wave_sync();
    if (outt) {
#pragma unroll
        for (int k1 = 0; k1 < RA; ++k1) {
            const double2 v = P[zr * PS + RA * lo + k1];
            xr[k1] = v.x;
            xi[k1] = v.y;
        }
        dft_reg<M, RA, true>(xr, xi);
#pragma unroll
        for (int n1 = 0; n1 < RA; ++n1) {
            const int yo = (lo + 8 * n1 + 1) & (M - 1);
            if (yo < NO) dst[zr * NO + yo] = make_double2(xr[n1], xi[n1]);
        }
    }
}

// ---------------------------------------------------------------- passes 1 and 5
// x transforms with the column kernels' stages: column b of a block is
// complex channel j = b % NCC of row b / NCC; its value at x is the pair of
// real channels (j, j + NCC) (the real channel alone when NC = 1).

// Where the x passes keep their complex spectra: value (row g, column c),
// c = kx NCC + j, sits at (g / rps) bstride + (g % rps) rstride + c cstride.
// Row-major ([row][c]): rstride = W, cstride = 1, one block of all rows.
// Column planes ([setting][c][row], the fused y-z pass's layout): rps rows
// per setting, rstride = 1, cstride = the plane's padded length.
struct RowLayout {
    uint32_t rps;
    int64_t bstride, rstride, cstride;
    __host__ __device__ int64_t at(uint32_t g) const { return (int64_t)(g / rps) * bstride + (int64_t)(g % rps) * rstride; }
};

// pass 1: rho[row][x < nx][NC] -> out (row g, column kx NCC + j), clearing rho
template <int M, int NC>
__global__ __launch_bounds__(ColCfg<M>::NT) void k_fft_rows_fwd(double* __restrict__ rho, double2* __restrict__ out,
                                                                int nx, int rows, RowLayout lay,
                                                                const double2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int R1 = C::R1, R2 = C::R2, NG = C::NG, BC = C::BC;
    constexpr int NCC = NC == 1 ? 1 : NC / 2;
    static_assert(BC % NCC == 0, "whole rows per block");
    __shared__ double ex[M * BC], twr[M], twi[M];  // exchange buffer: real parts, then imaginary parts
    for (int m = threadIdx.x; m < M; m += C::NT) {
        const double2 w = tw[m];
        twr[m] = w.x;
        twi[m] = w.y;
    }
    const int b = threadIdx.x % BC;
    const int r = threadIdx.x / BC;
    const int64_t row = (int64_t)blockIdx.x * (BC / NCC) + b / NCC;
    const int j = b % NCC;
    const bool valid = row < rows;
    double* src = rho + row * nx * NC + j;
    double xr[R1], xi[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
        const int x = R2 * n1 + r;
        xr[n1] = 0.0;
        xi[n1] = 0.0;
        if (valid && x < nx) {
            xr[n1] = src[x * NC];
            src[x * NC] = 0.0;
            if (NC > 1) {
                xi[n1] = src[x * NC + NCC];
                src[x * NC + NCC] = 0.0;
            }
        }
    }
    __syncthreads();  // twiddle table
    dft_reg<M, R1, false>(xr, xi);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) twiddle<M, false>(xr[k1], xi[k1], r * k1, twr, twi);
    double hr[NG][R2], hi[NG][R2];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) ex[(k1 * R2 + r) * BC + b] = xr[k1];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) hr[g][n2] = ex[((r + R2 * g) * R2 + n2) * BC + b];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) ex[(k1 * R2 + r) * BC + b] = xi[k1];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) hi[g][n2] = ex[((r + R2 * g) * R2 + n2) * BC + b];
        dft_reg<M, R2, false>(hr[g], hi[g]);
    }
    if (!valid) return;
    double2* dst = out + lay.at((uint32_t)row) + j * lay.cstride;
    const int64_t kxs = NCC * lay.cstride;
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) dst[(r + R2 * g + R1 * k2) * kxs] = make_double2(hr[g][k2], hi[g][k2]);
}

// pass 5: in (row g, column kx NCC + j) -> phi[row][xo < nxo][NC]; output
// slot xo holds transform position xo - shift
template <int M, int NC>
__global__ __launch_bounds__(ColCfg<M>::NT) void k_fft_rows_inv(const double2* __restrict__ in, double* __restrict__ phi,
                                                                int nxo, int shift, int rows, RowLayout lay,
                                                                const double2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int R1 = C::R1, R2 = C::R2, NG = C::NG, BC = C::BC;
    constexpr int NCC = NC == 1 ? 1 : NC / 2;
    static_assert(BC % NCC == 0, "whole rows per block");
    __shared__ double ex[M * BC], twr[M], twi[M];
    for (int m = threadIdx.x; m < M; m += C::NT) {
        const double2 w = tw[m];
        twr[m] = w.x;
        twi[m] = w.y;
    }
    const int b = threadIdx.x % BC;
    const int r = threadIdx.x / BC;
    const int64_t row = (int64_t)blockIdx.x * (BC / NCC) + b / NCC;
    const int j = b % NCC;
    const bool valid = row < rows;
    const double2* src = in + lay.at((uint32_t)row) + j * lay.cstride;
    const int64_t kxs = NCC * lay.cstride;
    double hr[NG][R2], hi[NG][R2];  // groups k1 = r + R2 g, values over k2
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            double2 v = make_double2(0.0, 0.0);
            if (valid) v = src[(r + R2 * g + R1 * k2) * kxs];
            hr[g][k2] = v.x;
            hi[g][k2] = v.y;
        }
    __syncthreads();  // twiddle table
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int k1 = r + R2 * g;
        dft_reg<M, R2, true>(hr[g], hi[g]);
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            twiddle<M, true>(hr[g][n2], hi[g][n2], n2 * k1, twr, twi);
            ex[(n2 * R1 + k1) * BC + b] = hr[g][n2];
        }
    }
    __syncthreads();
    double xr[R1], xi[R1];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) xr[k1] = ex[(r * R1 + k1) * BC + b];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) ex[(n2 * R1 + r + R2 * g) * BC + b] = hi[g][n2];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) xi[k1] = ex[(r * R1 + k1) * BC + b];
    dft_reg<M, R1, true>(xr, xi);
    if (!valid) return;
    double* dst = phi + row * nxo * NC + j;
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
        const int xo = (r + R2 * n1 + shift) & (M - 1);
        if (xo < nxo) {
            dst[xo * NC] = xr[n1];
            if (NC > 1) dst[xo * NC + NCC] = xi[n1];
        }
    }
}


template <int MODE>
static hipError_t launch_cols(int M, int n_outer, int nb, const ColArgs& a, const double2* in, double2* out,
                              const double2* tw, hipStream_t s) {
    switch (M) {
#define DPIC_COLS(MM)                                                                                 \
    case MM: {                                                                                        \
        using C = ColCfg<MM>;                                                                         \
        const unsigned blocks = (unsigned)n_outer * (unsigned)((a.W + C::BC - 1) / C::BC);            \
        hipLaunchKernelGGL((k_fft_cols<MM, MODE>), dim3(blocks, nb), dim3(C::NT), 0, s, in, out, a, tw); \
        break;                                                                                        \
    }
        DPIC_COLS(16) DPIC_COLS(32) DPIC_COLS(64) DPIC_COLS(128)
#undef DPIC_COLS
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NC>
static hipError_t launch_rows_fwd_nc(int M, double* rho, double2* out, int nx, int rows, const RowLayout& lay,
                                     const double2* tw, hipStream_t s) {
    constexpr int NCC = NC == 1 ? 1 : NC / 2;
    switch (M) {
#define DPIC_ROWS_FWD(MM)                                                                                        \
    case MM: {                                                                                                   \
        constexpr int RB = ColCfg<MM>::BC / NCC;                                                                 \
        hipLaunchKernelGGL((k_fft_rows_fwd<MM, NC>), dim3((rows + RB - 1) / RB), dim3(ColCfg<MM>::NT), 0, s, rho, \
                           out, nx, rows, lay, tw);                                                              \
        break;                                                                                                   \
    }
        DPIC_ROWS_FWD(16) DPIC_ROWS_FWD(32) DPIC_ROWS_FWD(64) DPIC_ROWS_FWD(128)
#undef DPIC_ROWS_FWD
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NC>
static hipError_t launch_rows_inv_nc(int M, const double2* in, double* phi, int nxo, int shift, int rows,
                                     const RowLayout& lay, const double2* tw, hipStream_t s) {
    constexpr int NCC = NC == 1 ? 1 : NC / 2;
    switch (M) {
#define DPIC_ROWS_INV(MM)                                                                                       \
    case MM: {                                                                                                  \
        constexpr int RB = ColCfg<MM>::BC / NCC;                                                                \
        hipLaunchKernelGGL((k_fft_rows_inv<MM, NC>), dim3((rows + RB - 1) / RB), dim3(ColCfg<MM>::NT), 0, s, in, \
                           phi, nxo, shift, rows, lay, tw);                                                     \
        break;                                                                                                  \
    }
        DPIC_ROWS_INV(16) DPIC_ROWS_INV(32) DPIC_ROWS_INV(64) DPIC_ROWS_INV(128)
#undef DPIC_ROWS_INV
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// out(t) = sum_q in(q) G((t - shift) - q) per dimension, on windows of the
// doubled grid: input window index q sits at grid position q, output window
// index t holds grid position t - shift; both arrays are real [z][y][x][NC].
// The forward solve uses nin = n (rho) and nout = n + 2 with shift 1 (the
// ghost ring at position -1 = M - 1); the adjoint solve uses nin = n + 2 (its
// source already shifted by one) and nout = n with shift -1.
hipError_t launch_conv(dpic_ctx* cx, double* in, const int nin[3], double* out, const int nout[3], int shift, int NC,
                       int nb) {
    const int nx = cx->dims.nx, ny = cx->dims.ny, nz = cx->dims.nz;
    const int Mx = 2 * nx, My = 2 * ny, Mz = 2 * nz;
    const int NCC = NC == 1 ? 1 : NC / 2;
    const double2* twx = cx->ws.tw;
    const double2* twy = cx->ws.tw + Mx;
    const double2* twz = cx->ws.tw + Mx + My;
    hipStream_t s = cx->stream;
    hipError_t e;
    const int64_t W = (int64_t)Mx * NCC;
    // passes 2-4 fused where y and z both have 32 or 64 nodes (forward solve)
    const bool fused = My == Mz && (My == 128 || My == 64) && nin[1] == My / 2 && nin[2] == My / 2 &&
                       nout[1] == My / 2 + 2 && nout[2] == My / 2 + 2 && shift == 1 && W % 8 == 0;
    const int rows_in = nin[1] * nin[2], rows_out = nout[1] * nout[2];
    // the fused pass reads and writes column planes (one column's rows
    // contiguous), so that its loads and stores take whole cache lines; the
    // output plane is padded to a multiple of 8 rows (128 bytes). Both fit
    // the work arrays, which hold nb (nz + 2) My W values.
    const int64_t cp_in = rows_in, cp_out = (rows_out + 7) / 8 * 8;
    const RowLayout lay_in = fused ? RowLayout{(uint32_t)rows_in, W * cp_in, 1, cp_in} : RowLayout{1u << 31, 0, W, 1};
    const RowLayout lay_out =
        fused ? RowLayout{(uint32_t)rows_out, W * cp_out, 1, cp_out} : RowLayout{1u << 31, 0, W, 1};
    // 1: x forward, in -> A (rows z, y of nin; columns kx, channel)
    switch (NC) {
        case 1: e = launch_rows_fwd_nc<1>(Mx, in, cx->ws.buf0, nin[0], rows_in * nb, lay_in, twx, s); break;
        case 8: e = launch_rows_fwd_nc<8>(Mx, in, cx->ws.buf0, nin[0], rows_in * nb, lay_in, twx, s); break;
        default: e = launch_rows_fwd_nc<16>(Mx, in, cx->ws.buf0, nin[0], rows_in * nb, lay_in, twx, s); break;
    }
    if (e != hipSuccess) return e;
    if (fused) {
        // 2-4 fused: A -> D without the two intermediates
        YzArgs y{};
        y.W = (int)W;
        y.cp_in = cp_in;
        y.cp_out = cp_out;
        y.in_batch = W * cp_in;
        y.out_batch = W * cp_out;
        y.ghat = cx->ws.ghat;
        y.ncc = NCC;
        y.gnx1 = nx + 1;
        y.Mx = Mx;
        if (My == 128)
            hipLaunchKernelGGL(k_fft_yz<128>, dim3((unsigned)W, nb), dim3(YzCfg<128>::NT), 0, s, cx->ws.buf0,
                               cx->ws.buf1, y, twy);
        else
            hipLaunchKernelGGL(k_fft_yz<64>, dim3((unsigned)W, nb), dim3(YzCfg<64>::NT), 0, s, cx->ws.buf0,
                               cx->ws.buf1, y, twy);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int rows = rows_out * nb;
        switch (NC) {
            case 1: return launch_rows_inv_nc<1>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
            case 8: return launch_rows_inv_nc<8>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
            default: return launch_rows_inv_nc<16>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
        }
    }
    ColArgs a{};
    a.W = (int)W;
    a.bstride = 1;
    a.ghat = cx->ws.ghat;
    a.ncc = NCC;
    a.gnx1 = nx + 1;
    a.Mx = Mx;
    a.My = My;
    // settings are back to back in every array
    // 2: y forward, A -> B[nin_z][My][Mx]
    a.in_outer = (int64_t)nin[1] * W;
    a.in_stride = W;
    a.n_in = nin[1];
    a.out_outer = (int64_t)My * W;
    a.out_stride = W;
    a.n_out = My;
    a.out_shift = 0;
    a.in_batch = (int64_t)nin[2] * a.in_outer;
    a.out_batch = (int64_t)nin[2] * a.out_outer;
    if ((e = launch_cols<0>(My, nin[2], nb, a, cx->ws.buf0, cx->ws.buf1, twy, s)) != hipSuccess) return e;
    // 3: z forward, Ghat, z inverse, B -> C[nout_z][My][Mx]
    a.in_outer = W;
    a.in_stride = (int64_t)My * W;
    a.n_in = nin[2];
    a.out_outer = W;
    a.out_stride = (int64_t)My * W;
    a.n_out = nout[2];
    a.out_shift = shift;
    a.in_batch = (int64_t)nin[2] * My * W;
    a.out_batch = (int64_t)nout[2] * My * W;
    if ((e = launch_cols<1>(Mz, My, nb, a, cx->ws.buf1, cx->ws.buf0, twz, s)) != hipSuccess) return e;
    // 4: y inverse, C -> D[nout_z][nout_y][Mx]
    a.in_outer = (int64_t)My * W;
    a.in_stride = W;
    a.n_in = My;
    a.out_outer = (int64_t)nout[1] * W;
    a.out_stride = W;
    a.n_out = nout[1];
    a.out_shift = shift;
    a.in_batch = (int64_t)nout[2] * a.in_outer;
    a.out_batch = (int64_t)nout[2] * a.out_outer;
    if ((e = launch_cols<2>(My, nout[2], nb, a, cx->ws.buf0, cx->ws.buf1, twy, s)) != hipSuccess) return e;
    // 5: x inverse, D -> out
    const int rows = rows_out * nb;
    switch (NC) {
        case 1: return launch_rows_inv_nc<1>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
        case 8: return launch_rows_inv_nc<8>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
        default: return launch_rows_inv_nc<16>(Mx, cx->ws.buf1, out, nout[0], shift, rows, lay_out, twx, s);
    }
}

hipError_t launch_solve(dpic_ctx* cx) {
    const int n[3] = {cx->dims.nx, cx->dims.ny, cx->dims.nz};
    const int g[3] = {n[0] + 2, n[1] + 2, n[2] + 2};
    return launch_conv(cx, cx->ws.rho, n, cx->ws.phi, g, 1, cx->NC, cx->B);
}

// ---------------------------------------------------------------- Green's function
// Mean of 1/r over the box [-a,a] x [-b,b] x [-c,c] from the closed-form
// antiderivative F of 1/r (d^3 F / dx dy dz = 1/r):
// F = yz ln(x+r) + xz ln(y+r) + xy ln(z+r)
//     - x^2/2 atan(yz/(xr)) - y^2/2 atan(xz/(yr)) - z^2/2 atan(xy/(zr)),
// evaluated over the octant [0,a]x[0,b]x[0,c] by inclusion-exclusion; the
// corners with a zero coordinate only keep the yz ln r style terms.
__device__ double inv_r_antideriv(double x, double y, double z) {
    const double r = sqrt(x * x + y * y + z * z);
    double t = 0.0;
    if (y > 0.0 && z > 0.0) t += y * z * log(x + r);
    if (x > 0.0 && z > 0.0) t += x * z * log(y + r);
    if (x > 0.0 && y > 0.0) t += x * y * log(z + r);
    if (x > 0.0) t -= 0.5 * x * x * atan(y * z / (x * r));
    if (y > 0.0) t -= 0.5 * y * y * atan(x * z / (y * r));
    if (z > 0.0) t -= 0.5 * z * z * atan(x * y / (z * r));
    return t;
}

__device__ double mean_inv_r(double hx, double hy, double hz) {
    const double a = 0.5 * hx, b = 0.5 * hy, c = 0.5 * hz;
    double s = 0.0;
    for (int i = 0; i < 8; ++i) {
        const double x = (i & 1) ? 0.0 : a;
        const double y = (i & 2) ? 0.0 : b;
        const double z = (i & 4) ? 0.0 : c;
        const double sg = (__popc(i) & 1) ? -1.0 : 1.0;
        s += sg * inv_r_antideriv(x, y, z);
    }
    return 8.0 * s / (hx * hy * hz);
}

// G on the doubled grid [Mz][My][Mx]; hz_rest = gamma0 hz (rest-frame cell).
__global__ void k_green_fill(double2* __restrict__ g, int nx, int ny, int nz, double hx, double hy, double hz_rest,
                             double coef) {
    const int Mx = 2 * nx, My = 2 * ny, Mz = 2 * nz;
    const int64_t total = (int64_t)Mx * My * Mz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int ix = (int)(i % Mx);
    const int iy = (int)((i / Mx) % My);
    const int iz = (int)(i / ((int64_t)Mx * My));
    const int ox = ix <= nx ? ix : ix - Mx;
    const int oy = iy <= ny ? iy : iy - My;
    const int oz = iz <= nz ? iz : iz - Mz;
    double v;
    if (ox == 0 && oy == 0 && oz == 0) {
        v = coef * mean_inv_r(hx, hy, hz_rest);
    } else {
        const double rx = ox * hx, ry = oy * hy, rz = oz * hz_rest;
        v = coef / sqrt(rx * rx + ry * ry + rz * rz);
    }
    g[i] = make_double2(v, 0.0);
}

__global__ void k_green_extract(const double2* __restrict__ G, double* __restrict__ ghat, int nx, int ny, int nz,
                                double scale) {
    const int Mx = 2 * nx, My = 2 * ny;
    const int64_t total = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int ix = (int)(i % (nx + 1));
    const int iy = (int)((i / (nx + 1)) % (ny + 1));
    const int iz = (int)(i / ((int64_t)(nx + 1) * (ny + 1)));
    ghat[((int64_t)iy * (nx + 1) + ix) * (nz + 1) + iz] = G[((int64_t)iz * My + iy) * Mx + ix].x * scale;
}

// tw[m] = exp(-2 pi i m / M) for each axis, tables back to back.
__global__ void k_twiddles(double2* __restrict__ tw, int Mx, int My, int Mz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int M, m;
    if (i < Mx) {
        M = Mx;
        m = i;
    } else if (i < Mx + My) {
        M = My;
        m = i - Mx;
    } else if (i < Mx + My + Mz) {
        M = Mz;
        m = i - Mx - My;
    } else {
        return;
    }
    double sn, cs;
    sincospi(2.0 * (double)m / (double)M, &sn, &cs);
    tw[i] = make_double2(cs, -sn);
}

hipError_t launch_green(dpic_ctx* cx) {
    const int nx = cx->dims.nx, ny = cx->dims.ny, nz = cx->dims.nz;
    const int Mx = 2 * nx, My = 2 * ny, Mz = 2 * nz;
    hipStream_t s = cx->stream;
    hipLaunchKernelGGL(k_twiddles, dim3((Mx + My + Mz + 255) / 256), dim3(256), 0, s, cx->ws.tw, Mx, My, Mz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double eps0 = 8.8541878128e-12;
    const double pi = 3.14159265358979323846;
    const double coef = 1.0 / (4.0 * pi * eps0);
    const int64_t total = (int64_t)Mx * My * Mz;
    hipLaunchKernelGGL(k_green_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, cx->ws.buf0, nx, ny, nz,
                       cx->h[0], cx->h[1], cx->gamma0 * cx->h[2], coef);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const double2* twx = cx->ws.tw;
    const double2* twy = cx->ws.tw + Mx;
    const double2* twz = cx->ws.tw + Mx + My;
    ColArgs a{};
    // x: outer z, columns y (stride Mx), rows x (stride 1)
    a.W = My;
    a.bstride = Mx;
    a.in_outer = (int64_t)Mx * My;
    a.in_stride = 1;
    a.n_in = Mx;
    a.out_outer = (int64_t)Mx * My;
    a.out_stride = 1;
    a.n_out = Mx;
    a.out_shift = 0;
    if ((e = launch_cols<0>(Mx, Mz, 1, a, cx->ws.buf0, cx->ws.buf1, twx, s)) != hipSuccess) return e;
    // y: outer z, columns x (stride 1), rows y (stride Mx)
    a.W = Mx;
    a.bstride = 1;
    a.in_stride = Mx;
    a.n_in = My;
    a.out_stride = Mx;
    a.n_out = My;
    if ((e = launch_cols<0>(My, Mz, 1, a, cx->ws.buf1, cx->ws.buf0, twy, s)) != hipSuccess) return e;
    // z: outer y, columns x, rows z (stride Mx My)
    a.in_outer = Mx;
    a.in_stride = (int64_t)Mx * My;
    a.n_in = Mz;
    a.out_outer = Mx;
    a.out_stride = (int64_t)Mx * My;
    a.n_out = Mz;
    if ((e = launch_cols<0>(Mz, My, 1, a, cx->ws.buf0, cx->ws.buf1, twz, s)) != hipSuccess) return e;
    const int64_t oct = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    hipLaunchKernelGGL(k_green_extract, dim3((unsigned)((oct + 255) / 256)), dim3(256), 0, s, cx->ws.buf1, cx->ws.ghat,
                       nx, ny, nz, 1.0 / (double)total);
    return hipGetLastError();
}

// ---------------------------------------------------------------- field
// E = -grad phi by central differences on every node; phi carries one ghost
// ring. cz includes 1/gamma0 (rest-frame longitudinal field).
template <int NC>
__global__ void k_field(const double* __restrict__ phi, double* __restrict__ E, int nx, int ny, int nz, int nb,
                        double cx, double cy, double cz) {
    constexpr int CP = NC >= 2 ? 2 : 1;  // channels per thread (16-byte accesses)
    constexpr int NT = NC / CP;
    // blocks go round-robin to the 8 XCDs, each with its own L2: give each
    // XCD a contiguous range of blocks (whole z-slabs), so that the y and z
    // neighbours a row reads are in its own L2 (17.3 -> 13.8 us at 64^3 nodes)
    uint32_t lb = blockIdx.x;
    if ((gridDim.x & 7u) == 0u) lb = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int64_t gid = (int64_t)lb * blockDim.x + threadIdx.x;
    const int64_t nodes = (int64_t)nx * ny * nz;
    if (gid >= nodes * NT * nb) return;
    const int c = (int)(gid % NT) * CP;
    const int64_t gnode = gid / NT;
    const int64_t b = gnode / nodes;
    const int64_t node = gnode - b * nodes;
    const int ix = (int)(node % nx);
    const int iy = (int)((node / nx) % ny);
    const int iz = (int)(node / ((int64_t)nx * ny));
    const int64_t sx = NC, sy = (int64_t)(nx + 2) * NC, sz = (int64_t)(nx + 2) * (ny + 2) * NC;
    const double* p = phi + b * (nz + 2) * sz + (iz + 1) * sz + (iy + 1) * sy + (ix + 1) * sx + c;
    double* o = E + gnode * 3 * NC + c;
    if constexpr (CP == 2) {
        auto ld = [](const double* q) { return *reinterpret_cast<const double2*>(q); };
        auto st = [](double* q, double2 v) { *reinterpret_cast<double2*>(q) = v; };
        const double2 xp = ld(p + sx), xm = ld(p - sx), yp = ld(p + sy), ym = ld(p - sy), zp = ld(p + sz), zm = ld(p - sz);
        st(o, make_double2(cx * (xp.x - xm.x), cx * (xp.y - xm.y)));
        st(o + NC, make_double2(cy * (yp.x - ym.x), cy * (yp.y - ym.y)));
        st(o + 2 * NC, make_double2(cz * (zp.x - zm.x), cz * (zp.y - zm.y)));
    } else {
        o[0] = cx * (p[sx] - p[-sx]);
        o[NC] = cy * (p[sy] - p[-sy]);
        o[2 * NC] = cz * (p[sz] - p[-sz]);
    }
}

hipError_t launch_field(dpic_ctx* cx) {
    const int nx = cx->dims.nx, ny = cx->dims.ny, nz = cx->dims.nz;
    const double fx = -0.5 / cx->h[0], fy = -0.5 / cx->h[1], fz = -0.5 / (cx->h[2] * cx->gamma0);
    const int nb = cx->B;
    const int64_t total = (int64_t)nx * ny * nz * (cx->NC >= 2 ? cx->NC / 2 : 1) * nb;
    dim3 grid((unsigned)((total + 255) / 256)), block(256);
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_field<1>, grid, block, 0, cx->stream, cx->ws.phi, cx->ws.E, nx, ny, nz, nb, fx, fy, fz); break;
        case 8: hipLaunchKernelGGL(k_field<8>, grid, block, 0, cx->stream, cx->ws.phi, cx->ws.E, nx, ny, nz, nb, fx, fy, fz); break;
        default: hipLaunchKernelGGL(k_field<16>, grid, block, 0, cx->stream, cx->ws.phi, cx->ws.E, nx, ny, nz, nb, fx, fy, fz); break;
    }
    return hipGetLastError();
}

}  // namespace dpic
