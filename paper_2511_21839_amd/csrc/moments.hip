// Dual beam moments and emittances (Sec. 4: eps_x = sqrt(<x^2><px^2> - <x px>^2)
// with 1/N sums over all macroparticles, every quantity a dual number).
//
// Pass 1: each block accumulates, per lane channel, the 15 sums
// (u^2, u p, p^2, u, p for the planes (x,px), (y,py), (z,delta)) over a
// grid-stride range of particles and writes one partial row per block.
// Pass 2: one block adds the partial rows in a fixed order (the result is
// bitwise reproducible for a given particle order), divides by N and forms
// the raw and the centred emittances with the dual rules.
#include "context.hpp"

namespace dpic {

constexpr int MOM_THREADS = 256;

template <int NC>
__global__ __launch_bounds__(MOM_THREADS) void k_moments_partial(const double* __restrict__ st, int64_t n, int64_t cap,
                                                                 double* __restrict__ part) {
    constexpr int PPB = MOM_THREADS / NC;  // particles per block per sweep
    const int c = threadIdx.x % NC;
    const int64_t cs = cap * NC;
    double acc[MOM_N];
#pragma unroll
    for (int m = 0; m < MOM_N; ++m) acc[m] = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * PPB + threadIdx.x / NC; p < n; p += (int64_t)gridDim.x * PPB) {
        const double* sp = st + p * NC;
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
            const LD u = ldload(sp + (2 * pl) * cs, c);
            const LD q = ldload(sp + (2 * pl + 1) * cs, c);
            acc[pl * 5 + 0] += ldchan(u * u, c);
            acc[pl * 5 + 1] += ldchan(u * q, c);
            acc[pl * 5 + 2] += ldchan(q * q, c);
            acc[pl * 5 + 3] += ldchan(u, c);
            acc[pl * 5 + 4] += ldchan(q, c);
        }
    }
    // lanes with equal channel sit NC apart: fold the wavefront onto its first NC lanes
#pragma unroll
    for (int m = 0; m < MOM_N; ++m) {
#pragma unroll
        for (int off = 32; off >= NC; off >>= 1) acc[m] += __shfl_down(acc[m], off, 64);
    }
    __shared__ double red[MOM_THREADS / 64][MOM_N][NC];
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (lane < NC) {
#pragma unroll
        for (int m = 0; m < MOM_N; ++m) red[wave][m][lane] = acc[m];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MOM_N * NC; i += MOM_THREADS) {
        const int m = i / NC, ch = i % NC;
        double s = 0.0;
        for (int w = 0; w < MOM_THREADS / 64; ++w) s += red[w][m][ch];
        part[(size_t)blockIdx.x * MOM_N * NC + i] = s;
    }
}

template <int NC>
__global__ void k_moments_final(const double* __restrict__ part, int nblocks, double inv_n, double* __restrict__ mom,
                                double* __restrict__ emit) {
    __shared__ double sm[MOM_N * NC];
    for (int i = threadIdx.x; i < MOM_N * NC; i += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * MOM_N * NC + i];
        sm[i] = s * inv_n;
        mom[i] = s * inv_n;
    }
    __syncthreads();
    const int c = threadIdx.x;
    if (c >= NC) return;
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
        const double* m = sm + pl * 5 * NC;
        LD uu = ldload(m + 0 * NC, c), up = ldload(m + 1 * NC, c), pp = ldload(m + 2 * NC, c);
        const LD u = ldload(m + 3 * NC, c), q = ldload(m + 4 * NC, c);
        emit[(0 * 3 + pl) * NC + c] = ldchan(dsqrt(uu * pp - up * up), c);
        uu = uu - u * u;
        up = up - u * q;
        pp = pp - q * q;
        emit[(1 * 3 + pl) * NC + c] = ldchan(dsqrt(uu * pp - up * up), c);
    }
}

hipError_t launch_moments(dpic_ctx* cx) {
    int64_t want = (cx->n * cx->NC + MOM_THREADS - 1) / MOM_THREADS;
    int nblocks = (int)(want < MOM_BLOCKS ? (want < 1 ? 1 : want) : MOM_BLOCKS);
    const double inv_n = cx->n > 0 ? 1.0 / (double)cx->n : 0.0;
    hipStream_t s = cx->stream;
    switch (cx->NC) {
        case 1:
            hipLaunchKernelGGL(k_moments_partial<1>, dim3(nblocks), dim3(MOM_THREADS), 0, s, cx->ws.st, cx->n, cx->dims.n_particles, cx->ws.mom_part);
            hipLaunchKernelGGL(k_moments_final<1>, dim3(1), dim3(256), 0, s, cx->ws.mom_part, nblocks, inv_n, cx->ws.mom, cx->ws.emit);
            break;
        case 8:
            hipLaunchKernelGGL(k_moments_partial<8>, dim3(nblocks), dim3(MOM_THREADS), 0, s, cx->ws.st, cx->n, cx->dims.n_particles, cx->ws.mom_part);
            hipLaunchKernelGGL(k_moments_final<8>, dim3(1), dim3(256), 0, s, cx->ws.mom_part, nblocks, inv_n, cx->ws.mom, cx->ws.emit);
            break;
        default:
            hipLaunchKernelGGL(k_moments_partial<16>, dim3(nblocks), dim3(MOM_THREADS), 0, s, cx->ws.st, cx->n, cx->dims.n_particles, cx->ws.mom_part);
            hipLaunchKernelGGL(k_moments_final<16>, dim3(1), dim3(256), 0, s, cx->ws.mom_part, nblocks, inv_n, cx->ws.mom, cx->ws.emit);
            break;
    }
    return hipGetLastError();
}

}  // namespace dpic
