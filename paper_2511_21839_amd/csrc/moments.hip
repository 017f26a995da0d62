// Dual beam moments and emittances (Sec. 4: eps_x = sqrt(<x^2><px^2> - <x px>^2)
// with 1/N sums over all macroparticles, every quantity a dual number).
//
// Pass 1: each block accumulates, per lane channel, the 15 sums
// (u^2, u p, p^2, u, p for the planes (x,px), (y,py), (z,delta)) over a
// grid-stride range of particles and writes one partial row per block.
// Each setting of a batch has its own partial rows and result.
// Pass 2: one block adds the partial rows in a fixed order (the result is
// bitwise reproducible for a given particle order), divides by N and forms
// the raw and the centred emittances with the dual rules.
#include "context.hpp"

namespace dpic {

constexpr int MOM_THREADS = 256;

// grid (blocks per setting, B): block x of setting y sums a grid-stride part
// of the setting's slots [off, off + n)
template <int NC>
__global__ __launch_bounds__(MOM_THREADS) void k_moments_partial(const double* __restrict__ st, int64_t cap,
                                                                 const SettingDev* __restrict__ set,
                                                                 double* __restrict__ part) {
    constexpr int PPB = MOM_THREADS / NC;  // particles per block per sweep
    const int c = threadIdx.x % NC;
    const int64_t cs = cap * NC;
    const SettingDev sd = set[blockIdx.y];
    const int64_t end = sd.off + sd.n;
    double acc[MOM_N];
#pragma unroll
    for (int m = 0; m < MOM_N; ++m) acc[m] = 0.0;
    for (int64_t p = sd.off + (int64_t)blockIdx.x * PPB + threadIdx.x / NC; p < end; p += (int64_t)gridDim.x * PPB) {
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
        part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * MOM_N * NC + i] = s;
    }
}

// one block per setting
template <int NC>
__global__ void k_moments_final(const double* __restrict__ part, int nblocks, const SettingDev* __restrict__ set,
                                double* __restrict__ mom, double* __restrict__ emit) {
    __shared__ double sm[MOM_N * NC];
    const int sb = blockIdx.x;
    const double inv_n = set[sb].n > 0 ? 1.0 / (double)set[sb].n : 0.0;
    part += (size_t)sb * nblocks * MOM_N * NC;
    mom += (size_t)sb * MOM_N * NC;
    emit += (size_t)sb * 6 * NC;
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
    int64_t nmax = 0;
    for (int b = 0; b < cx->B; ++b) nmax = nmax > cx->nb[b] ? nmax : cx->nb[b];
    const int64_t want = (nmax * cx->NC + MOM_THREADS - 1) / MOM_THREADS;
    const int cap_blocks = mom_blocks_for(cx->B);
    const int nblocks = (int)(want < cap_blocks ? (want < 1 ? 1 : want) : cap_blocks);
    hipStream_t s = cx->stream;
    const Workspace& w = cx->ws;
    const int64_t cap = cx->dims.n_particles;
    const dim3 g1(nblocks, cx->B), g2(cx->B);
    switch (cx->NC) {
        case 1:
            hipLaunchKernelGGL(k_moments_partial<1>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, w.mom_part);
            hipLaunchKernelGGL(k_moments_final<1>, g2, dim3(256), 0, s, w.mom_part, nblocks, w.set, w.mom, w.emit);
            break;
        case 8:
            hipLaunchKernelGGL(k_moments_partial<8>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, w.mom_part);
            hipLaunchKernelGGL(k_moments_final<8>, g2, dim3(256), 0, s, w.mom_part, nblocks, w.set, w.mom, w.emit);
            break;
        default:
            hipLaunchKernelGGL(k_moments_partial<16>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, w.mom_part);
            hipLaunchKernelGGL(k_moments_final<16>, g2, dim3(256), 0, s, w.mom_part, nblocks, w.set, w.mom, w.emit);
            break;
    }
    return hipGetLastError();
}

}  // namespace dpic
