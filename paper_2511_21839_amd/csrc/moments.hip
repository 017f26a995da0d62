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
#include <stdio.h>

#include <mutex>

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

// partial-sum blocks per setting for the context's current beams
static int moment_blocks(const dpic_ctx* cx) {
    int64_t nmax = 0;
    for (int b = 0; b < cx->B; ++b) nmax = nmax > cx->nb[b] ? nmax : cx->nb[b];
    const int64_t want = (nmax * cx->NC + MOM_THREADS - 1) / MOM_THREADS;
    const int cap_blocks = mom_blocks_for(cx->B);
    return (int)(want < cap_blocks ? (want < 1 ? 1 : want) : cap_blocks);
}

// partials [B][nblocks][MOM_N][NC], moments [B][MOM_N][NC], emittances [B][2][3][NC]
static hipError_t launch_moments_into(dpic_ctx* cx, int nblocks, double* part, double* mom, double* emit) {
    hipStream_t s = cx->stream;
    const Workspace& w = cx->ws;
    const int64_t cap = cx->dims.n_particles;
    const dim3 g1(nblocks, cx->B), g2(cx->B);
    switch (cx->NC) {
        case 1:
            hipLaunchKernelGGL(k_moments_partial<1>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, part);
            hipLaunchKernelGGL(k_moments_final<1>, g2, dim3(256), 0, s, part, nblocks, w.set, mom, emit);
            break;
        case 8:
            hipLaunchKernelGGL(k_moments_partial<8>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, part);
            hipLaunchKernelGGL(k_moments_final<8>, g2, dim3(256), 0, s, part, nblocks, w.set, mom, emit);
            break;
        default:
            hipLaunchKernelGGL(k_moments_partial<16>, g1, dim3(MOM_THREADS), 0, s, w.st, cap, w.set, part);
            hipLaunchKernelGGL(k_moments_final<16>, g2, dim3(256), 0, s, part, nblocks, w.set, mom, emit);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_moments(dpic_ctx* cx) {
    return launch_moments_into(cx, moment_blocks(cx), cx->ws.mom_part, cx->ws.mom, cx->ws.emit);
}

// ---------------------------------------------------------------- allocation-free read-back
// The emittance read-back of dpic_read_emittance_noalloc stages its partial
// sums, moments and emittance duals in this array (one copy per device,
// held until the process ends) instead of the context workspace, and writes
// its result to caller device memory. Host code never uses the array's name
// as an address: it takes the device address from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[NOALLOC_MAX_DEVICES];

// emit [B][2][3][NC] -> out [B][3][1 + ntan] (raw or centred), zeros for an
// empty setting; one block per setting
template <int NC>
__global__ void k_emittance_out(const double* __restrict__ emit, const SettingDev* __restrict__ set, int ntan,
                                int centred, double* __restrict__ out) {
    const int b = blockIdx.x;
    const bool empty = set[b].n == 0;
    const double* e = emit + ((size_t)b * 6 + (centred ? 3 : 0)) * NC;
    double* o = out + (size_t)b * 3 * (ntan + 1);
    for (int i = threadIdx.x; i < 3 * (ntan + 1); i += blockDim.x) {
        const int pl = i / (ntan + 1), ch = i % (ntan + 1);
        o[i] = empty ? 0.0 : e[pl * NC + ch];
    }
}

}  // namespace dpic

using namespace dpic;

extern "C" int dpic_read_emittance_noalloc(dpic_ctx* c, int centred, double* out_dev) {
    if (!c || !out_dev) return DPIC_EINVAL;
    if (!c->beam_init) {
        c->err = "read_emittance_noalloc: no beam";
        return DPIC_ESTATE;
    }
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES) {
        c->err = "read_emittance_noalloc: device index beyond the library's table";
        return DPIC_EUNSUPPORTED;
    }
    const int nblocks = moment_blocks(c);
    const size_t per = (size_t)c->B * c->NC;
    const size_t need = (per * nblocks * MOM_N + per * MOM_N + per * 6) * sizeof(double);
    if (need > NOALLOC_SCRATCH_BYTES) {
        char buf[160];
        snprintf(buf, sizeof buf, "read_emittance_noalloc: needs %zu bytes of scratch, the static array holds %zu",
                 need, NOALLOC_SCRATCH_BYTES);
        c->err = buf;
        return DPIC_EINVAL;
    }
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[c->device]) {
            int cur = 0;
            hipError_t e = hipGetDevice(&cur);
            if (e == hipSuccess && cur != c->device) e = hipSetDevice(c->device);
            void* p = nullptr;
            if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (cur != c->device) (void)hipSetDevice(cur);
            if (e != hipSuccess || !p) {
                c->err = std::string("read_emittance_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e);
                return DPIC_EHIP;
            }
            g_scratch_dev[c->device] = (double*)p;
        }
        base = g_scratch_dev[c->device];
    }
    double* part = base;
    double* mom = part + per * nblocks * MOM_N;
    double* emit = mom + per * MOM_N;
    hipError_t e = launch_moments_into(c, nblocks, part, mom, emit);
    if (e == hipSuccess) {
        switch (c->NC) {
            case 1: hipLaunchKernelGGL(k_emittance_out<1>, dim3(c->B), dim3(64), 0, c->stream, emit, c->ws.set, c->ntan, centred, out_dev); break;
            case 8: hipLaunchKernelGGL(k_emittance_out<8>, dim3(c->B), dim3(64), 0, c->stream, emit, c->ws.set, c->ntan, centred, out_dev); break;
            default: hipLaunchKernelGGL(k_emittance_out<16>, dim3(c->B), dim3(64), 0, c->stream, emit, c->ws.set, c->ntan, centred, out_dev); break;
        }
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        c->err = std::string("read_emittance_noalloc: ") + hipGetErrorString(e);
        return DPIC_EHIP;
    }
    return DPIC_OK;
}
