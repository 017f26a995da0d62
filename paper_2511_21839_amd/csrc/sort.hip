// Particle re-ordering by grid tile (counting sort), run every k steps.
//
// Particles that share a tile of TILE_EDGE^3 cells become neighbours in
// memory, so the gather reads and the deposit atomics of a wavefront hit a
// few cache lines of E and rho instead of scattering over the whole grid.
// Key = tile index of the particle's cell; particles outside the box go to a
// final bin. The scatter is a counting sort (histogram, exclusive scan,
// atomic slot claim per bin); the order inside a bin is not fixed. The
// original particle index travels with the state so read-back stays in the
// original order.
#include "context.hpp"

namespace dpic {

constexpr int TILE_EDGE = 4;

struct SortGeom {
    double lo0, lo1, lo2, ih0, ih1, ih2;
    int nx, ny, nz;
    int tx, ty, tz;  // tiles per dimension
    int nbins;       // tx*ty*tz + 1
};

__device__ __forceinline__ uint32_t tile_key(double x, double y, double z, const SortGeom& g) {
    const double sx = (x - g.lo0) * g.ih0, sy = (y - g.lo1) * g.ih1, sz = (z - g.lo2) * g.ih2;
    const bool inside = (sx >= 0.0) && (sx < (double)(g.nx - 1)) && (sy >= 0.0) && (sy < (double)(g.ny - 1)) &&
                        (sz >= 0.0) && (sz < (double)(g.nz - 1));
    if (!inside) return (uint32_t)(g.nbins - 1);
    const int ix = (int)sx / TILE_EDGE, iy = (int)sy / TILE_EDGE, iz = (int)sz / TILE_EDGE;
    return (uint32_t)((iz * g.ty + iy) * g.tx + ix);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <int NC>
__global__ void k_sort_keys(const double* __restrict__ st, int64_t n, int64_t cap, SortGeom g,
                            uint32_t* __restrict__ key, uint32_t* __restrict__ hist) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t cs = cap * NC;
    const uint32_t k = tile_key(st[p * NC], st[2 * cs + p * NC], st[4 * cs + p * NC], g);
    key[p] = k;
    atomicAdd(hist + k, 1u);
}

// Exclusive scan of nbins counts (one block of 1024 threads); offsets go to
// hist[nbins..2 nbins) and the per-bin cursors are reset in place.
__global__ void k_sort_scan(uint32_t* __restrict__ hist, int nbins) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (nbins + 1023) / 1024;
    const int b0 = t * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nbins) s += hist[b0 + i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;  // exclusive prefix of this thread's range
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < nbins) {
            const uint32_t c = hist[b];
            hist[nbins + b] = run;
            hist[b] = 0u;
            run += c;
        }
    }
}

template <int NC>
__global__ void k_sort_scatter(const double* __restrict__ st, const int32_t* __restrict__ pid, int64_t n, int64_t cap,
                               const uint32_t* __restrict__ key, uint32_t* __restrict__ hist, int nbins,
                               double* __restrict__ st2, int32_t* __restrict__ pid2) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    const bool valid = p < n;
    uint32_t dst = 0;
    if (valid && c == 0) {
        const uint32_t k = key[p];
        dst = hist[nbins + k] + atomicAdd(hist + k, 1u);
    }
    // the group leader owns the slot; every lane of the group copies its channel
    dst = __shfl(dst, (int)(threadIdx.x & 63) & ~(NC - 1), 64);
    if (!valid) return;
    const int64_t cs = cap * NC;
#pragma unroll
    for (int j = 0; j < 6; ++j) st2[j * cs + (int64_t)dst * NC + c] = st[j * cs + p * NC + c];
    if (c == 0) pid2[dst] = pid[p];
}

hipError_t launch_sort(dpic_ctx* cx) {
    if (cx->n == 0) return hipSuccess;
    SortGeom g;
    g.lo0 = cx->lo[0];
    g.lo1 = cx->lo[1];
    g.lo2 = cx->lo[2];
    g.ih0 = 1.0 / cx->h[0];
    g.ih1 = 1.0 / cx->h[1];
    g.ih2 = 1.0 / cx->h[2];
    g.nx = cx->dims.nx;
    g.ny = cx->dims.ny;
    g.nz = cx->dims.nz;
    g.tx = (g.nx - 1 + TILE_EDGE - 1) / TILE_EDGE;
    g.ty = (g.ny - 1 + TILE_EDGE - 1) / TILE_EDGE;
    g.tz = (g.nz - 1 + TILE_EDGE - 1) / TILE_EDGE;
    g.nbins = g.tx * g.ty * g.tz + 1;
    if (g.nbins > NUM_TILE_BINS_MAX + 1) return hipErrorInvalidValue;
    hipStream_t s = cx->stream;
    const int64_t cap = cx->dims.n_particles;
    hipLaunchKernelGGL(k_fill_u32, dim3((2 * g.nbins + 255) / 256), dim3(256), 0, s, cx->ws.hist, 2 * g.nbins);
    const unsigned pb = (unsigned)((cx->n + 255) / 256);
    const unsigned cb = (unsigned)((cx->n * cx->NC + 255) / 256);
    switch (cx->NC) {
#define DPIC_SORT(NCV)                                                                                               \
    case NCV:                                                                                                        \
        hipLaunchKernelGGL(k_sort_keys<NCV>, dim3(pb), dim3(256), 0, s, cx->ws.st, cx->n, cap, g, cx->ws.key,       \
                           cx->ws.hist);                                                                             \
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, cx->ws.hist, g.nbins);                            \
        hipLaunchKernelGGL(k_sort_scatter<NCV>, dim3(cb), dim3(256), 0, s, cx->ws.st, cx->ws.pid, cx->n, cap,       \
                           cx->ws.key, cx->ws.hist, g.nbins, cx->ws.st2, cx->ws.pid2);                               \
        break;
        DPIC_SORT(1)
        DPIC_SORT(8)
        DPIC_SORT(16)
#undef DPIC_SORT
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* t = cx->ws.st;
    cx->ws.st = cx->ws.st2;
    cx->ws.st2 = t;
    int32_t* q = cx->ws.pid;
    cx->ws.pid = cx->ws.pid2;
    cx->ws.pid2 = q;
    return hipSuccess;
}

}  // namespace dpic
