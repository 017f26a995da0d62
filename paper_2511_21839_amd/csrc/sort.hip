// Particle re-ordering by grid tile (counting sort) and the chunk work list of
// the tiled particle kernel.
//
// Particles that share a tile of TILE_EDGE^3 cells become neighbours in
// memory, so a workgroup can accumulate their deposit in an LDS copy of the
// tile's nodes and flush it once. Key = tile index of the particle's cell;
// particles outside the box go to a final bin.
//
// Counting sort over nbins keys:
//   count:   each block of SORT_PB particles builds an LDS histogram and writes
//            its column counts[bin][block];
//   scan:    exclusive scan of counts in bin-major order (three kernels);
//   scatter: each block claims slots from its column offsets with LDS atomics
//            and moves the particles (all channels) into the second buffer.
// The order inside one bin of one block is not fixed. The original particle
// index travels with the state so read-back stays in the original order.
//
// Work list: every bin's particle range is cut into chunks of at most
// TILE_CHUNK particles; chunk = (tile, first particle, count).
#include "context.hpp"

namespace dpic {

struct SortGeom {
    double lo0, lo1, lo2, ih0, ih1, ih2;
    int nx, ny, nz;
    int tx, ty, tz;  // tiles per dimension
    int nbins;       // tx*ty*tz + 1 (last bin: outside the box)
};

__device__ __forceinline__ uint32_t tile_key(double x, double y, double z, const SortGeom& g) {
    const double sx = (x - g.lo0) * g.ih0, sy = (y - g.lo1) * g.ih1, sz = (z - g.lo2) * g.ih2;
    const bool inside = (sx >= 0.0) && (sx < (double)(g.nx - 1)) && (sy >= 0.0) && (sy < (double)(g.ny - 1)) &&
                        (sz >= 0.0) && (sz < (double)(g.nz - 1));
    if (!inside) return (uint32_t)(g.nbins - 1);
    const int ix = (int)sx / TILE_EDGE, iy = (int)sy / TILE_EDGE, iz = (int)sz / TILE_EDGE;
    return (uint32_t)((iz * g.ty + iy) * g.tx + ix);
}

constexpr int SORT_THREADS = 1024;

template <int NC>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_count(const double* __restrict__ st, int64_t n, int64_t cap,
                                                             SortGeom g, uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ counts, int nblocks) {
    __shared__ uint32_t h[NUM_TILE_BINS_MAX + 1];
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS) h[b] = 0u;
    __syncthreads();
    const int64_t cs = cap * NC;
    const int64_t p0 = (int64_t)blockIdx.x * SORT_PB;
    for (int i = threadIdx.x; i < SORT_PB; i += SORT_THREADS) {
        const int64_t p = p0 + i;
        if (p < n) {
            const uint32_t k = tile_key(st[p * NC], st[2 * cs + p * NC], st[4 * cs + p * NC], g);
            key[p] = k;
            atomicAdd(&h[k], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS) counts[(int64_t)b * nblocks + blockIdx.x] = h[b];
}

// Exclusive scan of m values in place: per-segment sums, scan of the sums in
// one block, then each segment re-scanned with its offset.
constexpr int SCAN_SEG = 1024;

__global__ __launch_bounds__(1024) void k_scan_seg_sums(const uint32_t* __restrict__ v, int64_t m,
                                                        uint32_t* __restrict__ seg) {
    __shared__ uint32_t red[1024];
    const int64_t i = (int64_t)blockIdx.x * SCAN_SEG + threadIdx.x;
    red[threadIdx.x] = i < m ? v[i] : 0u;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) seg[blockIdx.x] = red[0];
}

__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t x, uint32_t* sh, uint32_t* total) {
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const uint32_t incl = sh[threadIdx.x];
    if (total) *total = sh[1023];
    __syncthreads();
    return incl - x;
}

// one block: exclusive scan of nseg segment sums (any count), in place
__global__ __launch_bounds__(1024) void k_scan_seg_offsets(uint32_t* __restrict__ seg, int nseg) {
    __shared__ uint32_t sh[1024];
    const int per = (nseg + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nseg) s += seg[b0 + i];
    uint32_t run = block_excl_scan_1024(s, sh, nullptr);
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < nseg) {
            const uint32_t c = seg[b];
            seg[b] = run;
            run += c;
        }
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(uint32_t* __restrict__ v, int64_t m,
                                                     const uint32_t* __restrict__ seg) {
    __shared__ uint32_t sh[1024];
    const int64_t i = (int64_t)blockIdx.x * SCAN_SEG + threadIdx.x;
    const uint32_t x = i < m ? v[i] : 0u;
    const uint32_t ex = block_excl_scan_1024(x, sh, nullptr);
    if (i < m) v[i] = ex + seg[blockIdx.x];
}

template <int NC>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const double* __restrict__ st,
                                                               const int32_t* __restrict__ pid, int64_t n,
                                                               int64_t cap, const uint32_t* __restrict__ key,
                                                               const uint32_t* __restrict__ offs, int nbins,
                                                               int nblocks, double* __restrict__ st2,
                                                               int32_t* __restrict__ pid2) {
    __shared__ uint32_t cur[NUM_TILE_BINS_MAX + 1];
    for (int b = threadIdx.x; b < nbins; b += SORT_THREADS) cur[b] = offs[(int64_t)b * nblocks + blockIdx.x];
    __syncthreads();
    const int64_t cs = cap * NC;
    const int64_t p0 = (int64_t)blockIdx.x * SORT_PB;
    // lanes in groups of NC: the group leader claims the slot, every lane copies its channel
    for (int i = threadIdx.x; i < SORT_PB * NC; i += SORT_THREADS) {
        const int64_t p = p0 + i / NC;
        const int c = i % NC;
        const bool valid = p < n;
        uint32_t dst = 0;
        if (valid && c == 0) dst = atomicAdd(&cur[key[p]], 1u);
        dst = __shfl(dst, (int)(threadIdx.x & 63) & ~(NC - 1), 64);
        if (valid) {
#pragma unroll
            for (int j = 0; j < 6; ++j) st2[j * cs + (int64_t)dst * NC + c] = st[j * cs + p * NC + c];
            if (c == 0) pid2[dst] = pid[p];
        }
    }
}

// One block: chunk list from the bin ranges. Bin b holds particles
// [offs[b*nblocks], offs[(b+1)*nblocks]) (n for the last bin).
__global__ __launch_bounds__(1024) void k_build_chunks(const uint32_t* __restrict__ offs, int nbins, int nblocks,
                                                       int64_t n, int4* __restrict__ chunks,
                                                       uint32_t* __restrict__ nchunks) {
    __shared__ uint32_t sh[1024];
    const int per = (nbins + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < nbins) {
            const uint32_t a = offs[(int64_t)b * nblocks];
            const uint32_t e = (b + 1 < nbins) ? offs[(int64_t)(b + 1) * nblocks] : (uint32_t)n;
            s += (e - a + TILE_CHUNK - 1) / TILE_CHUNK;
        }
    }
    uint32_t total = 0;
    uint32_t run = block_excl_scan_1024(s, sh, &total);
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < nbins) {
            const uint32_t a = offs[(int64_t)b * nblocks];
            const uint32_t e = (b + 1 < nbins) ? offs[(int64_t)(b + 1) * nblocks] : (uint32_t)n;
            for (uint32_t q = a; q < e; q += TILE_CHUNK) {
                const uint32_t cnt = (e - q) < (uint32_t)TILE_CHUNK ? (e - q) : (uint32_t)TILE_CHUNK;
                chunks[run++] = make_int4(b, (int)q, (int)cnt, 0);
            }
        }
    }
    if (threadIdx.x == 0) *nchunks = total;
}

bool sort_geometry(const dpic_ctx* cx, int* tiles, int* nbins) {
    int t[3];
    const int n[3] = {cx->dims.nx, cx->dims.ny, cx->dims.nz};
    for (int d = 0; d < 3; ++d) t[d] = (n[d] - 1 + TILE_EDGE - 1) / TILE_EDGE;
    if (tiles)
        for (int d = 0; d < 3; ++d) tiles[d] = t[d];
    *nbins = t[0] * t[1] * t[2] + 1;
    return *nbins <= NUM_TILE_BINS_MAX + 1;
}

hipError_t launch_sort(dpic_ctx* cx) {
    SortGeom g;
    int t[3];
    if (!sort_geometry(cx, t, &g.nbins)) return hipErrorInvalidValue;
    g.lo0 = cx->lo[0];
    g.lo1 = cx->lo[1];
    g.lo2 = cx->lo[2];
    g.ih0 = 1.0 / cx->h[0];
    g.ih1 = 1.0 / cx->h[1];
    g.ih2 = 1.0 / cx->h[2];
    g.nx = cx->dims.nx;
    g.ny = cx->dims.ny;
    g.nz = cx->dims.nz;
    g.tx = t[0];
    g.ty = t[1];
    g.tz = t[2];
    hipStream_t s = cx->stream;
    const int64_t cap = cx->dims.n_particles;
    const int64_t n = cx->n;
    const int nblocks = (int)((n + SORT_PB - 1) / SORT_PB) > 0 ? (int)((n + SORT_PB - 1) / SORT_PB) : 1;
    const int64_t m = (int64_t)g.nbins * nblocks;
    const int nseg = (int)((m + SCAN_SEG - 1) / SCAN_SEG);
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_sort_count<1>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, n, cap, g, cx->ws.key, cx->ws.counts, nblocks); break;
        case 8: hipLaunchKernelGGL(k_sort_count<8>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, n, cap, g, cx->ws.key, cx->ws.counts, nblocks); break;
        default: hipLaunchKernelGGL(k_sort_count<16>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, n, cap, g, cx->ws.key, cx->ws.counts, nblocks); break;
    }
    hipLaunchKernelGGL(k_scan_seg_sums, dim3(nseg), dim3(1024), 0, s, cx->ws.counts, m, cx->ws.seg);
    hipLaunchKernelGGL(k_scan_seg_offsets, dim3(1), dim3(1024), 0, s, cx->ws.seg, nseg);
    hipLaunchKernelGGL(k_scan_apply, dim3(nseg), dim3(1024), 0, s, cx->ws.counts, m, cx->ws.seg);
    if (n > 0) {
        switch (cx->NC) {
            case 1: hipLaunchKernelGGL(k_sort_scatter<1>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, cx->ws.pid, n, cap, cx->ws.key, cx->ws.counts, g.nbins, nblocks, cx->ws.st2, cx->ws.pid2); break;
            case 8: hipLaunchKernelGGL(k_sort_scatter<8>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, cx->ws.pid, n, cap, cx->ws.key, cx->ws.counts, g.nbins, nblocks, cx->ws.st2, cx->ws.pid2); break;
            default: hipLaunchKernelGGL(k_sort_scatter<16>, dim3(nblocks), dim3(SORT_THREADS), 0, s, cx->ws.st, cx->ws.pid, n, cap, cx->ws.key, cx->ws.counts, g.nbins, nblocks, cx->ws.st2, cx->ws.pid2); break;
        }
    }
    hipLaunchKernelGGL(k_build_chunks, dim3(1), dim3(1024), 0, s, cx->ws.counts, g.nbins, nblocks, n, cx->ws.chunks,
                       cx->ws.nchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > 0) {
        double* tmp = cx->ws.st;
        cx->ws.st = cx->ws.st2;
        cx->ws.st2 = tmp;
        int32_t* q = cx->ws.pid;
        cx->ws.pid = cx->ws.pid2;
        cx->ws.pid2 = q;
    }
    cx->chunks_valid = true;
    return hipSuccess;
}

}  // namespace dpic
