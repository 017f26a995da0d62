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
// Batches: each setting is sorted within its own storage range (see
// k_sort_count); bins are per setting.
//
// Work list: every bin's particle range is cut into chunks of at most
// `chunk` particles; chunk = (tile, first slot, count, setting).
#include <algorithm>

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

// Sort block k covers storage segment k, which belongs to setting
// b = owner[k]. Its column of counts sits at
// nbins * seg0_b + bin * nseg_b + (k - seg0_b) (seg0_b = off_b / SEG, nseg_b
// the setting's segments): the array is ordered [setting][bin][segment], so
// one exclusive scan over it gives every particle's packed destination.
struct SegInfo {
    int b;
    int64_t lo, hi;       // slots of this segment holding particles
    int64_t col, nseg;    // counts index of (bin 0, this segment), segments of the setting
    int64_t delta;
};

__device__ __forceinline__ SegInfo seg_info(const SettingDev* set, const int32_t* owner, int nbins, int64_t k) {
    SegInfo r;
    r.b = owner[k];
    const SettingDev sd = set[r.b];
    const int64_t seg0 = sd.off / SEG;
    r.nseg = (sd.n + SEG - 1) / SEG;
    r.lo = k * SEG;
    const int64_t end = sd.off + sd.n;
    r.hi = (k + 1) * SEG < end ? (k + 1) * SEG : end;
    r.col = (int64_t)nbins * seg0 + (k - seg0);
    r.delta = sd.delta;
    return r;
}

// FROM_KEYS: the keys were written by the particle launch that produced
// these positions; only the histogram is built.
template <int NC, bool FROM_KEYS>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_count(const double* __restrict__ st, int64_t cap,
                                                             const SettingDev* __restrict__ set,
                                                             const int32_t* __restrict__ owner, SortGeom g,
                                                             uint32_t* __restrict__ key, uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[NUM_TILE_BINS_MAX + 1];
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS) h[b] = 0u;
    __syncthreads();
    const SegInfo si = seg_info(set, owner, g.nbins, blockIdx.x);
    const int64_t cs = cap * NC;
    for (int i = threadIdx.x; i < SORT_PB; i += SORT_THREADS) {
        const int64_t p = si.lo + i;
        if (p < si.hi) {
            uint32_t k;
            if (FROM_KEYS) {
                k = key[p];
            } else {
                k = tile_key(st[p * NC], st[2 * cs + p * NC], st[4 * cs + p * NC], g);
                key[p] = k;
            }
            atomicAdd(&h[k], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS) counts[si.col + (int64_t)b * si.nseg] = h[b];
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
                                                               const int32_t* __restrict__ pid, int64_t cap,
                                                               const SettingDev* __restrict__ set,
                                                               const int32_t* __restrict__ owner,
                                                               const uint32_t* __restrict__ key,
                                                               const uint32_t* __restrict__ offs, int nbins,
                                                               double* __restrict__ st2, int32_t* __restrict__ pid2) {
    __shared__ uint32_t cur[NUM_TILE_BINS_MAX + 1];
    const SegInfo si = seg_info(set, owner, nbins, blockIdx.x);
    for (int b = threadIdx.x; b < nbins; b += SORT_THREADS) cur[b] = offs[si.col + (int64_t)b * si.nseg];
    __syncthreads();
    const int64_t cs = cap * NC;
    // lanes in groups of NC: the group leader claims the slot, every lane copies its channel
    for (int i = threadIdx.x; i < SORT_PB * NC; i += SORT_THREADS) {
        const int64_t p = si.lo + i / NC;
        const int c = i % NC;
        const bool valid = p < si.hi;
        uint32_t dst = 0;
        if (valid && c == 0) dst = atomicAdd(&cur[key[p]], 1u);
        dst = __shfl(dst, (int)(threadIdx.x & 63) & ~(NC - 1), 64);
        if (valid) {
            const int64_t d = (int64_t)dst + si.delta;  // packed position -> storage slot
#pragma unroll
            for (int j = 0; j < 6; ++j) st2[j * cs + d * NC + c] = st[j * cs + p * NC + c];
            if (c == 0) pid2[d] = pid[p];
        }
    }
}

// One block: work list from the bin ranges of every setting. Flattened bin
// f = b * nbins + bin holds slots [start(b, bin), start(b, bin + 1)), the
// last bin ending at off_b + n_b; each range is cut into items of at most
// `chunk` particles: (tile, first slot, count, setting).
__device__ __forceinline__ void bin_range(const SettingDev* set, const uint32_t* offs, int nbins, int f, int64_t* a,
                                          int64_t* e) {
    const int b = f / nbins, bin = f - b * nbins;
    const SettingDev sd = set[b];
    const int64_t nseg = (sd.n + SEG - 1) / SEG;
    if (nseg == 0) {
        *a = *e = 0;
        return;
    }
    const int64_t base = (int64_t)nbins * (sd.off / SEG);
    *a = (int64_t)offs[base + (int64_t)bin * nseg] + sd.delta;
    *e = bin + 1 < nbins ? (int64_t)offs[base + (int64_t)(bin + 1) * nseg] + sd.delta : sd.off + sd.n;
}

__global__ __launch_bounds__(1024) void k_build_chunks(const SettingDev* __restrict__ set,
                                                       const uint32_t* __restrict__ offs, int nbins, int nb,
                                                       int chunk, int4* __restrict__ chunks,
                                                       uint32_t* __restrict__ nchunks) {
    __shared__ uint32_t sh[1024];
    const int nf = nbins * nb;
    const int per = (nf + 1023) / 1024;
    const int f0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i) {
        const int f = f0 + i;
        if (f < nf) {
            int64_t a, e;
            bin_range(set, offs, nbins, f, &a, &e);
            s += (uint32_t)((e - a + chunk - 1) / chunk);
        }
    }
    uint32_t total = 0;
    uint32_t run = block_excl_scan_1024(s, sh, &total);
    for (int i = 0; i < per; ++i) {
        const int f = f0 + i;
        if (f < nf) {
            int64_t a, e;
            bin_range(set, offs, nbins, f, &a, &e);
            const int b = f / nbins;
            for (int64_t q = a; q < e; q += chunk) {
                const int64_t cnt = (e - q) < chunk ? (e - q) : chunk;
                chunks[run++] = make_int4(f - b * nbins, (int)q, (int)cnt, b);
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

// Upper bound of the work items: every non-empty (setting, bin) range gives
// at most one item more than its particles / chunk.
size_t max_chunks(const dpic_ctx* cx) {
    int nbins = 0;
    sort_geometry(cx, nullptr, &nbins);
    size_t bins = 0;
    for (int b = 0; b < cx->B; ++b) bins += (size_t)std::min<int64_t>(cx->nb[b], nbins);
    return bins + (size_t)(cx->n / cx->chunk) + 1;
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
    const Workspace& w = cx->ws;
    const int nsegs = (int)((cx->used + SEG - 1) / SEG);
    const int64_t m = (int64_t)g.nbins * nsegs;
    const int nscan = (int)((m + SCAN_SEG - 1) / SCAN_SEG);
    if (nsegs > 0) {
        if (cx->keys_ready) {
            hipLaunchKernelGGL((k_sort_count<1, true>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, w.key,
                               w.counts);
        } else {
            switch (cx->NC) {
                case 1: hipLaunchKernelGGL((k_sort_count<1, false>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, w.key, w.counts); break;
                case 8: hipLaunchKernelGGL((k_sort_count<8, false>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, w.key, w.counts); break;
                default: hipLaunchKernelGGL((k_sort_count<16, false>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, w.key, w.counts); break;
            }
        }
        hipLaunchKernelGGL(k_scan_seg_sums, dim3(nscan), dim3(1024), 0, s, w.counts, m, w.seg);
        hipLaunchKernelGGL(k_scan_seg_offsets, dim3(1), dim3(1024), 0, s, w.seg, nscan);
        hipLaunchKernelGGL(k_scan_apply, dim3(nscan), dim3(1024), 0, s, w.counts, m, w.seg);
        switch (cx->NC) {
            case 1: hipLaunchKernelGGL(k_sort_scatter<1>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, w.counts, g.nbins, w.st2, w.pid2); break;
            case 8: hipLaunchKernelGGL(k_sort_scatter<8>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, w.counts, g.nbins, w.st2, w.pid2); break;
            default: hipLaunchKernelGGL(k_sort_scatter<16>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, w.counts, g.nbins, w.st2, w.pid2); break;
        }
    }
    hipLaunchKernelGGL(k_build_chunks, dim3(1), dim3(1024), 0, s, w.set, w.counts, g.nbins, cx->B, (int)cx->chunk,
                       w.chunks, w.nchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nsegs > 0) {
        std::swap(cx->ws.st, cx->ws.st2);
        std::swap(cx->ws.pid, cx->ws.pid2);
        cx->swapped = !cx->swapped;
    }
    cx->chunks_valid = true;
    cx->keys_ready = false;
    return hipSuccess;
}

}  // namespace dpic
