// Particle re-ordering by grid tile (counting sort) and the chunk work list of
// the tiled particle kernel.
//
// Particles that share a tile of TILE_EDGE^3 cells become neighbours in
// memory, so a workgroup can accumulate their deposit in an LDS copy of the
// tile's nodes and flush it once. Key = tile index of the particle's cell;
// particles outside the box go to a final bin.
//
// Counting sort over nbins keys per setting:
//   count:   each block of SORT_PB particles builds an LDS histogram and adds
//            it into the setting's bin totals;
//   starts:  an exclusive scan of each setting's totals gives every bin's
//            first storage slot;
//   scatter: each block claims a run of slots per bin (global atomics), then
//            its particles take slots in it (LDS atomics) and move with all
//            channels into the second buffer.
// In a run of steps the scatter is usually not a pass of its own: the bins
// are counted (launch_sort_counts) after the particle launch that wrote the
// keys, and the next particle launch stores every particle in its sorted
// slot itself (PF_SCATTER in particles.hip); launch_sort_finish then builds
// the work list and swaps the buffers.
// The order of particles inside a bin is not fixed. The original particle
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
    const CellPos c = grid_cell(x, y, z, g.lo0, g.lo1, g.lo2, g.ih0, g.ih1, g.ih2, g.nx, g.ny, g.nz);
    if (!c.inside) return (uint32_t)(g.nbins - 1);
    return (uint32_t)(((c.iz / TILE_EDGE) * g.ty + c.iy / TILE_EDGE) * g.tx + c.ix / TILE_EDGE);
}

constexpr int SORT_THREADS = 1024;

// Sort block k covers storage segment k, which belongs to setting
// b = owner[k]; its particles occupy slots [lo, hi).
struct SegInfo {
    int b;
    int64_t lo, hi;
};

__device__ __forceinline__ SegInfo seg_info(const SettingDev* set, const int32_t* owner, int64_t k) {
    SegInfo r;
    r.b = owner[k];
    const SettingDev sd = set[r.b];
    r.lo = k * SEG;
    const int64_t end = sd.off + sd.n;
    r.hi = (k + 1) * SEG < end ? (k + 1) * SEG : end;
    return r;
}

// Count: the block's histogram over the bins, added into the setting's
// totals tot[b][bin] (non-empty bins only). FROM_KEYS: the keys were
// written by the particle launch that produced these positions. A block
// counts SPB consecutive segments (one particle of each per thread, loaded
// together), which must belong to one setting: SPB > 1 only with one
// setting. Clearing and flushing the histogram's bins costs more than
// counting one segment, so one setting takes 4 segments per block.
template <int NC, bool FROM_KEYS, int SPB>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_count(const double* __restrict__ st, int64_t cap,
                                                             const SettingDev* __restrict__ set,
                                                             const int32_t* __restrict__ owner, SortGeom g,
                                                             int nsegs, uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ tot) {
    static_assert(SORT_PB == SORT_THREADS, "one particle of a segment per thread");
    __shared__ uint32_t h[NUM_TILE_BINS_MAX + 1];
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS) h[b] = 0u;
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * SPB;
    const SegInfo si = seg_info(set, owner, k0);
    const SettingDev sd = set[si.b];
    const int64_t end = sd.off + sd.n;  // the setting's last slot + 1
    const int64_t cs = cap * NC;
    uint32_t kv[SPB];
    bool in[SPB];
#pragma unroll
    for (int j = 0; j < SPB; ++j) {
        in[j] = false;
        kv[j] = 0u;
        if (k0 + j < nsegs) {
            const int64_t p = (k0 + j) * SEG + threadIdx.x;
            if (p < end) {
                in[j] = true;
                if (FROM_KEYS) {
                    kv[j] = key[p];
                } else {
                    kv[j] = tile_key(st[p * NC], st[2 * cs + p * NC], st[4 * cs + p * NC], g);
                    key[p] = kv[j];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < SPB; ++j)
        if (in[j]) atomicAdd(&h[kv[j]], 1u);
    __syncthreads();
    uint32_t* tb = tot + (int64_t)si.b * g.nbins;
    for (int b = threadIdx.x; b < g.nbins; b += SORT_THREADS)
        if (h[b] != 0u) atomicAdd(tb + b, h[b]);
}

// Exclusive prefix sum over a 1024-thread block: a scan inside each
// wavefront by shuffles, then every thread adds the sums of the wavefronts
// before its own (16 values in LDS, sh[0..15]). *total gets the block's sum.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t x, uint32_t* sh, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t u = sh[i];
        before += i < w ? u : 0u;
        all += u;
    }
    __syncthreads();  // sh is free again for the next scan
    if (total) *total = all;
    return before + v - x;
}

// Starts: one block per setting; its bin totals (cleared here for the next
// count) become the first storage slot of every bin (exclusive scan plus the
// setting's offset), in tot (for the work list) and cur (the slots the
// scatter claims), and its number of work items goes to nitems[b].
__global__ __launch_bounds__(1024) void k_sort_starts(const SettingDev* __restrict__ set, int nbins, int chunk,
                                                      uint32_t* __restrict__ hist, uint32_t* __restrict__ tot,
                                                      uint32_t* __restrict__ cur, uint32_t* __restrict__ nitems) {
    __shared__ uint32_t sh[16];
    const int b = blockIdx.x;
    const int64_t off = set[b].off;
    uint32_t* hb = hist + (int64_t)b * nbins;
    uint32_t* tb = tot + (int64_t)b * nbins;
    uint32_t* cb = cur + (int64_t)b * nbins;
    // at most PS bins per thread; their totals are loaded together (unrolled)
    // and kept in registers for the second loop
    constexpr int PS = (NUM_TILE_BINS_MAX + 1 + 1023) / 1024;
    const int per = (nbins + 1023) / 1024;
    const int f0 = threadIdx.x * per;
    const uint32_t ch = (uint32_t)chunk;
    uint32_t v[PS];
    uint32_t s = 0, si = 0;
#pragma unroll
    for (int i = 0; i < PS; ++i) {
        v[i] = (i < per && f0 + i < nbins) ? hb[f0 + i] : 0u;
        s += v[i];
        si += (v[i] + ch - 1u) / ch;
    }
#pragma unroll
    for (int i = 0; i < PS; ++i)
        if (i < per && f0 + i < nbins) hb[f0 + i] = 0u;
    uint32_t run = (uint32_t)off + block_excl_scan_1024(s, sh, nullptr);
    uint32_t items = 0;
    (void)block_excl_scan_1024(si, sh, &items);
#pragma unroll
    for (int i = 0; i < PS; ++i) {
        const int f = f0 + i;
        if (i < per && f < nbins) {
            tb[f] = run;
            cb[f] = run;
            run += v[i];
        }
    }
    if (threadIdx.x == 0) nitems[b] = items;
}

// Scatter: the block recounts its bins, claims a run of slots per non-empty
// bin from cur, then every particle takes the next slot of its bin (LDS
// atomics) and moves there with all channels.
template <int NC>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const double* __restrict__ st,
                                                               const int32_t* __restrict__ pid, int64_t cap,
                                                               const SettingDev* __restrict__ set,
                                                               const int32_t* __restrict__ owner,
                                                               const uint32_t* __restrict__ key,
                                                               uint32_t* __restrict__ cur, int nbins,
                                                               double* __restrict__ st2, int32_t* __restrict__ pid2) {
    __shared__ uint32_t h[NUM_TILE_BINS_MAX + 1];
    for (int b = threadIdx.x; b < nbins; b += SORT_THREADS) h[b] = 0u;
    __syncthreads();
    const SegInfo si = seg_info(set, owner, blockIdx.x);
    for (int i = threadIdx.x; i < SORT_PB; i += SORT_THREADS) {
        const int64_t p = si.lo + i;
        if (p < si.hi) atomicAdd(&h[key[p]], 1u);
    }
    __syncthreads();
    uint32_t* cb = cur + (int64_t)si.b * nbins;
    for (int b = threadIdx.x; b < nbins; b += SORT_THREADS)
        if (h[b] != 0u) h[b] = atomicAdd(cb + b, h[b]);
    __syncthreads();
    const int64_t cs = cap * NC;
    // lanes in groups of NC: the group leader claims the slot, every lane copies its channel
    for (int i = threadIdx.x; i < SORT_PB * NC; i += SORT_THREADS) {
        const int64_t p = si.lo + i / NC;
        const int c = i % NC;
        const bool valid = p < si.hi;
        uint32_t dst = 0;
        if (valid && c == 0) dst = atomicAdd(&h[key[p]], 1u);
        dst = __shfl(dst, (int)(threadIdx.x & 63) & ~(NC - 1), 64);
        if (valid) {
            const int64_t d = (int64_t)dst;
            // the state streams through once: nontemporal, like the particle kernel's accesses
#pragma unroll
            for (int j = 0; j < 6; ++j)
                __builtin_nontemporal_store(__builtin_nontemporal_load(st + j * cs + p * NC + c), st2 + j * cs + d * NC + c);
            if (c == 0) pid2[d] = pid[p];
        }
    }
}

// Cuts bins into work items and writes them in bin order from item index
// base on: s_start[f] is bin f's first slot (s_start[nbins] the end of the
// last), s_item[f] its first item index (s_item[nbins] the item count).
// Each thread finds its item's bin by bisection.
__device__ __forceinline__ void write_items(const uint32_t* s_start, const uint32_t* s_item, int nbins, uint32_t ch,
                                            int setting, uint32_t base, int4* __restrict__ chunks) {
    const uint32_t items = s_item[nbins];
    for (uint32_t k = threadIdx.x; k < items; k += 1024) {
        int lo = 0, hi = nbins - 1;  // s_item[lo] <= k; the bin is the last such
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_item[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t q = s_start[lo] + (k - s_item[lo]) * ch;
        const uint32_t left = s_start[lo + 1] - q;
        chunks[base + k] = make_int4(lo, (int)q, (int)(left < ch ? left : ch), setting);
    }
}

// Batches: one block per setting writes its work items after those of the
// settings before it (their counts from k_sort_starts), from its bins' first
// slots in tot. Item (tile, first slot, count, setting), at most `chunk`
// particles each.
__global__ __launch_bounds__(1024) void k_build_items(const SettingDev* __restrict__ set, int nbins, int chunk,
                                                      const uint32_t* __restrict__ tot,
                                                      const uint32_t* __restrict__ nitems, int nb,
                                                      int4* __restrict__ chunks, uint32_t* __restrict__ nchunks) {
    constexpr int PP = (NUM_TILE_BINS_MAX + 1 + 1023) / 1024;
    __shared__ uint32_t sh[16];
    __shared__ uint32_t s_start[NUM_TILE_BINS_MAX + 2], s_item[NUM_TILE_BINS_MAX + 2];
    const int b = blockIdx.x;
    const SettingDev sd = set[b];
    const uint32_t* tb = tot + (int64_t)b * nbins;
    const uint32_t end = (uint32_t)(sd.off + sd.n);
    const uint32_t ch = (uint32_t)chunk;
    uint32_t pre = 0, all = 0;
    for (int j = threadIdx.x; j < nb; j += 1024) {
        const uint32_t u = nitems[j];
        pre += j < b ? u : 0u;
        all += u;
    }
    uint32_t base = 0, total = 0;
    (void)block_excl_scan_1024(pre, sh, &base);
    (void)block_excl_scan_1024(all, sh, &total);
    const int per = (nbins + 1023) / 1024;
    const int f0 = threadIdx.x * per;
    uint32_t st[PP], c[PP];
    uint32_t si = 0;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int f = f0 + i;
        const bool in = i < per && f < nbins;
        st[i] = in ? tb[f] : 0u;
        c[i] = in ? (f + 1 < nbins ? tb[f + 1] : end) - st[i] : 0u;
        si += (c[i] + ch - 1u) / ch;
    }
    uint32_t items = 0;
    uint32_t irun = block_excl_scan_1024(si, sh, &items);
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int f = f0 + i;
        if (i < per && f < nbins) {
            s_start[f] = st[i];
            s_item[f] = irun;
            irun += (c[i] + ch - 1u) / ch;
        }
    }
    if (threadIdx.x == 0) {
        s_start[nbins] = end;
        s_item[nbins] = items;
        if (b == 0) *nchunks = total;
    }
    __syncthreads();
    write_items(s_start, s_item, nbins, ch, b, base, chunks);
}

// One setting: the starts and the work list in one block. Every bin's total
// (cleared here for the next count) gives its first slot, in tot and cur as
// k_sort_starts writes them. The work list keeps bin order; item sizes follow
// guide zones over the setting's sorted slots: with n particles and D
// resident workgroups, zone z (size chunk / 2^z, at least CHUNK_MIN) holds
// the slots whose remaining count n - P lies in [size_z D, size_(z-1) D),
// the last zone everything after. Each bin's range is cut at the zone
// boundaries and each piece into items of its zone's size. All threads then
// write the items, each finding its item's bin by bisection over the bins'
// first item indices and its piece by walking the zones.
struct GuideZones {
    uint32_t size[GUIDE_LEVELS];
    uint32_t start[GUIDE_LEVELS + 1];  // first slot of each zone (relative to the setting), then n
    __device__ GuideZones(uint32_t n, uint32_t chunk, uint32_t slots) {
        for (int z = 0; z < GUIDE_LEVELS; ++z) {
            const uint32_t c = chunk >> z;
            size[z] = c > (uint32_t)CHUNK_MIN ? c : (uint32_t)CHUNK_MIN;
        }
        start[0] = 0u;
        for (int z = 1; z < GUIDE_LEVELS; ++z) {
            const uint64_t keep = (uint64_t)size[z - 1] * slots;  // remaining count that ends zone z - 1
            const uint32_t p = keep >= n ? 0u : (uint32_t)(n - keep);
            start[z] = p > start[z - 1] ? p : start[z - 1];
        }
        start[GUIDE_LEVELS] = n;
    }
    // items of the slot range [a, e)
    __device__ uint32_t items(uint32_t a, uint32_t e) const {
        uint32_t k = 0;
        for (int z = 0; z < GUIDE_LEVELS; ++z) {
            const uint32_t lo = a > start[z] ? a : start[z], hi = e < start[z + 1] ? e : start[z + 1];
            if (hi > lo) k += (hi - lo + size[z] - 1u) / size[z];
        }
        return k;
    }
    // item j of the range [a, e): first slot and count
    __device__ void item(uint32_t a, uint32_t e, uint32_t j, uint32_t* q, uint32_t* cnt) const {
        for (int z = 0; z < GUIDE_LEVELS; ++z) {
            const uint32_t lo = a > start[z] ? a : start[z], hi = e < start[z + 1] ? e : start[z + 1];
            if (hi <= lo) continue;
            const uint32_t nz = (hi - lo + size[z] - 1u) / size[z];
            if (j < nz) {
                *q = lo + j * size[z];
                const uint32_t left = hi - *q;
                *cnt = left < size[z] ? left : size[z];
                return;
            }
            j -= nz;
        }
        *q = e;
        *cnt = 0u;
    }
};

__global__ __launch_bounds__(1024) void k_sort_plan(const SettingDev* __restrict__ set, int nbins, int chunk, int slots,
                                                    uint32_t* __restrict__ hist, uint32_t* __restrict__ tot,
                                                    uint32_t* __restrict__ cur, int4* __restrict__ chunks,
                                                    uint32_t* __restrict__ nchunks) {
    constexpr int PP = (NUM_TILE_BINS_MAX + 1 + 1023) / 1024;
    __shared__ uint32_t sh[16];
    __shared__ uint32_t s_start[NUM_TILE_BINS_MAX + 2], s_item[NUM_TILE_BINS_MAX + 2];
    const SettingDev sd = set[0];
    const uint32_t off = (uint32_t)sd.off, n = (uint32_t)sd.n;
    const GuideZones gz(n, (uint32_t)chunk, (uint32_t)slots);
    const int per = (nbins + 1023) / 1024;
    const int f0 = threadIdx.x * per;
    uint32_t c[PP];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int f = f0 + i;
        c[i] = (i < per && f < nbins) ? hist[f] : 0u;
        s += c[i];
    }
#pragma unroll
    for (int i = 0; i < PP; ++i)
        if (i < per && f0 + i < nbins) hist[f0 + i] = 0u;
    const uint32_t first = block_excl_scan_1024(s, sh, nullptr);  // relative to the setting
    uint32_t si = 0, rel = first;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        si += gz.items(rel, rel + c[i]);
        rel += c[i];
    }
    uint32_t items = 0;
    uint32_t irun = block_excl_scan_1024(si, sh, &items);
    uint32_t run = first;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int f = f0 + i;
        if (i < per && f < nbins) {
            tot[f] = off + run;
            cur[f] = off + run;
            s_start[f] = run;
            s_item[f] = irun;
            irun += gz.items(run, run + c[i]);
            run += c[i];
        }
    }
    if (threadIdx.x == 0) {
        s_start[nbins] = n;
        s_item[nbins] = items;
        *nchunks = items;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < items; k += 1024) {
        int lo = 0, hi = nbins - 1;  // s_item[lo] <= k; the bin is the last such
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_item[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        uint32_t q, cnt;
        gz.item(s_start[lo], s_start[lo + 1], k - s_item[lo], &q, &cnt);
        chunks[k] = make_int4(lo, (int)(off + q), (int)cnt, 0);
    }
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

// Upper bound of the work items: a non-empty (setting, bin) range gives at
// most one short item per guide zone, and every other item holds at least
// CHUNK_MIN particles.
size_t max_chunks(const dpic_ctx* cx) {
    int nbins = 0;
    sort_geometry(cx, nullptr, &nbins);
    size_t bins = 0;
    for (int b = 0; b < cx->B; ++b) bins += (size_t)std::min<int64_t>(cx->nb[b], nbins);
    return GUIDE_LEVELS * bins + (size_t)(cx->n / CHUNK_MIN) + 1;
}

static bool sort_geom(const dpic_ctx* cx, SortGeom* g) {
    int t[3];
    if (!sort_geometry(cx, t, &g->nbins)) return false;
    g->lo0 = cx->lo[0];
    g->lo1 = cx->lo[1];
    g->lo2 = cx->lo[2];
    g->ih0 = 1.0 / cx->h[0];
    g->ih1 = 1.0 / cx->h[1];
    g->ih2 = 1.0 / cx->h[2];
    g->nx = cx->dims.nx;
    g->ny = cx->dims.ny;
    g->nz = cx->dims.nz;
    g->tx = t[0];
    g->ty = t[1];
    g->tz = t[2];
    return true;
}

// Bin totals of every setting (from the stored keys when the last particle
// launch wrote them, else from the positions), then first slots into tot and
// cur and the work list of the sorted order into chunks2. The totals stay
// zero between sorts: the planning kernels clear them.
hipError_t launch_sort_counts(dpic_ctx* cx) {
    SortGeom g;
    if (!sort_geom(cx, &g)) return hipErrorInvalidValue;
    hipStream_t s = cx->stream;
    const int64_t cap = cx->dims.n_particles;
    const Workspace& w = cx->ws;
    const int nsegs = (int)((cx->used + SEG - 1) / SEG);
    const int64_t nbt = (int64_t)cx->B * g.nbins;
    uint32_t* tot = w.bins;
    uint32_t* cur = w.bins + nbt;
    if (!cx->hist_clean) {
        hipError_t ez = launch_zero(cx, (double*)w.hist, (size_t)(nbt + 1) / 2);
        if (ez != hipSuccess) return ez;
    }
    cx->hist_clean = false;
    if (nsegs > 0) {
        if (cx->keys_ready) {
            if (cx->B == 1)
                hipLaunchKernelGGL((k_sort_count<1, true, 4>), dim3((nsegs + 3) / 4), dim3(SORT_THREADS), 0, s, w.st, cap,
                                   w.set, w.owner, g, nsegs, w.key, w.hist);
            else
                hipLaunchKernelGGL((k_sort_count<1, true, 1>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set,
                                   w.owner, g, nsegs, w.key, w.hist);
        } else {
            switch (cx->NC) {
                case 1: hipLaunchKernelGGL((k_sort_count<1, false, 1>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, nsegs, w.key, w.hist); break;
                case 8: hipLaunchKernelGGL((k_sort_count<8, false, 1>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, nsegs, w.key, w.hist); break;
                default: hipLaunchKernelGGL((k_sort_count<16, false, 1>), dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, cap, w.set, w.owner, g, nsegs, w.key, w.hist); break;
            }
        }
    }
    if (cx->B == 1) {
        hipLaunchKernelGGL(k_sort_plan, dim3(1), dim3(1024), 0, s, w.set, g.nbins, (int)cx->chunk, cx->part_slots,
                           w.hist, tot, cur, w.chunks2, w.nchunks2);
    } else {
        hipLaunchKernelGGL(k_sort_starts, dim3(cx->B), dim3(1024), 0, s, w.set, g.nbins, (int)cx->chunk, w.hist, tot,
                           cur, w.nitems);
        hipLaunchKernelGGL(k_build_items, dim3(cx->B), dim3(1024), 0, s, w.set, g.nbins, (int)cx->chunk, tot, w.nitems,
                           cx->B, w.chunks2, w.nchunks2);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) cx->hist_clean = true;
    return e;
}

// scattered: a particle launch has already stored the state in sorted order
// in the second buffers; otherwise the scatter kernel moves it there. Then
// the state, the original rows and the work list swap with their second
// buffers.
hipError_t launch_sort_finish(dpic_ctx* cx, bool scattered) {
    SortGeom g;
    if (!sort_geom(cx, &g)) return hipErrorInvalidValue;
    hipStream_t s = cx->stream;
    const int64_t cap = cx->dims.n_particles;
    const Workspace& w = cx->ws;
    const int nsegs = (int)((cx->used + SEG - 1) / SEG);
    uint32_t* cur = w.bins + (int64_t)cx->B * g.nbins;
    if (nsegs > 0 && !scattered) {
        switch (cx->NC) {
            case 1: hipLaunchKernelGGL(k_sort_scatter<1>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, cur, g.nbins, w.st2, w.pid2); break;
            case 8: hipLaunchKernelGGL(k_sort_scatter<8>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, cur, g.nbins, w.st2, w.pid2); break;
            default: hipLaunchKernelGGL(k_sort_scatter<16>, dim3(nsegs), dim3(SORT_THREADS), 0, s, w.st, w.pid, cap, w.set, w.owner, w.key, cur, g.nbins, w.st2, w.pid2); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    swap_sorted_buffers(cx->ws);
    cx->swapped = !cx->swapped;
    cx->chunks_valid = true;
    cx->keys_ready = false;
    return hipSuccess;
}

hipError_t launch_sort(dpic_ctx* cx) {
    hipError_t e = launch_sort_counts(cx);
    if (e != hipSuccess) return e;
    return launch_sort_finish(cx, false);
}

}  // namespace dpic
