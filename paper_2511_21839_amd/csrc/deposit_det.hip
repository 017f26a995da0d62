// Deterministic charge deposit: the cloud-in-cell assignment of rho and of
// its derivative arrays (Sec. 4) summed in a fixed order, so that repeated
// runs give bit-identical node charges and therefore bit-identical steps.
//
// The fused particle kernel adds its contributions with floating-point
// atomics, in whatever order the hardware applies them; addition does not
// associate, so the last bits of rho, and everything computed from it, vary
// between runs. This path has no floating-point atomics:
//   keys:   every stored particle gets (setting * nodes + base node) << 32 |
//           storage slot, the base node being the lower corner of its cell,
//           or ~0 when it is outside the box;
//   sort:   a bitonic sorting network over the keys, a data-independent
//           sequence of compare-exchanges, so the same keys always come out in
//           the same order; passes with partner distance below one LDS block
//           run inside the block;
//   starts: the particles with base node s = setting * nodes + node are the
//           sorted positions [start[s], start[s + 1]), found by binary search;
//   sum:    one workgroup per (setting, node) adds the shares of the 8 cells
//           around its node in a fixed order (below) and stores the sum.
// Each particle is read once per corner, so the mode costs several times the
// atomic deposit: it is a reproducibility witness, not the production path.
//
// Buffers: the keys take the second state buffer (unused while the mode
// keeps the stored order fixed) and the segment starts the first FFT work
// array (the solve that follows overwrites it), so the mode needs no memory
// of its own.
#include "context.hpp"

namespace dpic {

constexpr int DET_BLOCK = 2048;  // keys one workgroup sorts in LDS
constexpr uint64_t DET_OUTSIDE = ~0ull;

struct DetGeom {
    double lo0, lo1, lo2, ih0, ih1, ih2;
    int nx, ny, nz;
    int64_t nodes;
};

__global__ void k_det_keys(const double* __restrict__ st, int64_t cap, int64_t used, int NC,
                           const SettingDev* __restrict__ set, const int32_t* __restrict__ owner, DetGeom g,
                           uint64_t* __restrict__ keys, int64_t n2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n2) return;
    uint64_t key = DET_OUTSIDE;
    if (p < used) {
        const int b = owner[p / SEG];
        const SettingDev& sd = set[b];
        if (p - sd.off < sd.n) {
            const CellPos c = grid_cell(st[p * NC], st[(2 * cap + p) * NC], st[(4 * cap + p) * NC], g.lo0, g.lo1,
                                        g.lo2, g.ih0, g.ih1, g.ih2, g.nx, g.ny, g.nz);
            if (c.inside) {
                const int64_t node = ((int64_t)c.iz * g.ny + c.iy) * g.nx + c.ix;
                key = ((uint64_t)(b * g.nodes + node) << 32) | (uint64_t)p;
            }
        }
    }
    keys[p] = key;
}

__device__ __forceinline__ void det_cmpx(uint64_t& a, uint64_t& b, bool ascending) {
    if ((a > b) == ascending) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
}

// Stages k = k_lo, 2 k_lo, ..., k_hi of the network, restricted to partner
// distances below the block (L keys, L / 2 threads, one compare-exchange per
// thread and pass). Directions come from the global index, so a block takes
// part in merges wider than itself.
__global__ __launch_bounds__(DET_BLOCK / 2) void k_det_sort_local(uint64_t* __restrict__ keys, int L, int64_t k_lo,
                                                                 int64_t k_hi) {
    __shared__ uint64_t s[DET_BLOCK];
    const int t = threadIdx.x, half = L / 2;
    const int64_t base = (int64_t)blockIdx.x * L;
    s[t] = keys[base + t];
    s[t + half] = keys[base + t + half];
    __syncthreads();
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int j = (int)(k / 2 < half ? k / 2 : half); j > 0; j >>= 1) {
            const int i = 2 * j * (t / j) + (t % j);
            uint64_t a = s[i], b = s[i + j];
            det_cmpx(a, b, ((base + i) & k) == 0);
            s[i] = a;
            s[i + j] = b;
            __syncthreads();
        }
    }
    keys[base + t] = s[t];
    keys[base + t + half] = s[t + half];
}

// One pass (stage k, partner distance j >= the block) over all n2 keys.
__global__ void k_det_sort_global(uint64_t* __restrict__ keys, int64_t n2, int64_t k, int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 / 2) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    uint64_t a = keys[i], b = keys[i + j];
    det_cmpx(a, b, (i & k) == 0);
    keys[i] = a;
    keys[i + j] = b;
}

// start[s] = first sorted position whose key is >= s << 32, s = 0 .. nseg.
__global__ void k_det_starts(const uint64_t* __restrict__ keys, int64_t n2, int64_t nseg,
                             uint32_t* __restrict__ start) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nseg) return;
    const uint64_t target = (uint64_t)s << 32;
    int64_t lo = 0, hi = n2;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    start[s] = (uint32_t)lo;
}

// Node charge of one (setting, node): a workgroup walks the particles of the
// 8 cells that have the node as a corner, concatenated cell after cell;
// thread t takes items t, t + DET_SUM_THREADS, ... and sums their shares
// (each particle's CIC weight for this node as a dual) in that order, then
// the threads' sums meet in a fixed butterfly per wavefront and the
// wavefronts in index order. Every step of the order depends only on the
// sorted keys, so the result is the same on every run.
constexpr int DET_SUM_THREADS = 256;

template <int NC>
__global__ __launch_bounds__(DET_SUM_THREADS) void k_det_sum(const double* __restrict__ st, int64_t cap,
                                                             const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ start,
                                                             const SettingDev* __restrict__ set, DetGeom g) {
    __shared__ double red[DET_SUM_THREADS / 64][NC];
    const int b = blockIdx.y;  // setting
    const int64_t node = blockIdx.x;
    const int ix = (int)(node % g.nx), iy = (int)((node / g.nx) % g.ny), iz = (int)(node / ((int64_t)g.nx * g.ny));
    // the 8 cells, corner order (kz, ky, kx); cells off the grid are empty
    uint32_t beg[8], cum[9];
    cum[0] = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int cx = ix - (c & 1), cy = iy - ((c >> 1) & 1), cz = iz - (c >> 2);
        uint32_t n = 0u;
        beg[c] = 0u;
        if (cx >= 0 && cy >= 0 && cz >= 0) {
            const int64_t s = (int64_t)b * g.nodes + ((int64_t)cz * g.ny + cy) * g.nx + cx;
            beg[c] = start[s];
            n = start[s + 1] - beg[c];
        }
        cum[c + 1] = cum[c] + n;
    }
    double* out = set[b].rho + node * NC;
    if (cum[8] == 0u) {
        if (threadIdx.x < NC) out[threadIdx.x] = 0.0;
        return;
    }
    const double q = set[b].q;
    double acc[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.0;
    for (uint32_t j = threadIdx.x; j < cum[8]; j += DET_SUM_THREADS) {
        int c = 0;
#pragma unroll
        for (int k = 1; k < 8; ++k) c += j >= cum[k] ? 1 : 0;
        const int kx = c & 1, ky = (c >> 1) & 1, kz = c >> 2;
        const int64_t p = (int64_t)(keys[beg[c] + (j - cum[c])] & 0xffffffffull);
        const double* xs = st + p * NC;
        const double* ys = st + (2 * cap + p) * NC;
        const double* zs = st + (4 * cap + p) * NC;
        const double sx = (xs[0] - g.lo0) * g.ih0, sy = (ys[0] - g.lo1) * g.ih1, sz = (zs[0] - g.lo2) * g.ih2;
        // the cell's lower corner is (ix - kx, iy - ky, iz - kz); weight factor f or 1 - f per dimension
        const double fx = sx - (double)(ix - kx), fy = sy - (double)(iy - ky), fz = sz - (double)(iz - kz);
        const double ax = kx ? fx : 1.0 - fx, ay = ky ? fy : 1.0 - fy, az = kz ? fz : 1.0 - fz;
        const double sgx = kx ? g.ih0 : -g.ih0, sgy = ky ? g.ih1 : -g.ih1, sgz = kz ? g.ih2 : -g.ih2;
        const double ayz = ay * az;
        acc[0] += (ax * ayz) * q;
#pragma unroll
        for (int ch = 1; ch < NC; ++ch) {
            // d(ax ay az) = dax (ay az) + ax (day az + ay daz)
            const double dyz = fma(ay, zs[ch] * sgz, (ys[ch] * sgy) * az);
            const double w = fma(xs[ch] * sgx, ayz, ax * dyz);
            acc[ch] += w * q;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
        double v = acc[ch];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][ch] = v;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        double v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < DET_SUM_THREADS / 64; ++w) v += red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
}

// Stored order back to the packed original order: the particle in slot p
// (original row pid[p]) moves to slot pid[p] + delta of its setting.
template <int NC>
__global__ void k_det_unsort(const double* __restrict__ st, const int32_t* __restrict__ pid, int64_t used,
                             int64_t cap, const SettingDev* __restrict__ set, const int32_t* __restrict__ owner,
                             double* __restrict__ st2, int32_t* __restrict__ pid2) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= used) return;
    const SettingDev& sd = set[owner[p / SEG]];
    if (p - sd.off >= sd.n) return;
    const int64_t d = (int64_t)pid[p] + sd.delta;
#pragma unroll
    for (int j = 0; j < 6; ++j) st2[((int64_t)j * cap + d) * NC + c] = st[((int64_t)j * cap + p) * NC + c];
    if (c == 0) pid2[d] = pid[p];
}

static int64_t pow2_at_least(int64_t n) {
    int64_t p = 2;
    while (p < n) p <<= 1;
    return p;
}

hipError_t launch_deposit_det(dpic_ctx* cx) {
    const Workspace& w = cx->ws;
    const int NC = cx->NC, B = cx->B;
    const int64_t cap = cx->dims.n_particles;
    DetGeom g;
    g.lo0 = cx->lo[0];
    g.lo1 = cx->lo[1];
    g.lo2 = cx->lo[2];
    g.ih0 = 1.0 / cx->h[0];
    g.ih1 = 1.0 / cx->h[1];
    g.ih2 = 1.0 / cx->h[2];
    g.nx = cx->dims.nx;
    g.ny = cx->dims.ny;
    g.nz = cx->dims.nz;
    g.nodes = (int64_t)grid_nodes(cx);
    const int64_t n2 = pow2_at_least(cx->used);
    const int L = (int)std::min<int64_t>(n2, DET_BLOCK);
    const int64_t nseg = (int64_t)B * g.nodes;
    // room: n2 <= 2 used keys in 48 cap NC bytes; nseg + 1 starts in the FFT
    // array of at least 2 B nodes complex values
    if ((size_t)n2 * sizeof(uint64_t) > (size_t)6 * cap * NC * sizeof(double) || n2 > (1ll << 31) ||
        nseg >= (int64_t)0xffffffffll)
        return hipErrorInvalidValue;
    uint64_t* keys = (uint64_t*)w.st2;
    uint32_t* start = (uint32_t*)w.buf0;
    hipLaunchKernelGGL(k_det_keys, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, cx->stream, w.st, cap, cx->used,
                       NC, w.set, w.owner, g, keys, n2);
    const unsigned lblocks = (unsigned)(n2 / L);
    hipLaunchKernelGGL(k_det_sort_local, dim3(lblocks), dim3(L / 2), 0, cx->stream, keys, L, (int64_t)2, (int64_t)L);
    for (int64_t k = 2 * (int64_t)L; k <= n2; k <<= 1) {
        for (int64_t j = k / 2; j >= L; j >>= 1)
            hipLaunchKernelGGL(k_det_sort_global, dim3((unsigned)((n2 / 2 + 255) / 256)), dim3(256), 0, cx->stream,
                               keys, n2, k, j);
        hipLaunchKernelGGL(k_det_sort_local, dim3(lblocks), dim3(L / 2), 0, cx->stream, keys, L, k, k);
    }
    hipLaunchKernelGGL(k_det_starts, dim3((unsigned)((nseg + 1 + 255) / 256)), dim3(256), 0, cx->stream, keys, n2,
                       nseg, start);
    const dim3 grid((unsigned)g.nodes, (unsigned)B), block(DET_SUM_THREADS);
    switch (NC) {
        case 1: hipLaunchKernelGGL(k_det_sum<1>, grid, block, 0, cx->stream, w.st, cap, keys, start, w.set, g); break;
        case 8: hipLaunchKernelGGL(k_det_sum<8>, grid, block, 0, cx->stream, w.st, cap, keys, start, w.set, g); break;
        default: hipLaunchKernelGGL(k_det_sum<16>, grid, block, 0, cx->stream, w.st, cap, keys, start, w.set, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_unsort(dpic_ctx* cx) {
    const int64_t threads = cx->used * cx->NC;
    if (threads == 0) return hipSuccess;
    const Workspace& w = cx->ws;
    const int64_t cap = cx->dims.n_particles;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_det_unsort<1>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2, w.pid2); break;
        case 8: hipLaunchKernelGGL(k_det_unsort<8>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2, w.pid2); break;
        default: hipLaunchKernelGGL(k_det_unsort<16>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2, w.pid2); break;
    }
    return hipGetLastError();
}

}  // namespace dpic
