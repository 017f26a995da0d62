// Particle-side kernels: per-element dual constants, beam initialisation,
// the fused gather / kick / map / deposit kernel, canonical read-back.
//
// Particle state is SoA over coordinates with the tangents interleaved:
// st[coord][particle][NC]. In the fused step a particle owns a group of
// G = NC / 2 consecutive lanes (G = 1 when NC = 1); lane q of the group holds
// channels 2q, 2q + 1 of every dual plus the value, so one 16-byte load per
// lane moves its part of a coordinate and a wavefront touches one contiguous
// kilobyte. The value reaches the other lanes of the group by DPP broadcasts.
// Lane 0's slot for channel 0 is kept at zero (its value is the separate
// `v`), so the dual rules need no per-lane branch.
//
// The step runs storage-ordered (deposit by global atomics) or tiled: a
// workgroup takes one chunk of particles sorted into one grid tile and
// accumulates the deposit in LDS over the tile's nodes plus a halo, flushing
// it once.
// On the step before a re-sort the tiled kernel can store every particle in
// its sorted slot of the second state buffer (k_particles_sorted), from tile
// keys written one launch earlier: the sort then needs no pass over the state.
#include "context.hpp"

namespace dpic {

// ---------------------------------------------------------------- lattice
struct ElemTable {
    int kind[DPIC_MAX_ELEMENTS];
    int nsteps[DPIC_MAX_ELEMENTS];
};

template <int NC>
__global__ void k_element_consts(ElemTable tab, int n_elem, const double* __restrict__ elem_in,
                                 double* __restrict__ ec, double inv_g2) {
    const int e = blockIdx.x;
    const int c = threadIdx.x;
    if (e >= n_elem || c >= NC) return;
    elem_in += (size_t)blockIdx.y * DPIC_MAX_ELEMENTS * 2 * NC;  // setting
    ec += (size_t)blockIdx.y * DPIC_MAX_ELEMENTS * EC_N * NC;
    LD L = ldload(elem_in + (e * 2 + 0) * NC, c);
    LD k = ldload(elem_in + (e * 2 + 1) * NC, c);
    const double ns = (double)tab.nsteps[e];
    LD tau = LD{L.v / ns, L.t / ns};  // tau = L / n_steps
    LD s = tau * 0.5;
    Map2 ax, ay;
    if (tab.kind[e] == 1) {
        ax = plane_map(k, s);
        ay = plane_map(-k, s);
    } else {
        ax = Map2{ldc(1.0), s, ldc(0.0), ldc(1.0)};
        ay = ax;
    }
    LD slip = s * inv_g2;
    double* o = ec + (size_t)e * EC_N * NC + c;
    o[EC_TAU * NC] = ldchan(tau, c);
    double* h = o + EC_HALF * NC;
    h[(MB_AX + 0) * NC] = ldchan(ax.a, c);
    h[(MB_AX + 1) * NC] = ldchan(ax.b, c);
    h[(MB_AX + 2) * NC] = ldchan(ax.c, c);
    h[(MB_AX + 3) * NC] = ldchan(ax.d, c);
    h[(MB_AY + 0) * NC] = ldchan(ay.a, c);
    h[(MB_AY + 1) * NC] = ldchan(ay.b, c);
    h[(MB_AY + 2) * NC] = ldchan(ay.c, c);
    h[(MB_AY + 3) * NC] = ldchan(ay.d, c);
    h[MB_SLIP * NC] = ldchan(slip, c);
}

// Fused map blocks: B A for the half-step maps A (this element) and B (this
// element again, or the next element of the period).
template <int NC>
__device__ void combine_block(const double* A, const double* B, double* out, int c) {
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
        const int o = pl * 4;
        const LD a00 = ldload(A + (o + 0) * NC, c), a01 = ldload(A + (o + 1) * NC, c);
        const LD a10 = ldload(A + (o + 2) * NC, c), a11 = ldload(A + (o + 3) * NC, c);
        const LD b00 = ldload(B + (o + 0) * NC, c), b01 = ldload(B + (o + 1) * NC, c);
        const LD b10 = ldload(B + (o + 2) * NC, c), b11 = ldload(B + (o + 3) * NC, c);
        out[(o + 0) * NC] = ldchan(b00 * a00 + b01 * a10, c);
        out[(o + 1) * NC] = ldchan(b00 * a01 + b01 * a11, c);
        out[(o + 2) * NC] = ldchan(b10 * a00 + b11 * a10, c);
        out[(o + 3) * NC] = ldchan(b10 * a01 + b11 * a11, c);
    }
    out[MB_SLIP * NC] = ldchan(ldload(A + MB_SLIP * NC, c) + ldload(B + MB_SLIP * NC, c), c);
}

template <int NC>
__global__ void k_element_combine(int n_elem, double* __restrict__ ec) {
    const int e = blockIdx.x;
    const int c = threadIdx.x;
    if (e >= n_elem || c >= NC) return;
    ec += (size_t)blockIdx.y * DPIC_MAX_ELEMENTS * EC_N * NC;  // setting
    const int en = (e + 1) % n_elem;
    const double* A = ec + (size_t)e * EC_N * NC + EC_HALF * NC;
    const double* Bn = ec + (size_t)en * EC_N * NC + EC_HALF * NC;
    combine_block<NC>(A, A, ec + (size_t)e * EC_N * NC + EC_SAME * NC + c, c);
    combine_block<NC>(A, Bn, ec + (size_t)e * EC_N * NC + EC_NEXT * NC + c, c);
}

hipError_t launch_element_consts_into(dpic_ctx* cx, int NC, int nb, const double* elem_in, double* ec) {
    ElemTable tab{};
    for (int e = 0; e < cx->n_elem; ++e) {
        tab.kind[e] = cx->kind[e];
        tab.nsteps[e] = cx->n_steps[e];
    }
    const double inv_g2 = 1.0 / (cx->gamma0 * cx->gamma0);
    dim3 grid(cx->n_elem, nb), block(64);
    switch (NC) {
        case 1:
            hipLaunchKernelGGL(k_element_consts<1>, grid, block, 0, cx->stream, tab, cx->n_elem, elem_in, ec, inv_g2);
            hipLaunchKernelGGL(k_element_combine<1>, grid, block, 0, cx->stream, cx->n_elem, ec);
            break;
        case 8:
            hipLaunchKernelGGL(k_element_consts<8>, grid, block, 0, cx->stream, tab, cx->n_elem, elem_in, ec, inv_g2);
            hipLaunchKernelGGL(k_element_combine<8>, grid, block, 0, cx->stream, cx->n_elem, ec);
            break;
        case 16:
            hipLaunchKernelGGL(k_element_consts<16>, grid, block, 0, cx->stream, tab, cx->n_elem, elem_in, ec, inv_g2);
            hipLaunchKernelGGL(k_element_combine<16>, grid, block, 0, cx->stream, cx->n_elem, ec);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_element_consts(dpic_ctx* cx) {
    return launch_element_consts_into(cx, cx->NC, cx->B, cx->ws.elem_in, cx->ws.ec);
}

// ---------------------------------------------------------------- beam init
// Storage slot p of setting b = owner[p / SEG] takes packed row p - delta_b of
// xi; slots past the setting's n (segment padding) are left alone.
template <int NC>
__global__ void k_init_beam(const double* __restrict__ xi, int64_t used, int64_t cap,
                            const SettingDev* __restrict__ set, const int32_t* __restrict__ owner,
                            const double* __restrict__ sig, double* __restrict__ st, int32_t* __restrict__ pid) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= used) return;
    const int b = owner[p / SEG];
    const SettingDev sd = set[b];
    if (p - sd.off >= sd.n) return;
    const int64_t row = p - sd.delta;
    const double* sg = sig + (size_t)b * 6 * NC;
#pragma unroll
    for (int j = 0; j < 6; ++j) st[((int64_t)j * cap + p) * NC + c] = sg[j * NC + c] * xi[row * 6 + j];
    if (c == 0) pid[p] = (int32_t)row;
}

hipError_t launch_init_beam(dpic_ctx* cx, const double* xi) {
    const int64_t threads = cx->used * cx->NC;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    if (threads == 0) return hipSuccess;
    const Workspace& w = cx->ws;
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_init_beam<1>, grid, block, 0, cx->stream, xi, cx->used, cx->dims.n_particles, w.set, w.owner, w.sig, w.st, w.pid); break;
        case 8: hipLaunchKernelGGL(k_init_beam<8>, grid, block, 0, cx->stream, xi, cx->used, cx->dims.n_particles, w.set, w.owner, w.sig, w.st, w.pid); break;
        default: hipLaunchKernelGGL(k_init_beam<16>, grid, block, 0, cx->stream, xi, cx->used, cx->dims.n_particles, w.set, w.owner, w.sig, w.st, w.pid); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- group duals
// A particle owns a group of G consecutive lanes; lane q holds channels
// [q K, q K + K). Two channels per lane (one 16-byte load per coordinate)
// measured fastest at both 8 and 16 channels: one channel per lane frees
// registers for a third wave per SIMD but doubles the memory and LDS
// instructions per byte, four per lane cost the second wave.
template <int NC>
struct LaneGroup {
    static constexpr int G = NC == 1 ? 1 : NC / 2;
    static constexpr int K = NC / G;
};

// The particle state streams through once per step (768 bytes per particle
// at 8 channels), so its loads and stores carry the nontemporal hint: they
// then do not push the grids that the solve, the field and the next deposit
// reuse out of the caches. With 1e6 particles on 64^3 nodes the solve fell
// from 101 to 91 us per step; the particle kernel itself is unchanged.
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int K>
struct QD {
    double v;     // value, equal in every lane of the group
    double t[K];  // this lane's channels (slot 0 of lane 0 stays 0)
};

// 32-bit broadcast of the first lane of each group of G lanes by DPP: the
// quad_perm [0,0,0,0] copy, then row_shr:4 into the odd banks (lanes 4-7 and
// 12-15 of a row) for G >= 8, then row_shr:8 into banks 2 and 3 for G = 16.
template <int G>
__device__ __forceinline__ int group_bcast_u32(int x) {
    int b = __builtin_amdgcn_mov_dpp(x, 0x00, 0xf, 0xf, false);
    if constexpr (G >= 8) b = __builtin_amdgcn_update_dpp(b, b, 0x114, 0xf, 0xa, false);
    if constexpr (G >= 16) b = __builtin_amdgcn_update_dpp(b, b, 0x118, 0xf, 0xc, false);
    return b;
}

template <int G>
__device__ __forceinline__ double group_bcast(double x) {
    static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
    const long long b = __double_as_longlong(x);
    const int lo = group_bcast_u32<G>((int)(b & 0xffffffffll));
    const int hi = group_bcast_u32<G>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int K, int G>
__device__ __forceinline__ QD<K> qd_load(const double* __restrict__ p, int q) {
    QD<K> r;
    const double* s = p + q * K;
    if constexpr (K == 1) {
        r.t[0] = s[0];
    } else {
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const double2 w = reinterpret_cast<const double2*>(s)[i];
            r.t[2 * i] = w.x;
            r.t[2 * i + 1] = w.y;
        }
    }
    if constexpr (G == 1)
        r.v = r.t[0];
    else
        r.v = group_bcast<G>(r.t[0]);
    if (q == 0) r.t[0] = 0.0;
    return r;
}

template <int K>
__device__ __forceinline__ double qd_chan(const QD<K>& x, int q, int k) {
    return (q == 0 && k == 0) ? x.v : x.t[k];
}

// a state coordinate to global memory, nontemporal (the state streams)
template <int K>
__device__ __forceinline__ void qd_store(double* __restrict__ p, const QD<K>& x, int q) {
    double* s = p + q * K;
    if constexpr (K == 1) {
        __builtin_nontemporal_store(qd_chan(x, q, 0), s);
    } else {
#pragma unroll
        for (int i = 0; i < K / 2; ++i)
            __builtin_nontemporal_store(dvec2{qd_chan(x, q, 2 * i), x.t[2 * i + 1]}, reinterpret_cast<dvec2*>(s) + i);
    }
}

// LDS duals in split layout: lds_dual<NC>() doubles per dual. Slots
// [0, NC) hold the channels with channel 0 (the value) replaced by 0, slot NC
// the value, slot NC + 1 pads to 16 bytes. Lane q of a group reads its K
// slots with aligned 16-byte loads (lane 0's slot 0 is already the zero the
// dual rules need) and the value with a group-uniform read that the LDS
// serves as a broadcast: no DPP move and no select on the read path.
template <int NC>
constexpr int lds_dual() {
    return NC == 1 ? 1 : NC + 2;
}

template <int NC>
__device__ __forceinline__ void put_split(double* d, int ch, double val) {
    if constexpr (NC == 1) {
        d[0] = val;
    } else if (ch == 0) {
        d[0] = 0.0;
        d[NC] = val;
    } else {
        d[ch] = val;
    }
}

template <int NC>
__device__ __forceinline__ QD<LaneGroup<NC>::K> qd_load_split(const double* p, int q) {
    constexpr int K = LaneGroup<NC>::K;
    QD<K> r;
    if constexpr (NC == 1) {
        r.v = p[0];
        r.t[0] = 0.0;
    } else {
        const double* s = p + q * K;
        if constexpr (K == 1) {
            r.t[0] = s[0];
        } else {
#pragma unroll
            for (int i = 0; i < K / 2; ++i) {
                const double2 w = reinterpret_cast<const double2*>(s)[i];
                r.t[2 * i] = w.x;
                r.t[2 * i + 1] = w.y;
            }
        }
        r.v = p[NC];
    }
    return r;
}

// product rule
template <int K>
__device__ __forceinline__ QD<K> qd_mul(const QD<K>& x, const QD<K>& y) {
    QD<K> r;
    r.v = x.v * y.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = fma(x.v, y.t[k], x.t[k] * y.v);
    return r;
}

// acc + x y
template <int K>
__device__ __forceinline__ void qd_fmad(const QD<K>& x, const QD<K>& y, QD<K>& acc) {
    acc.v = fma(x.v, y.v, acc.v);
#pragma unroll
    for (int k = 0; k < K; ++k) acc.t[k] = fma(x.v, y.t[k], fma(x.t[k], y.v, acc.t[k]));
}

template <int K>
__device__ __forceinline__ QD<K> qd_scale(const QD<K>& x, double s) {
    QD<K> r;
    r.v = x.v * s;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = x.t[k] * s;
    return r;
}

template <int K>
__device__ __forceinline__ QD<K> qd_zero() {
    QD<K> r;
    r.v = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) r.t[k] = 0.0;
    return r;
}

// CIC weight pair of one dimension: f = s - floor(s) with df = du / h, g = 1 - f.
template <int K>
__device__ __forceinline__ QD<K> qd_frac(const QD<K>& u, double s, int i, double ih) {
    QD<K> f;
    f.v = s - (double)i;
#pragma unroll
    for (int k = 0; k < K; ++k) f.t[k] = u.t[k] * ih;
    return f;
}

template <int K>
__device__ __forceinline__ QD<K> qd_one_minus(const QD<K>& f) {
    QD<K> g;
    g.v = 1.0 - f.v;
#pragma unroll
    for (int k = 0; k < K; ++k) g.t[k] = -f.t[k];
    return g;
}

// ---------------------------------------------------------------- fused step
struct PartArgs {
    double* st;
    int64_t cap, used;
    const SettingDev* set;  // per-setting arrays and charge
    const int32_t* owner;
    int tau_off;            // dual step of the current element in a setting's element table
    int map_off;            // map block (MB_N duals) in it
    int nx, ny, nz;
    double lo0, lo1, lo2, ih0, ih1, ih2;
    double kperp, kpar;
    uint32_t* key_out;      // PF_KEYS: each particle's tile key for the next sort
    int ktx, kty, knbins;   // tiles in x and y, sort bins (the last one: outside the box)
    double* st_out;         // PF_SCATTER: second state buffer, sorted order
    const int32_t* pid_in;  // PF_SCATTER: original rows, stored order
    int32_t* pid_out;       //             and sorted order
    int64_t step;           // schedule step of this launch (for the non-finite record)
};

// the arrays and charge of one setting
struct SetView {
    const double* E;
    double* rho;
    unsigned long long* cnt;
    double q;
};

__device__ __forceinline__ SetView set_view(const SettingDev& sd) { return SetView{sd.E, sd.rho, sd.cnt, sd.q}; }

struct TiledArgs {
    const int4* chunks;
    const uint32_t* nchunks;
    const double* E0;  // field of setting b at E0 + b * estride
    int64_t estride;
    int tx, ty, nbins;
    const uint32_t* key_in;  // PF_SCATTER: tile keys, stored order (counted into the bin starts)
    uint32_t* cur;           // PF_SCATTER: [setting][bin] next free sorted slot
};

// PF_SCATTER: position of tile key k among the 27 tiles around (tx, ty, tz),
// or -1 (farther, or outside the box)
__device__ __forceinline__ int near_tile(uint32_t k, int tx, int ty, int tz, const TiledArgs& t) {
    if ((int)k >= t.nbins - 1) return -1;
    const int kx = (int)k % t.tx, ky = ((int)k / t.tx) % t.ty, kz = (int)k / (t.tx * t.ty);
    const int dx = kx - tx + 1, dy = ky - ty + 1, dz = kz - tz + 1;
    if ((unsigned)dx > 2u || (unsigned)dy > 2u || (unsigned)dz > 2u) return -1;
    return (dz * 3 + dy) * 3 + dx;
}

// LDS copy of the deposit tile: the nodes [o, o + TILE_R)^2 x [oz, oz +
// dep_rz) around the grid tile, channel-major with a channel stride of 1 mod
// 16 doubles, so channel c of node n sits in bank pair (c + n) mod 16: the
// lanes of a group (channels k, k+K, ..) and particles at different nodes
// spread over the banks. It has the drift allowance in z only without
// PF_EHALO: with the fields in the caches, the few particles that cross a z
// face deposit by global atomics at no measurable cost, and the smaller tile
// is cheaper to clear and flush; with the fields (and charges) streaming from
// HBM those atomics cost more than the larger tile.
template <int F>
constexpr int dep_rz() {
    return (F & PF_EHALO) ? TILE_EDGE + 1 : TILE_R;
}
template <int F>
constexpr int dep_offz() {
    return (F & PF_EHALO) ? 0 : TILE_HALO;
}
template <int F>
constexpr int dep_nodes() {
    return TILE_R * TILE_R * dep_rz<F>();
}
template <int F>
constexpr int dep_cstride() {
    return ((dep_nodes<F>() + 15) / 16) * 16 + 1;
}
// LDS copy of E: the nodes [o + EO, o + EO + ER)^2 x [tile z, + TILE_RZ_E),
// [node][component] duals in the split layout. With PF_EHALO it has
// the transverse drift allowance (ER = TILE_R nodes, EO = 0), else it covers
// the tile's own nodes (ER = TILE_EDGE + 1, EO = TILE_HALO). The allowance
// keeps drifted particles on the LDS path, but each item stages twice the
// nodes: it pays while the fields of all settings stay in the caches (one
// beam of 1e6 particles on 64^3 nodes: 2% faster) and not once they stream
// from HBM (64 beams of 1e5-1e6 particles: 7% slower).
// The E tile is staged only where it leaves room for two workgroups per CU:
// at 16 channels it and the deposit tile would take 122 KB.
template <int F>
constexpr int etile_r() {
    return (F & PF_EHALO) ? TILE_R : TILE_EDGE + 1;
}
template <int F>
constexpr int etile_off() {
    return (F & PF_EHALO) ? 0 : TILE_HALO;
}
template <int F>
constexpr int etile_nodes() {
    return etile_r<F>() * etile_r<F>() * TILE_RZ_E;
}
template <int NC, int F>
constexpr bool use_etile() {
    return (F & PF_KICK) && NC <= 8;
}
constexpr int PART_THREADS = 256;
constexpr int STAGE_BATCH = 8;  // E-tile staging loads in flight per thread
#ifndef DPIC_FB_CORNERS
#define DPIC_FB_CORNERS 4
#endif
constexpr int FB_CORNERS = DPIC_FB_CORNERS;  // corners per round trip of the global-memory gather
constexpr double EHALO_MAX_BYTES = 128.0 * (1 << 20);  // fields of all settings, for PF_EHALO

// Wavefront max of the extents (all 64 lanes take part), one atomic per
// wave and dimension, nothing waited for: for a workgroup that moves on to
// another setting's items (each setting has its own counters).
__device__ __forceinline__ void extent_flush_wave(unsigned long long* cnt, double e0, double e1, double e2) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        e0 = fmax(e0, __shfl_xor(e0, off, 64));
        e1 = fmax(e1, __shfl_xor(e1, off, 64));
        e2 = fmax(e2, __shfl_xor(e2, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(cnt + CNT_EXT_X, (unsigned long long)__double_as_longlong(e0));
        atomicMax(cnt + CNT_EXT_Y, (unsigned long long)__double_as_longlong(e1));
        atomicMax(cnt + CNT_EXT_Z, (unsigned long long)__double_as_longlong(e2));
    }
}

// Workgroup max of the extents (every thread of the workgroup calls it),
// merged into the setting's counters by one thread, with an atomic only
// where it raises the stored value. All workgroups update the same three
// words: atomics there queue behind each other, and a wave's later loads
// wait for its earlier atomics, so they are kept rare (once per workgroup
// and setting; the extents stop growing after the first steps).
__device__ __forceinline__ void extent_flush(unsigned long long* cnt, double e0, double e1, double e2,
                                             double (*sext)[3]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        e0 = fmax(e0, __shfl_xor(e0, off, 64));
        e1 = fmax(e1, __shfl_xor(e1, off, 64));
        e2 = fmax(e2, __shfl_xor(e2, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sext[threadIdx.x / 64][0] = e0;
        sext[threadIdx.x / 64][1] = e1;
        sext[threadIdx.x / 64][2] = e2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double m = sext[0][d];
            for (int w = 1; w < (int)(blockDim.x / 64); ++w) m = fmax(m, sext[w][d]);
            // non-negative doubles order like their bit patterns
            const unsigned long long v = (unsigned long long)__double_as_longlong(m);
            if (v > __hip_atomic_load(cnt + CNT_EXT_X + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(cnt + CNT_EXT_X + d, v);
        }
    }
    __syncthreads();  // sext is reused
}

// Record the launch's step in the setting's non-finite counter when any lane
// of the wave stored a NaN or Inf (all 64 lanes take part).
__device__ __forceinline__ void nonfinite_flush_wave(unsigned long long* cnt, bool nf, int64_t step) {
    const unsigned long long m = __ballot(nf);
    if (m != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1))
        atomicMax(cnt + CNT_NONFINITE, NONFINITE_BASE - (unsigned long long)step);
}

template <int K>
__device__ __forceinline__ int qd_nonfinite(const QD<K>& x) {  // 0 or 1, so that checks combine without branches
    bool bad = !__builtin_isfinite(x.v);
#pragma unroll
    for (int k = 0; k < K; ++k) bad |= !__builtin_isfinite(x.t[k]);
    return bad;
}

__device__ __forceinline__ CellPos cell_of(double x, double y, double z, const PartArgs& a) {
    return grid_cell(x, y, z, a.lo0, a.lo1, a.lo2, a.ih0, a.ih1, a.ih2, a.nx, a.ny, a.nz);
}

// One particle's share of a fused step, lane q of its group: gather and kick
// (PF_KICK), one map block (PF_MAP), then deposit (PF_DEPOSIT) or count
// (PF_COUNT). With TILED the deposit goes to the workgroup's LDS copy `lr` of
// the nodes [o, o + TILE_R) when all 8 corners fall inside it, else to global
// memory.
// A particle's six coordinates as this lane's raw channels (no broadcast
// yet), so that the loads of the next particle can be issued before the
// current one is processed.
template <int K>
struct RawState {
    double r[6][K];
};

template <int NC>
__device__ __forceinline__ RawState<LaneGroup<NC>::K> load_raw(const PartArgs& a, int64_t p, int q) {
    constexpr int K = LaneGroup<NC>::K;
    RawState<K> s;
    const int64_t cs = a.cap * NC;
    const double* sp = a.st + p * NC + q * K;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        if constexpr (K == 1) {
            s.r[j][0] = __builtin_nontemporal_load(sp + j * cs);
        } else {
#pragma unroll
            for (int i = 0; i < K / 2; ++i) {
                const dvec2 w = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(sp + j * cs) + i);
                s.r[j][2 * i] = w.x;
                s.r[j][2 * i + 1] = w.y;
            }
        }
    }
    return s;
}

// An empty use of prefetched registers. The compiler's wait for a load
// covers every store issued before it too (loads and stores share one
// counter), so a prefetch first used after the current particle's stores
// waits for those stores; used here, just before them, it waits only for
// loads issued a whole particle earlier and for the previous particle's
// stores, long done by then.
template <int K>
__device__ __forceinline__ void pin_raw(const RawState<K>& s) {
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) asm volatile("" ::"v"(s.r[j][k]));
}

template <int K, int G>
__device__ __forceinline__ QD<K> raw_to_qd(const double* r, int q) {
    QD<K> x;
#pragma unroll
    for (int k = 0; k < K; ++k) x.t[k] = r[k];
    if constexpr (G == 1)
        x.v = x.t[0];
    else
        x.v = group_bcast<G>(x.t[0]);
    if (q == 0) x.t[0] = 0.0;
    return x;
}

template <int NC, int F, bool TILED, class Dest>
__device__ __forceinline__ void particle_body(const PartArgs& a, const SetView& sv, const double* __restrict__ smap,
                                              const double* __restrict__ stau, int64_t p, Dest dest, int q,
                                              const RawState<LaneGroup<NC>::K>& raw, double* lr, const double* le, int ox,
                                              int oy, int oz, int oze, bool use_tile, double& e0, double& e1, double& e2,
                                              bool& nf) {
    constexpr int G = LaneGroup<NC>::G, K = LaneGroup<NC>::K;
    const int64_t cs = a.cap * NC;
    QD<K> x = raw_to_qd<K, G>(raw.r[0], q), px = raw_to_qd<K, G>(raw.r[1], q), y = raw_to_qd<K, G>(raw.r[2], q);
    QD<K> py = raw_to_qd<K, G>(raw.r[3], q), z = raw_to_qd<K, G>(raw.r[4], q), d = raw_to_qd<K, G>(raw.r[5], q);
    const int64_t sxy = (int64_t)a.nx * a.ny;
    if (F & PF_KICK) {
        const CellPos g = cell_of(x.v, y.v, z.v, a);
        if (g.inside) {
            const QD<K> fx = qd_frac(x, g.sx, g.ix, a.ih0), fy = qd_frac(y, g.sy, g.iy, a.ih1),
                        fz = qd_frac(z, g.sz, g.iz, a.ih2);
            QD<K> ex = qd_zero<K>(), ey = qd_zero<K>(), ez = qd_zero<K>();
            constexpr int ER = etile_r<F>();
            const int tlx = g.ix - ox - etile_off<F>(), tly = g.iy - oy - etile_off<F>(), tlz = g.iz - oze;
            const bool in_etile = TILED && use_etile<NC, F>() && use_tile && tlx >= 0 && tlx <= ER - 2 &&
                                  tly >= 0 && tly <= ER - 2 && tlz >= 0 && tlz <= TILE_RZ_E - 2;
            if (in_etile) {
                const int l0 = (tlz * ER + tly) * ER + tlx;
#pragma unroll
                for (int kz = 0; kz < 2; ++kz) {
#pragma unroll
                    for (int ky = 0; ky < 2; ++ky) {
                        const QD<K> wyz = qd_mul(ky ? fy : qd_one_minus(fy), kz ? fz : qd_one_minus(fz));
#pragma unroll
                        for (int kx = 0; kx < 2; ++kx) {
                            const QD<K> w = qd_mul(kx ? fx : qd_one_minus(fx), wyz);
                            constexpr int D = lds_dual<NC>();
                            const double* ep = le + (l0 + kx + ky * ER + kz * ER * ER) * 3 * D;
                            qd_fmad(w, qd_load_split<NC>(ep, q), ex);
                            qd_fmad(w, qd_load_split<NC>(ep + D, q), ey);
                            qd_fmad(w, qd_load_split<NC>(ep + 2 * D, q), ez);
                        }
                    }
                }
            } else if constexpr ((F & PF_EHALO) != 0) {
                // E from global memory (a wavefront with one particle outside
                // the E tile takes this path). The 8 corners' values of one
                // component are loaded together before any is used: one round
                // trip per component, where loads consumed one by one waited
                // for each other. Same corner order and weights as above.
                const int64_t n0 = ((int64_t)g.iz * a.ny + g.iy) * a.nx + g.ix;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
#pragma unroll
                  for (int h = 0; h < 8; h += FB_CORNERS) {
                    double raw[8][K];
#pragma unroll
                    for (int k = h; k < h + FB_CORNERS; ++k) {
                        const double* ep =
                            sv.E + (n0 + (k & 1) + ((k >> 1) & 1) * a.nx + (k >> 2) * sxy) * 3 * NC + c * NC + q * K;
                        if constexpr (K == 1) {
                            raw[k][0] = ep[0];
                        } else {
#pragma unroll
                            for (int i = 0; i < K / 2; ++i) {
                                const double2 v = reinterpret_cast<const double2*>(ep)[i];
                                raw[k][2 * i] = v.x;
                                raw[k][2 * i + 1] = v.y;
                            }
                        }
                    }
                    QD<K>& acc = c == 0 ? ex : (c == 1 ? ey : ez);
#pragma unroll
                    for (int k = h; k < h + FB_CORNERS; ++k) {
                        QD<K> e;
#pragma unroll
                        for (int i = 0; i < K; ++i) e.t[i] = raw[k][i];
                        if constexpr (G == 1)
                            e.v = e.t[0];
                        else
                            e.v = group_bcast<G>(e.t[0]);
                        if (q == 0) e.t[0] = 0.0;
                        const QD<K> wyz = qd_mul(((k >> 1) & 1) ? fy : qd_one_minus(fy), (k >> 2) ? fz : qd_one_minus(fz));
                        const QD<K> w = qd_mul((k & 1) ? fx : qd_one_minus(fx), wyz);
                        qd_fmad(w, e, acc);
                    }
                  }
                }
            } else {
                // the same sum with each load consumed as it arrives: the
                // variants without the drift allowance keep this form, since
                // the batched loads above raise their register allocation and
                // slow their particle loop
                const int64_t n0 = ((int64_t)g.iz * a.ny + g.iy) * a.nx + g.ix;
#pragma unroll
                for (int kz = 0; kz < 2; ++kz) {
#pragma unroll
                    for (int ky = 0; ky < 2; ++ky) {
                        const QD<K> wyz = qd_mul(ky ? fy : qd_one_minus(fy), kz ? fz : qd_one_minus(fz));
#pragma unroll
                        for (int kx = 0; kx < 2; ++kx) {
                            const QD<K> w = qd_mul(kx ? fx : qd_one_minus(fx), wyz);
                            const double* ep = sv.E + (n0 + kx + ky * a.nx + kz * sxy) * 3 * NC;
                            qd_fmad(w, qd_load<K, G>(ep, q), ex);
                            qd_fmad(w, qd_load<K, G>(ep + NC, q), ey);
                            qd_fmad(w, qd_load<K, G>(ep + 2 * NC, q), ez);
                        }
                    }
                }
            }
            const QD<K> tau = qd_load_split<NC>(stau, q);
            qd_fmad(tau, qd_scale(ex, a.kperp), px);
            qd_fmad(tau, qd_scale(ey, a.kperp), py);
            qd_fmad(tau, qd_scale(ez, a.kpar), d);
        }
    }
    if (F & PF_MAP) {
        constexpr int D = lds_dual<NC>();
        {
            const double* m = smap + MB_AX * D;
            QD<K> nu = qd_mul(qd_load_split<NC>(m, q), x), np = qd_mul(qd_load_split<NC>(m + 2 * D, q), x);
            qd_fmad(qd_load_split<NC>(m + D, q), px, nu);
            qd_fmad(qd_load_split<NC>(m + 3 * D, q), px, np);
            x = nu;
            px = np;
        }
        {
            const double* m = smap + MB_AY * D;
            QD<K> nu = qd_mul(qd_load_split<NC>(m, q), y), np = qd_mul(qd_load_split<NC>(m + 2 * D, q), y);
            qd_fmad(qd_load_split<NC>(m + D, q), py, nu);
            qd_fmad(qd_load_split<NC>(m + 3 * D, q), py, np);
            y = nu;
            py = np;
        }
        qd_fmad(qd_load_split<NC>(smap + MB_SLIP * D, q), d, z);
    }
    if (F & (PF_DEPOSIT | PF_COUNT)) {
        const CellPos g = cell_of(x.v, y.v, z.v, a);
        // the sort's key of this position (the sort that follows reads it
        // instead of the positions)
        if ((F & PF_KEYS) && q == 0)
            a.key_out[p] = g.inside ? (uint32_t)(((g.iz / TILE_EDGE) * a.kty + g.iy / TILE_EDGE) * a.ktx + g.ix / TILE_EDGE)
                                    : (uint32_t)(a.knbins - 1);
        if (g.inside) {
            if (F & PF_DEPOSIT) {
                const QD<K> fx = qd_frac(x, g.sx, g.ix, a.ih0), fy = qd_frac(y, g.sy, g.iy, a.ih1),
                            fz = qd_frac(z, g.sz, g.iz, a.ih2);
                const int lx = g.ix - ox, ly = g.iy - oy, lz = g.iz - oz;
                const bool local = TILED && use_tile && lx >= 0 && lx <= TILE_R - 2 && ly >= 0 &&
                                   ly <= TILE_R - 2 && lz >= 0 && lz <= dep_rz<F>() - 2;
                if (TILED && local) {
                    const int l0 = (lz * TILE_R + ly) * TILE_R + lx;
#pragma unroll
                    for (int kz = 0; kz < 2; ++kz) {
#pragma unroll
                        for (int ky = 0; ky < 2; ++ky) {
                            const QD<K> wyz = qd_mul(ky ? fy : qd_one_minus(fy), kz ? fz : qd_one_minus(fz));
#pragma unroll
                            for (int kx = 0; kx < 2; ++kx) {
                                const QD<K> w = qd_mul(kx ? fx : qd_one_minus(fx), wyz);
                                constexpr int CS = dep_cstride<F>();
                                double* l = lr + (q * K) * CS + l0 + kx + ky * TILE_R + kz * TILE_R * TILE_R;
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    unsafeAtomicAdd(l + k * CS, qd_chan(w, q, k) * sv.q);
                            }
                        }
                    }
                } else {
                    const int64_t n0 = ((int64_t)g.iz * a.ny + g.iy) * a.nx + g.ix;
#pragma unroll
                    for (int kz = 0; kz < 2; ++kz) {
#pragma unroll
                        for (int ky = 0; ky < 2; ++ky) {
                            const QD<K> wyz = qd_mul(ky ? fy : qd_one_minus(fy), kz ? fz : qd_one_minus(fz));
#pragma unroll
                            for (int kx = 0; kx < 2; ++kx) {
                                const QD<K> w = qd_mul(kx ? fx : qd_one_minus(fx), wyz);
                                double* r = sv.rho + (n0 + kx + ky * a.nx + kz * sxy) * NC + q * K;
#pragma unroll
                                for (int k = 0; k < K; ++k) unsafeAtomicAdd(r + k, qd_chan(w, q, k) * sv.q);
                            }
                        }
                    }
                }
            }
        } else if (q == 0) {
            atomicAdd(sv.cnt + CNT_OUTSIDE, 1ull);
        }
        e0 = fmax(e0, fabs(x.v));
        e1 = fmax(e1, fabs(y.v));
        e2 = fmax(e2, fabs(z.v));
    }
    nf |= qd_nonfinite(x) | qd_nonfinite(px) | qd_nonfinite(y) | qd_nonfinite(py) | qd_nonfinite(z) | qd_nonfinite(d);
    // the slot the state goes to: p, or with PF_SCATTER its sorted slot
    double* sp = ((F & PF_SCATTER) ? a.st_out : a.st) + dest() * NC;
    qd_store(sp, x, q);
    qd_store(sp + cs, px, q);
    qd_store(sp + 2 * cs, y, q);
    qd_store(sp + 3 * cs, py, q);
    qd_store(sp + 4 * cs, z, q);
    qd_store(sp + 5 * cs, d, q);
}

// Copy a setting's step constants (tau and one map block) into LDS, split layout.
template <int NC>
__device__ __forceinline__ void stage_consts(const PartArgs& a, const double* __restrict__ ec, double* smap,
                                             double* stau) {
    constexpr int D = lds_dual<NC>();
    for (int j = threadIdx.x; j < MB_N * NC; j += PART_THREADS)
        put_split<NC>(smap + (j / NC) * D, j % NC, ec[a.map_off + j]);
    for (int j = threadIdx.x; j < NC; j += PART_THREADS) put_split<NC>(stau, j, ec[a.tau_off + j]);
}

// Storage-order kernel: deposit by global atomics. A workgroup covers
// PART_THREADS / G consecutive slots, which never straddle a storage segment,
// so its setting is that of its first slot.
template <int NC, int F>
__global__ __launch_bounds__(PART_THREADS) void k_particles(PartArgs a) {
    constexpr int G = LaneGroup<NC>::G;
    __shared__ __align__(16) double smap[MB_N * lds_dual<NC>()];
    __shared__ __align__(16) double stau[lds_dual<NC>()];
    __shared__ double sext[PART_THREADS / 64][3];
    const int64_t p0 = (int64_t)blockIdx.x * (PART_THREADS / G);
    const SettingDev sd = a.set[a.owner[p0 / SEG]];
    stage_consts<NC>(a, sd.ec, smap, stau);
    __syncthreads();
    const SetView sv = set_view(sd);
    const int64_t p = p0 + threadIdx.x / G;
    const int q = (int)(threadIdx.x % G);
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    bool nf = false;
    if (p - sd.off < sd.n) {
        const RawState<LaneGroup<NC>::K> raw = load_raw<NC>(a, p, q);
        particle_body<NC, F, false>(a, sv, smap, stau, p, [p]() { return p; }, q, raw, nullptr, nullptr, 0, 0, 0, 0, false, e0, e1, e2,
                                    nf);
    }
    nonfinite_flush_wave(sv.cnt, nf, a.step);
    if (F & (PF_DEPOSIT | PF_COUNT)) extent_flush(sv.cnt, e0, e1, e2, sext);
}

// PF_SCATTER: the sorted slot of a particle with tile key k and original row
// `row` (both loaded by the group's first lane with its state), claimed by
// that lane from its tile's run (sclaim) or singly from the bin's cursor; the
// lane also moves the original row.
template <int G>
__device__ __forceinline__ int64_t scatter_slot(const PartArgs& a, const TiledArgs& t, int q, uint32_t k, int32_t row,
                                                uint32_t* sclaim, int setting, int tx, int ty, int tz, bool use_tile) {
    uint32_t slot = 0u;
    if (q == 0) {
        const int l = use_tile ? near_tile(k, tx, ty, tz, t) : -1;
        slot = l >= 0 ? atomicAdd(&sclaim[l], 1u) : atomicAdd(t.cur + (int64_t)setting * t.nbins + k, 1u);
        a.pid_out[slot] = row;
    }
    if constexpr (G > 1) slot = (uint32_t)group_bcast_u32<G>((int)slot);
    return (int64_t)slot;
}

// Tiled kernel, persistent: each workgroup walks the work list with a grid
// stride. A work item is one chunk of particles of one setting sorted into
// one grid tile; the deposit accumulates in LDS over the tile's nodes plus a
// TILE_HALO-cell halo (particles drift between re-sorts) and is flushed once:
// only nodes that received charge issue global atomics.
template <int NC, int F>
__device__ __forceinline__ void tiled_body(const PartArgs& a, const TiledArgs& t) {
    constexpr int G = LaneGroup<NC>::G;
    constexpr int LDSN = (F & PF_DEPOSIT) ? dep_cstride<F>() * NC : 1;
    constexpr int LDSE = use_etile<NC, F>() ? etile_nodes<F>() * 3 * lds_dual<NC>() : 1;
    __shared__ __align__(16) double lr[LDSN];
    __shared__ __align__(16) double le[LDSE];
    __shared__ __align__(16) double smap[MB_N * lds_dual<NC>()];
    __shared__ __align__(16) double stau[lds_dual<NC>()];
    __shared__ double sext[PART_THREADS / 64][3];
    __shared__ uint32_t sclaim[(F & PF_SCATTER) ? 27 : 1];  // PF_SCATTER: per nearby tile, next sorted slot
    const uint32_t nck = *t.nchunks;
    const int q = threadIdx.x % G;
    constexpr int STRIDE = PART_THREADS / G;
    int cur = -1;
    SetView sv{nullptr, nullptr, nullptr, 0.0};
    const int i0 = threadIdx.x / G;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;  // this thread's extents in the current setting
    bool nf = false;                      // and whether it stored a non-finite value there
#pragma unroll 1
    for (uint32_t ci = blockIdx.x; ci < nck; ci += gridDim.x) {
        const int4 ck = t.chunks[ci];
        if (ci != blockIdx.x) __syncthreads();  // the previous item's flush is done with lr and smap
        if (ck.w != cur) {
            if (cur >= 0) {
                nonfinite_flush_wave(sv.cnt, nf, a.step);
                nf = false;
            }
            if ((F & (PF_DEPOSIT | PF_COUNT)) && cur >= 0) {
                extent_flush_wave(sv.cnt, e0, e1, e2);
                e0 = e1 = e2 = 0.0;
            }
            cur = ck.w;
            const SettingDev sd = a.set[cur];
            sv = set_view(sd);
            stage_consts<NC>(a, sd.ec, smap, stau);
        }
        if (F & PF_DEPOSIT)
            for (int j = threadIdx.x; j < LDSN; j += PART_THREADS) lr[j] = 0.0;
        const bool use_tile = ck.x < t.nbins - 1;
        const int tx = ck.x % t.tx, ty = (ck.x / t.tx) % t.ty, tz = ck.x / (t.tx * t.ty);
        const int ox = tx * TILE_EDGE - TILE_HALO, oy = ty * TILE_EDGE - TILE_HALO, oz = tz * TILE_EDGE - dep_offz<F>();
        const int oze = tz * TILE_EDGE;  // E tile: no allowance in z
        if (F & PF_SCATTER) {
            // the item's particles by destination bin: one run of sorted
            // slots claimed per tile around the item's own, single slots for
            // particles farther away (LDS cleared after the previous item's
            // last use at the barrier that opened this one)
            if (threadIdx.x < 27) sclaim[threadIdx.x] = 0u;
            __syncthreads();
            if (use_tile)
                for (int j = threadIdx.x; j < ck.z; j += PART_THREADS) {
                    const int l = near_tile(t.key_in[(int64_t)ck.y + j], tx, ty, tz, t);
                    if (l >= 0) atomicAdd(&sclaim[l], 1u);
                }
            __syncthreads();
            if (threadIdx.x < 27 && sclaim[threadIdx.x] != 0u) {
                const int l = threadIdx.x;
                const int key = ((tz + l / 9 - 1) * t.ty + (ty + (l / 3) % 3 - 1)) * t.tx + (tx + l % 3 - 1);
                sclaim[l] = atomicAdd(t.cur + (int64_t)ck.w * t.nbins + key, sclaim[l]);
            }
            // ordered before the particle loop by the barrier after the E staging
        }
        // first particle's loads, in flight during the staging below
        RawState<LaneGroup<NC>::K> next;
        uint32_t knext = 0u;  // PF_SCATTER: the next particle's tile key and original row (first lane),
        int32_t rnext = 0;    // loaded with its state
        if (i0 < ck.z) {
            next = load_raw<NC>(a, (int64_t)ck.y + i0, q);
            if ((F & PF_SCATTER) && q == 0) {
                knext = t.key_in[(int64_t)ck.y + i0];
                rnext = a.pid_in[(int64_t)ck.y + i0];
            }
        }
        if (use_etile<NC, F>() && use_tile) {
            // the setting's field from its index: the staging need not wait
            // for the setting record
            const double* __restrict__ Eb = t.E0 + (int64_t)ck.w * t.estride;
            // E of the tile's nodes (runs of TILE_R nodes x 3 x NC doubles
            // along x in global memory) into the split layout
            constexpr int ER = etile_r<F>(), EN = etile_nodes<F>();
            if constexpr (NC >= 2 && NC % 2 == 0 && (F & PF_EHALO) != 0) {
                // In the variants with the drift allowance (which every kick
                // at up to 8 channels takes): straight from global memory into
                // LDS, 16 bytes per lane, every load of the tile in flight at
                // once and none through registers. A wavefront's load fills 64 consecutive 16-byte
                // chunks of the tile; a dual's chunks are its channel pairs
                // (0, 1), (2, 3), .. and (value, pad), each one aligned chunk
                // of the node's E, so the first holds the value where the
                // split layout wants a zero, written after the loads land
                // (by every thread over the duals after a barrier: measured
                // faster than each lane zeroing the chunks it loaded). Nodes
                // outside the grid get zeros by plain LDS stores.
                constexpr int CD = lds_dual<NC>() / 2, CN = 3 * CD, SC = EN * CN;
                const int c0w = (int)(threadIdx.x & ~63u), lane = (int)(threadIdx.x & 63u);
#pragma unroll 1
                for (int c0 = c0w; c0 < SC; c0 += PART_THREADS) {
                    const int c = c0 + lane;
                    const int node = c / CN, rc = c - node * CN, comp = rc / CD, k = rc - comp * CD;
                    const int lx = node % ER, ly = (node / ER) % ER, lz = node / (ER * ER);
                    const int gx = ox + etile_off<F>() + lx, gy = oy + etile_off<F>() + ly, gz = oze + lz;
                    if (c < SC) {
                        if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz) {
                            const double* src = Eb + (((int64_t)gz * a.ny + gy) * a.nx + gx) * 3 * NC + comp * NC +
                                                2 * (k == CD - 1 ? 0 : k);
                            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(le + 2 * c0),
                                                             16, 0, 0);
                        } else {
                            reinterpret_cast<double2*>(le)[c] = make_double2(0.0, 0.0);
                        }
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);  // the direct loads have written LDS
                __syncthreads();
                for (int j = threadIdx.x; j < EN * 3; j += PART_THREADS) le[j * lds_dual<NC>()] = 0.0;
            } else {
            // SB loads in flight per thread before their LDS writes
            constexpr int SN = EN * 3 * NC, SB = STAGE_BATCH;
#pragma unroll 1
            for (int j0 = 0; j0 < SN; j0 += SB * PART_THREADS) {
                double v[SB];
#pragma unroll
                for (int k = 0; k < SB; ++k) {
                    const int j = j0 + threadIdx.x + k * PART_THREADS;
                    const int node = j / (3 * NC), r = j - node * (3 * NC);
                    const int lx = node % ER, ly = (node / ER) % ER, lz = node / (ER * ER);
                    const int gx = ox + etile_off<F>() + lx, gy = oy + etile_off<F>() + ly, gz = oze + lz;
                    v[k] = (j < SN && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz)
                               ? Eb[(((int64_t)gz * a.ny + gy) * a.nx + gx) * 3 * NC + r]
                               : 0.0;
                }
#pragma unroll
                for (int k = 0; k < SB; ++k) {
                    const int j = j0 + threadIdx.x + k * PART_THREADS;
                    const int node = j / (3 * NC), r = j - node * (3 * NC);
                    if (j < SN) put_split<NC>(le + (node * 3 + r / NC) * lds_dual<NC>(), r % NC, v[k]);
                }
            }
            }
        }
        __syncthreads();
        pin_raw(next);
        {
            // software pipeline: a thread's loads for its next particle are
            // issued before the current one is processed (two iterations deep
            // measured 18% slower with 1e6 particles on 64^3 nodes)
#pragma unroll 1
            for (int i = i0; i < ck.z; i += STRIDE) {
                const RawState<LaneGroup<NC>::K> curst = next;
                const uint32_t kin = knext;
                const int32_t rin = rnext;
                if (i + STRIDE < ck.z) {
                    next = load_raw<NC>(a, (int64_t)ck.y + i + STRIDE, q);
                    if ((F & PF_SCATTER) && q == 0) {
                        knext = t.key_in[(int64_t)ck.y + i + STRIDE];
                        rnext = a.pid_in[(int64_t)ck.y + i + STRIDE];
                    }
                }
                const int64_t p = (int64_t)ck.y + i;
                // PF_SCATTER: the sorted slot is claimed just before the stores
                auto dest = [&]() -> int64_t {
                    pin_raw(next);
                    if constexpr ((F & PF_SCATTER) != 0)
                        return scatter_slot<G>(a, t, q, kin, rin, sclaim, ck.w, tx, ty, tz, use_tile);
                    else
                        return p;
                };
                particle_body<NC, F, true>(a, sv, smap, stau, p, dest, q, curst, lr, le, ox, oy, oz, oze, use_tile,
                                           e0, e1, e2, nf);
            }
        }
        if (F & PF_DEPOSIT) {
            __syncthreads();
            // node-major walk (NC consecutive lanes write one node's channels),
            // started at an item-dependent node so that items of the same tile
            // flushing at the same time hit different addresses
            constexpr int DN = dep_nodes<F>(), CS = dep_cstride<F>();
            const int rot = (int)((ci * 61u) % DN);
            for (int j = threadIdx.x; j < DN * NC; j += PART_THREADS) {
                const int ch = j % NC;
                int node = j / NC + rot;
                node -= node >= DN ? DN : 0;
                const double v = lr[ch * CS + node];
                if (v != 0.0) {
                    const int lx = node % TILE_R, ly = (node / TILE_R) % TILE_R, lz = node / (TILE_R * TILE_R);
                    const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
                    if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz)
                        unsafeAtomicAdd(sv.rho + (((int64_t)gz * a.ny + gy) * a.nx + gx) * NC + ch, v);
                }
            }
        }
    }
    if (cur >= 0) nonfinite_flush_wave(sv.cnt, nf, a.step);
    if ((F & (PF_DEPOSIT | PF_COUNT)) && cur >= 0) extent_flush(sv.cnt, e0, e1, e2, sext);
}

template <int NC, int F>
__global__ __launch_bounds__(PART_THREADS) void k_particles_tiled(PartArgs a, TiledArgs t) {
    static_assert((F & PF_SCATTER) == 0, "sorted stores: k_particles_sorted");
    tiled_body<NC, F>(a, t);
}

// The same kernel storing the state in sorted order (PF_SCATTER), held to
// two waves per SIMD: the slot claims add registers, which would otherwise
// leave room for one.
template <int NC, int F>
__global__ __launch_bounds__(PART_THREADS, 2) void k_particles_sorted(PartArgs a, TiledArgs t) {
    static_assert((F & PF_SCATTER) != 0, "unsorted stores: k_particles_tiled");
    tiled_body<NC, F>(a, t);
}

// Resident workgroups per CU of one tiled-kernel instance (queried once).
template <int NC, int FL>
static int tiled_occupancy() {
    static int occ = 0;
    if (occ == 0) {
        int v = 0;
        hipError_t e;
        if constexpr ((FL & PF_SCATTER) != 0)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_particles_sorted<NC, FL>, PART_THREADS, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_particles_tiled<NC, FL>, PART_THREADS, 0);
        if (e != hipSuccess || v < 1) v = 1;
        occ = v;
    }
    return occ;
}

template <int NC>
static int resident_nc(int flags) {
    switch (flags) {
        case PF_MAP | PF_DEPOSIT: return tiled_occupancy<NC, PF_MAP | PF_DEPOSIT>();
        case PF_KICK | PF_MAP | PF_DEPOSIT: return tiled_occupancy<NC, PF_KICK | PF_MAP | PF_DEPOSIT>();
        case PF_KICK | PF_MAP: return tiled_occupancy<NC, PF_KICK | PF_MAP>();
        case PF_MAP | PF_COUNT: return tiled_occupancy<NC, PF_MAP | PF_COUNT>();
        case PF_MAP: return tiled_occupancy<NC, PF_MAP>();
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO: return tiled_occupancy<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO>();
        case PF_KICK | PF_MAP | PF_EHALO: return tiled_occupancy<NC, PF_KICK | PF_MAP | PF_EHALO>();
        default: return tiled_occupancy<NC, PF_DEPOSIT>();
    }
}

// Resident workgroups of the tiled kernel on the whole device for the
// step's main flag set; also fills the per-instance cache of every instance
// of this channel count (so that no query happens during graph capture).
int particle_resident_blocks(dpic_ctx* cx) {
    int r = 0;
    const int all[8] = {PF_MAP | PF_DEPOSIT, PF_KICK | PF_MAP | PF_DEPOSIT, PF_KICK | PF_MAP, PF_MAP | PF_COUNT,
                        PF_MAP, PF_DEPOSIT, PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO, PF_KICK | PF_MAP | PF_EHALO};
    for (int f : all) {
        const int v = cx->NC == 1 ? resident_nc<1>(f) : (cx->NC == 8 ? resident_nc<8>(f) : resident_nc<16>(f));
        if (f == (PF_KICK | PF_MAP | PF_DEPOSIT)) r = v;
    }
    return r * (cx->cu_count > 0 ? cx->cu_count : 256);
}

template <int NC, int FL, bool TL>
static void launch_one(dpic_ctx* cx, const PartArgs& a, const TiledArgs& t, size_t max_items) {
    constexpr int G = LaneGroup<NC>::G;
    dim3 block(PART_THREADS);
    if (TL) {
        // default: four times the resident workgroups as the runtime reports
        // them, more than the work items at the default item size, so that
        // every item gets a workgroup of its own and the hardware dispatcher
        // balances them (a workgroup that found two items set the time)
        size_t g = cx->part_blocks > 0
                       ? (size_t)cx->part_blocks
                       : 4 * (size_t)tiled_occupancy<NC, FL>() * (size_t)(cx->cu_count > 0 ? cx->cu_count : 256);
        if (g > max_items) g = max_items;
        if (g < 1) g = 1;
        if constexpr ((FL & PF_SCATTER) != 0)
            hipLaunchKernelGGL((k_particles_sorted<NC, FL>), dim3((unsigned)g), block, 0, cx->stream, a, t);
        else
            hipLaunchKernelGGL((k_particles_tiled<NC, FL>), dim3((unsigned)g), block, 0, cx->stream, a, t);
    } else {
        const int64_t blocks = (a.used * G + PART_THREADS - 1) / PART_THREADS;
        hipLaunchKernelGGL((k_particles<NC, FL>), dim3((unsigned)blocks), block, 0, cx->stream, a);
    }
}

template <int NC, bool TL>
static hipError_t launch_particles_nc(dpic_ctx* cx, int flags, const PartArgs& a, const TiledArgs& t,
                                      size_t max_items) {
    if (a.used == 0) return hipSuccess;
    switch (flags) {
        case PF_MAP | PF_DEPOSIT: launch_one<NC, PF_MAP | PF_DEPOSIT, TL>(cx, a, t, max_items); break;
        case PF_KICK | PF_MAP | PF_DEPOSIT: launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT, TL>(cx, a, t, max_items); break;
        case PF_KICK | PF_MAP: launch_one<NC, PF_KICK | PF_MAP, TL>(cx, a, t, max_items); break;
        case PF_KICK | PF_MAP | PF_COUNT:  // the deterministic deposit follows as its own pass
            if constexpr (TL) return hipErrorInvalidValue;
            else launch_one<NC, PF_KICK | PF_MAP | PF_COUNT, TL>(cx, a, t, max_items);
            break;
        case PF_MAP | PF_COUNT: launch_one<NC, PF_MAP | PF_COUNT, TL>(cx, a, t, max_items); break;
        case PF_MAP: launch_one<NC, PF_MAP, TL>(cx, a, t, max_items); break;
        case PF_DEPOSIT: launch_one<NC, PF_DEPOSIT, TL>(cx, a, t, max_items); break;
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO:
            if constexpr (!TL) return hipErrorInvalidValue;
            launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO, TL>(cx, a, t, max_items);
            break;
        case PF_KICK | PF_MAP | PF_EHALO:
            if constexpr (!TL) return hipErrorInvalidValue;
            launch_one<NC, PF_KICK | PF_MAP | PF_EHALO, TL>(cx, a, t, max_items);
            break;
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_KEYS:
            launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_KEYS, TL>(cx, a, t, max_items);
            break;
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO | PF_KEYS:
            if constexpr (!TL) return hipErrorInvalidValue;
            launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO | PF_KEYS, TL>(cx, a, t, max_items);
            break;
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_SCATTER:
            if constexpr (!TL) return hipErrorInvalidValue;
            launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_SCATTER, TL>(cx, a, t, max_items);
            break;
        case PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO | PF_SCATTER:
            if constexpr (!TL) return hipErrorInvalidValue;
            launch_one<NC, PF_KICK | PF_MAP | PF_DEPOSIT | PF_EHALO | PF_SCATTER, TL>(cx, a, t, max_items);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_particles(dpic_ctx* cx, int flags, int e_tau, int map_off, bool tiled, bool write_keys,
                            bool scatter) {
    PartArgs a;
    a.step = cx->cur_step;
    a.st = cx->ws.st;
    a.cap = cx->dims.n_particles;
    a.used = cx->used;
    a.set = cx->ws.set;
    a.owner = cx->ws.owner;
    a.tau_off = ec_offset(cx, e_tau, EC_TAU);
    a.map_off = map_off;
    a.nx = cx->dims.nx;
    a.ny = cx->dims.ny;
    a.nz = cx->dims.nz;
    a.lo0 = cx->lo[0];
    a.lo1 = cx->lo[1];
    a.lo2 = cx->lo[2];
    a.ih0 = 1.0 / cx->h[0];
    a.ih1 = 1.0 / cx->h[1];
    a.ih2 = 1.0 / cx->h[2];
    a.kperp = cx->kperp;
    a.kpar = cx->kpar;
    a.key_out = nullptr;
    a.ktx = a.kty = a.knbins = 0;
    a.st_out = nullptr;
    a.pid_in = nullptr;
    a.pid_out = nullptr;
    if (write_keys && (flags & PF_DEPOSIT)) {
        int tk[3], nb = 0;
        if (!sort_geometry(cx, tk, &nb)) return hipErrorInvalidValue;
        a.key_out = cx->ws.key;
        a.ktx = tk[0];
        a.kty = tk[1];
        a.knbins = nb;
        flags |= PF_KEYS;
    }
    TiledArgs t{};
    size_t items = 0;
    if (tiled) {
        int tiles[3], nbins;
        if (!cx->chunks_valid || !sort_geometry(cx, tiles, &nbins)) return hipErrorInvalidValue;
        t.chunks = cx->ws.chunks;
        t.nchunks = cx->ws.nchunks;
        t.E0 = cx->ws.E;
        t.estride = (int64_t)cx->dims.nx * cx->dims.ny * cx->dims.nz * 3 * cx->NC;
        t.tx = tiles[0];
        t.ty = tiles[1];
        t.nbins = nbins;
        items = max_chunks(cx);
    }
    if (scatter) {
        // the bin starts and cursors come from the keys of the previous
        // launch (launch_sort_counts); keys and scatter never share a launch
        if (!tiled || (flags & PF_KEYS) || !(flags & PF_KICK) || !(flags & PF_DEPOSIT)) return hipErrorInvalidValue;
        a.st_out = cx->ws.st2;
        a.pid_in = cx->ws.pid;
        a.pid_out = cx->ws.pid2;
        t.key_in = cx->ws.key;
        t.cur = cx->ws.bins + (size_t)cx->B * t.nbins;
        flags |= PF_SCATTER;
    }
    // the tiles with the drift allowance wherever an E tile is staged (up
    // to 8 channels), and otherwise while the fields of all settings fit in
    // the caches (at 16 channels the flag only shapes the deposit tile)
    const double ebytes = (double)cx->B * cx->dims.nx * cx->dims.ny * cx->dims.nz * 3.0 * cx->NC * sizeof(double);
    if (tiled && (flags & PF_KICK) && (cx->NC <= 8 || ebytes <= EHALO_MAX_BYTES)) flags |= PF_EHALO;
    switch (cx->NC) {
        case 1: return tiled ? launch_particles_nc<1, true>(cx, flags, a, t, items) : launch_particles_nc<1, false>(cx, flags, a, t, items);
        case 8: return tiled ? launch_particles_nc<8, true>(cx, flags, a, t, items) : launch_particles_nc<8, false>(cx, flags, a, t, items);
        default: return tiled ? launch_particles_nc<16, true>(cx, flags, a, t, items) : launch_particles_nc<16, false>(cx, flags, a, t, items);
    }
}

// ---------------------------------------------------------------- read-back
// st [6][cap][NC] in storage order -> st2 [n][6][NC] in packed original order
template <int NC>
__global__ void k_canonical(const double* __restrict__ st, const int32_t* __restrict__ pid, int64_t used, int64_t cap,
                            const SettingDev* __restrict__ set, const int32_t* __restrict__ owner,
                            double* __restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= used) return;
    const SettingDev sd = set[owner[p / SEG]];
    if (p - sd.off >= sd.n) return;
    const int64_t q = pid[p];
#pragma unroll
    for (int j = 0; j < 6; ++j) out[(q * 6 + j) * NC + c] = st[((int64_t)j * cap + p) * NC + c];
}

hipError_t launch_canonical_state(dpic_ctx* cx) {
    const int64_t threads = cx->used * cx->NC;
    if (threads == 0) return hipSuccess;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    const Workspace& w = cx->ws;
    const int64_t cap = cx->dims.n_particles;
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_canonical<1>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2); break;
        case 8: hipLaunchKernelGGL(k_canonical<8>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2); break;
        default: hipLaunchKernelGGL(k_canonical<16>, grid, block, 0, cx->stream, w.st, w.pid, cx->used, cap, w.set, w.owner, w.st2); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- fill
__global__ void k_zero(double* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n; j += stride) p[j] = 0.0;
}

hipError_t launch_zero(dpic_ctx* cx, double* p, size_t n) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, cx->stream, p, n);
    return hipGetLastError();
}

}  // namespace dpic
