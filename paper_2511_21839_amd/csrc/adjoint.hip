// Reverse-mode adjoint of the value-only step (the dual step with no
// tangents): gradients of J = sum_plane w_plane eps_plane (raw emittances,
// Sec. 4) with respect to the lattice parameters and the six initial beam
// sizes, at a cost independent of their number.
//
// One step with half-step map A, step tau and kick coefficients kappa is
//   z1 = A z0;  p2 = p1 + tau kappa E(x1);  z3 = A z2,
// with E = D (G * rho), rho = sum_p q W(x_p) (CIC weights W). Its adjoint,
// for the adjoint l of z3, is
//   l2 = A^T l                                   (dJ/dA += l z2^T)
//   dJ/dtau += l2_p . kappa E_p,   a_p = tau kappa l2_p
//   l1_x = l2_x + sum_c grad W_c(x1) (a . E_c)  +  q sum_n grad W_n(x1) psi_n
//   psi = G * chi (open-boundary convolution), chi = D^T Abar, Abar = sum_p a_p W(x1_p)
//   l0 = A^T l1                                  (dJ/dA += l1 z0^T)
// D^T is the transposed central difference onto the ghost-ring window; G is
// even, so the adjoint solve is the same Hockney convolution with the input
// and output windows exchanged. Parameter gradients follow from dJ/dA and
// dJ/dtau per element and the derivatives of A and tau with respect to the
// parameters (the element constants evaluated with dual numbers).
//
// Particles are processed one lane each (value-only state, NC = 1).
#include <algorithm>

#include "context.hpp"

namespace dpic {

constexpr int ADJ_THREADS = 256;

struct AdjArgs {
    const double* st0;   // state at the step's start [6][cap]
    const double* E;     // this step's field [node][3]
    double* lam;         // adjoint of the state [6][cap]
    double* abar;        // adjoint field deposit [node][3]
    const double* psi;   // adjoint potential [node]
    const double* map;   // half-step map block of the element (9 values)
    const double* tau;   // step of the element
    double* gacc;        // per-element accumulator: dJ/dA (9), dJ/dtau
    int64_t n, cap;
    int nx, ny, nz;
    double lo0, lo1, lo2, ih0, ih1, ih2;
    double kperp, kpar, q;
};

struct Pos {
    int ix, iy, iz;
    double fx, fy, fz;
    bool inside;
};

__device__ __forceinline__ Pos pos_of(double x, double y, double z, const AdjArgs& a) {
    Pos r;
    const double sx = (x - a.lo0) * a.ih0, sy = (y - a.lo1) * a.ih1, sz = (z - a.lo2) * a.ih2;
    r.inside = (sx >= 0.0) && (sx < (double)(a.nx - 1)) && (sy >= 0.0) && (sy < (double)(a.ny - 1)) && (sz >= 0.0) &&
               (sz < (double)(a.nz - 1));
    const double flx = floor(sx), fly = floor(sy), flz = floor(sz);
    r.ix = (int)flx;
    r.iy = (int)fly;
    r.iz = (int)flz;
    r.fx = sx - flx;
    r.fy = sy - fly;
    r.fz = sz - flz;
    return r;
}

// block sum of NV values, one atomic per value per block
template <int NV>
__device__ __forceinline__ void block_accumulate(double (&v)[NV], double* out) {
    __shared__ double red[ADJ_THREADS / 64][NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < ADJ_THREADS / 64; ++w) s += red[w][threadIdx.x];
        if (s != 0.0) unsafeAtomicAdd(out + threadIdx.x, s);
    }
}

struct St6 {
    double x, px, y, py, z, d;
};

__device__ __forceinline__ St6 load6(const double* s, int64_t p, int64_t cap) {
    return St6{s[p], s[cap + p], s[2 * cap + p], s[3 * cap + p], s[4 * cap + p], s[5 * cap + p]};
}

__device__ __forceinline__ St6 apply_map(const St6& z, const double* m) {
    St6 r;
    r.x = m[0] * z.x + m[1] * z.px;
    r.px = m[2] * z.x + m[3] * z.px;
    r.y = m[4] * z.y + m[5] * z.py;
    r.py = m[6] * z.y + m[7] * z.py;
    r.z = z.z + m[8] * z.d;
    r.d = z.d;
    return r;
}

// l <- A^T l, and dJ/dA += l z^T (z the map's input)
__device__ __forceinline__ void map_adjoint(St6& l, const St6& zin, const double* m, double (&g)[10]) {
    g[0] += l.x * zin.x;
    g[1] += l.x * zin.px;
    g[2] += l.px * zin.x;
    g[3] += l.px * zin.px;
    g[4] += l.y * zin.y;
    g[5] += l.y * zin.py;
    g[6] += l.py * zin.y;
    g[7] += l.py * zin.py;
    g[8] += l.z * zin.d;
    const double lx = m[0] * l.x + m[2] * l.px, lpx = m[1] * l.x + m[3] * l.px;
    const double ly = m[4] * l.y + m[6] * l.py, lpy = m[5] * l.y + m[7] * l.py;
    l.d += m[8] * l.z;
    l.x = lx;
    l.px = lpx;
    l.y = ly;
    l.py = lpy;
}

// Second half of the step backward for particle p, the kick's adjoint, the
// direct position term and the deposit of the adjoint field: into the LDS
// tile lt (nodes [o, o + TILE_R)^3 around a work item's grid tile, three
// components per node) when all 8 corners fall inside it, else by global
// atomics.
__device__ __forceinline__ void adj_kick_particle(const AdjArgs& a, int64_t p, double* lt, int ox, int oy, int oz,
                                                  double (&g)[10]) {
    double m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = a.map[k];
    const double tau = a.tau[0];
    const St6 z0 = load6(a.st0, p, a.cap);
    St6 z2 = apply_map(z0, m);
    const Pos c = pos_of(z2.x, z2.y, z2.z, a);
    double ex = 0.0, ey = 0.0, ez = 0.0;
    const int64_t sxy = (int64_t)a.nx * a.ny;
    const int64_t n0 = ((int64_t)c.iz * a.ny + c.iy) * a.nx + c.ix;
    if (c.inside) {
#pragma unroll
        for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int ky = 0; ky < 2; ++ky)
#pragma unroll
                for (int kx = 0; kx < 2; ++kx) {
                    const double w = (kx ? c.fx : 1.0 - c.fx) * (ky ? c.fy : 1.0 - c.fy) * (kz ? c.fz : 1.0 - c.fz);
                    const double* e = a.E + (n0 + kx + ky * a.nx + kz * sxy) * 3;
                    ex += w * e[0];
                    ey += w * e[1];
                    ez += w * e[2];
                }
        z2.px += tau * (ex * a.kperp);
        z2.py += tau * (ey * a.kperp);
        z2.d += tau * (ez * a.kpar);
    }
    St6 l = load6(a.lam, p, a.cap);
    map_adjoint(l, z2, m, g);
    if (c.inside) {
        g[9] += l.px * a.kperp * ex + l.py * a.kperp * ey + l.d * a.kpar * ez;
        const double ax = tau * a.kperp * l.px, ay = tau * a.kperp * l.py, az = tau * a.kpar * l.d;
        const int lx = c.ix - ox, ly = c.iy - oy, lz = c.iz - oz;
        const bool local = lt && lx >= 0 && lx <= TILE_R - 2 && ly >= 0 && ly <= TILE_R - 2 && lz >= 0 &&
                           lz <= TILE_R - 2;
        const int l0 = (lz * TILE_R + ly) * TILE_R + lx;
        double dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
        for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int ky = 0; ky < 2; ++ky)
#pragma unroll
                for (int kx = 0; kx < 2; ++kx) {
                    const double wx = kx ? c.fx : 1.0 - c.fx, wy = ky ? c.fy : 1.0 - c.fy, wz = kz ? c.fz : 1.0 - c.fz;
                    const double gx = (kx ? a.ih0 : -a.ih0), gy = (ky ? a.ih1 : -a.ih1), gz = (kz ? a.ih2 : -a.ih2);
                    const int64_t node = n0 + kx + ky * a.nx + kz * sxy;
                    const double* e = a.E + node * 3;
                    const double s = ax * e[0] + ay * e[1] + az * e[2];
                    dx += gx * wy * wz * s;
                    dy += wx * gy * wz * s;
                    dz += wx * wy * gz * s;
                    const double w = wx * wy * wz;
                    double* ab = local ? lt + (l0 + kx + ky * TILE_R + kz * TILE_R * TILE_R) * 3 : a.abar + node * 3;
                    unsafeAtomicAdd(ab + 0, w * ax);
                    unsafeAtomicAdd(ab + 1, w * ay);
                    unsafeAtomicAdd(ab + 2, w * az);
                }
        l.x += dx;
        l.y += dy;
        l.z += dz;
    }
    a.lam[p] = l.x;
    a.lam[a.cap + p] = l.px;
    a.lam[2 * a.cap + p] = l.y;
    a.lam[3 * a.cap + p] = l.py;
    a.lam[4 * a.cap + p] = l.z;
    a.lam[5 * a.cap + p] = l.d;
}

__global__ __launch_bounds__(ADJ_THREADS) void k_adj_kick(AdjArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double g[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = 0.0;
    if (p < a.n) adj_kick_particle(a, p, nullptr, 0, 0, 0, g);
    block_accumulate<10>(g, a.gacc);
}

// The same over the tiled work list (items of particles sorted into one grid
// tile): each item accumulates its adjoint-field deposit in an LDS tile and
// flushes the nonzero nodes by global atomics. With the particles sorted by
// tile, consecutive threads otherwise hit the same nodes with global
// atomics: 6.3 ms per step at 1e6 particles on 64^3 nodes.
struct AdjTiles {
    const int4* chunks;
    const uint32_t* nchunks;
    int tx, ty, nbins;
};

__global__ __launch_bounds__(ADJ_THREADS) void k_adj_kick_tiled(AdjArgs a, AdjTiles t) {
    constexpr int TN = TILE_R * TILE_R * TILE_R;
    __shared__ double lt[TN * 3];
    double g[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = 0.0;
    const uint32_t nck = *t.nchunks;
#pragma unroll 1
    for (uint32_t ci = blockIdx.x; ci < nck; ci += gridDim.x) {
        const int4 ck = t.chunks[ci];
        if (ci != blockIdx.x) __syncthreads();  // the previous item's flush is done with lt
        for (int j = threadIdx.x; j < TN * 3; j += ADJ_THREADS) lt[j] = 0.0;
        const bool use_tile = ck.x < t.nbins - 1;
        const int tx = ck.x % t.tx, ty = (ck.x / t.tx) % t.ty, tz = ck.x / (t.tx * t.ty);
        const int ox = tx * TILE_EDGE - TILE_HALO, oy = ty * TILE_EDGE - TILE_HALO, oz = tz * TILE_EDGE - TILE_HALO;
        __syncthreads();
        for (int i = threadIdx.x; i < ck.z; i += ADJ_THREADS)
            adj_kick_particle(a, (int64_t)ck.y + i, use_tile ? lt : nullptr, ox, oy, oz, g);
        __syncthreads();
        if (use_tile) {
            for (int j = threadIdx.x; j < TN * 3; j += ADJ_THREADS) {
                const double v = lt[j];
                if (v == 0.0) continue;
                const int node = j / 3, comp = j - node * 3;
                const int gx = ox + node % TILE_R, gy = oy + (node / TILE_R) % TILE_R, gz = oz + node / (TILE_R * TILE_R);
                if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz)
                    unsafeAtomicAdd(a.abar + (((int64_t)gz * a.ny + gy) * a.nx + gx) * 3 + comp, v);
            }
        }
    }
    block_accumulate<10>(g, a.gacc);
}

// chi = D^T Abar on the ghost-ring window (index shifted by one): the
// transpose of E_x(i) = cx (phi(i+1) - phi(i-1)) sends cx Abar_x(i) to
// position i+1 and -cx Abar_x(i) to position i-1.
__global__ void k_adj_divergence(const double* __restrict__ abar, double* __restrict__ chi, int nx, int ny, int nz,
                                 double cx, double cy, double cz) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int gx = nx + 2, gy = ny + 2, gz = nz + 2;
    if (gid >= (int64_t)gx * gy * gz) return;
    const int xp = (int)(gid % gx), yp = (int)((gid / gx) % gy), zp = (int)(gid / ((int64_t)gx * gy));
    auto A = [&](int i, int j, int k, int comp) -> double {
        if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) return 0.0;
        return abar[(((int64_t)k * ny + j) * nx + i) * 3 + comp];
    };
    const double v = cx * (A(xp - 2, yp - 1, zp - 1, 0) - A(xp, yp - 1, zp - 1, 0)) +
                     cy * (A(xp - 1, yp - 2, zp - 1, 1) - A(xp - 1, yp, zp - 1, 1)) +
                     cz * (A(xp - 1, yp - 1, zp - 2, 2) - A(xp - 1, yp - 1, zp, 2));
    chi[gid] = v;
}

// Indirect position term through the adjoint potential, then the first half
// map backward.
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_indirect(AdjArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double g[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = 0.0;
    if (p < a.n) {
        double m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = a.map[k];
        const St6 z0 = load6(a.st0, p, a.cap);
        const St6 z1 = apply_map(z0, m);
        const Pos c = pos_of(z1.x, z1.y, z1.z, a);
        St6 l = load6(a.lam, p, a.cap);
        if (c.inside) {
            const int64_t sxy = (int64_t)a.nx * a.ny;
            const int64_t n0 = ((int64_t)c.iz * a.ny + c.iy) * a.nx + c.ix;
            double dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
            for (int kz = 0; kz < 2; ++kz)
#pragma unroll
                for (int ky = 0; ky < 2; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 2; ++kx) {
                        const double wx = kx ? c.fx : 1.0 - c.fx, wy = ky ? c.fy : 1.0 - c.fy, wz = kz ? c.fz : 1.0 - c.fz;
                        const double gx = (kx ? a.ih0 : -a.ih0), gy = (ky ? a.ih1 : -a.ih1), gz = (kz ? a.ih2 : -a.ih2);
                        const double s = a.psi[n0 + kx + ky * a.nx + kz * sxy];
                        dx += gx * wy * wz * s;
                        dy += wx * gy * wz * s;
                        dz += wx * wy * gz * s;
                    }
            l.x += a.q * dx;
            l.y += a.q * dy;
            l.z += a.q * dz;
        }
        map_adjoint(l, z0, m, g);
        a.lam[p] = l.x;
        a.lam[a.cap + p] = l.px;
        a.lam[2 * a.cap + p] = l.y;
        a.lam[3 * a.cap + p] = l.py;
        a.lam[4 * a.cap + p] = l.z;
        a.lam[5 * a.cap + p] = l.d;
    }
    block_accumulate<10>(g, a.gacc);
}

// Adjoint of J = sum_plane w eps with eps = sqrt(<u^2><p^2> - <u p>^2):
// dJ/du_p = w (C u - B p)/(eps N), dJ/dp_p = w (A p - B u)/(eps N).
__global__ void k_adj_terminal(const double* __restrict__ st, int64_t n, int64_t cap, const double* __restrict__ mom,
                               double w0, double w1, double w2, double* __restrict__ lam) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double w[3] = {w0, w1, w2};
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
        const double A = mom[pl * 5 + 0], B = mom[pl * 5 + 1], C = mom[pl * 5 + 2];
        const double u = st[(2 * pl) * cap + p], q = st[(2 * pl + 1) * cap + p];
        double lu = 0.0, lq = 0.0;
        if (w[pl] != 0.0) {
            const double eps = sqrt(A * C - B * B);
            const double s = w[pl] / (eps * (double)n);
            lu = s * (C * u - B * q);
            lq = s * (A * q - B * u);
        }
        lam[(2 * pl) * cap + p] = lu;
        lam[(2 * pl + 1) * cap + p] = lq;
    }
}

// dJ/dsigma_j = sum_p l_j(p) xi_j(p) (zeta_j = sigma_j xi_j at the start)
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_sigma(const double* __restrict__ lam, const double* __restrict__ xi,
                                                           const int32_t* __restrict__ pid, int64_t n, int64_t cap,
                                                           double* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double g[6] = {0, 0, 0, 0, 0, 0};
    if (p < n) {
        const int64_t o = pid[p];
#pragma unroll
        for (int j = 0; j < 6; ++j) g[j] = lam[j * cap + p] * xi[o * 6 + j];
    }
    block_accumulate<6>(g, out);
}

// dJ/dp_j = sum_e (dJ/dA_e . dA_e/dp_j + dJ/dtau_e dtau_e/dp_j), with the
// element constants evaluated as duals (channel 1+j = d/dp_j).
template <int NCD>
__global__ void k_adj_params(const double* __restrict__ gacc, const double* __restrict__ ecd, int n_elem, int np,
                             double* __restrict__ out) {
    const int j = threadIdx.x;
    if (j >= np) return;
    double s = 0.0;
    for (int e = 0; e < n_elem; ++e) {
        const double* ce = ecd + (size_t)e * EC_N * NCD;
        for (int m = 0; m < MB_N; ++m) s += gacc[e * 10 + m] * ce[(EC_HALF + m) * NCD + 1 + j];
        s += gacc[e * 10 + 9] * ce[EC_TAU * NCD + 1 + j];
    }
    out[j] = s;
}

// ---------------------------------------------------------------- launchers
static AdjArgs adj_args(dpic_ctx* cx, int e, const double* st0, const double* E) {
    AdjArgs a;
    a.st0 = st0;
    a.E = E;
    a.lam = cx->adj.lam;
    a.abar = cx->ws.E;
    a.psi = cx->ws.rho;
    a.map = cx->ws.ec + (size_t)e * EC_N + EC_HALF;
    a.tau = cx->ws.ec + (size_t)e * EC_N + EC_TAU;
    a.gacc = cx->adj.gacc + (size_t)e * 10;
    a.n = cx->n;
    a.cap = cx->dims.n_particles;
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
    a.q = cx->n > 0 ? cx->bunch_charge / (double)cx->n : 0.0;
    return a;
}

hipError_t launch_adj_terminal(dpic_ctx* cx, const double w[3]) {
    hipError_t e = launch_moments(cx);
    if (e != hipSuccess || cx->n == 0) return e;
    const unsigned blocks = (unsigned)((cx->n + ADJ_THREADS - 1) / ADJ_THREADS);
    hipLaunchKernelGGL(k_adj_terminal, dim3(blocks), dim3(ADJ_THREADS), 0, cx->stream, cx->ws.st, cx->n,
                       cx->dims.n_particles, cx->ws.mom, w[0], w[1], w[2], cx->adj.lam);
    return hipGetLastError();
}

hipError_t launch_adj_step(dpic_ctx* cx, int e, const double* st0, const double* E, bool space_charge) {
    if (cx->n == 0) return hipSuccess;
    const int nx = cx->dims.nx, ny = cx->dims.ny, nz = cx->dims.nz;
    const unsigned blocks = (unsigned)((cx->n + ADJ_THREADS - 1) / ADJ_THREADS);
    AdjArgs a = adj_args(cx, e, st0, E);
    hipError_t err;
    if (!space_charge) {
        // no field: both half maps backward only (the kick terms vanish)
        a.q = 0.0;
        a.kperp = 0.0;
        a.kpar = 0.0;
    }
    if ((err = launch_zero(cx, cx->ws.E, (size_t)nx * ny * nz * 3)) != hipSuccess) return err;
    int tiles[3], nbins = 0;
    if (cx->chunks_valid && cx->B == 1 && sort_geometry(cx, tiles, &nbins)) {
        // the work list of the first sort (the adjoint keeps that order)
        const AdjTiles t{cx->ws.chunks, cx->ws.nchunks, tiles[0], tiles[1], nbins};
        const size_t items = max_chunks(cx);
        hipLaunchKernelGGL(k_adj_kick_tiled, dim3((unsigned)std::max<size_t>(items, 1)), dim3(ADJ_THREADS), 0,
                           cx->stream, a, t);
    } else {
        hipLaunchKernelGGL(k_adj_kick, dim3(blocks), dim3(ADJ_THREADS), 0, cx->stream, a);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (space_charge) {
        const int64_t g = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
        const double cxx = -0.5 / cx->h[0], cyy = -0.5 / cx->h[1], czz = -0.5 / (cx->h[2] * cx->gamma0);
        hipLaunchKernelGGL(k_adj_divergence, dim3((unsigned)((g + 255) / 256)), dim3(256), 0, cx->stream, cx->ws.E,
                           cx->ws.phi, nx, ny, nz, cxx, cyy, czz);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        const int nin[3] = {nx + 2, ny + 2, nz + 2};
        const int nout[3] = {nx, ny, nz};
        if ((err = launch_conv(cx, cx->ws.phi, nin, cx->ws.rho, nout, -1, 1, 1)) != hipSuccess) return err;
    } else {
        if ((err = launch_zero(cx, cx->ws.rho, (size_t)nx * ny * nz)) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_adj_indirect, dim3(blocks), dim3(ADJ_THREADS), 0, cx->stream, a);
    return hipGetLastError();
}

hipError_t launch_adj_finish(dpic_ctx* cx, int np) {
    hipError_t e;
    if ((e = launch_zero(cx, cx->adj.grad, (size_t)DPIC_MAX_PARAMS + 6)) != hipSuccess) return e;
    if (cx->n > 0) {
        const unsigned blocks = (unsigned)((cx->n + ADJ_THREADS - 1) / ADJ_THREADS);
        hipLaunchKernelGGL(k_adj_sigma, dim3(blocks), dim3(ADJ_THREADS), 0, cx->stream, cx->adj.lam, cx->adj.xi,
                           cx->ws.pid, cx->n, cx->dims.n_particles, cx->adj.grad + DPIC_MAX_PARAMS);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (np > 0) {
        switch (cx->adj.ncd) {
            case 8: hipLaunchKernelGGL(k_adj_params<8>, dim3(1), dim3(64), 0, cx->stream, cx->adj.gacc, cx->adj.ec_dual, cx->n_elem, np, cx->adj.grad); break;
            case 16: hipLaunchKernelGGL(k_adj_params<16>, dim3(1), dim3(64), 0, cx->stream, cx->adj.gacc, cx->adj.ec_dual, cx->n_elem, np, cx->adj.grad); break;
            default: return hipErrorInvalidValue;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dpic
