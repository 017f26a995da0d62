// Particle-side kernels: per-element dual constants, beam initialisation,
// the fused gather / kick / half-map / deposit kernel, canonical read-back.
//
// Thread mapping: one lane per (particle, channel); a particle's NC lanes are
// consecutive, so a wavefront handles 64/NC particles and every coordinate of
// a particle is one contiguous NC*8-byte run (tangents interleaved, SoA over
// coordinates).
#include "context.hpp"

namespace dpic {

// ---------------------------------------------------------------- lattice
struct ElemTable {
    int kind[DPIC_MAX_ELEMENTS];
    int nsteps[DPIC_MAX_ELEMENTS];
};

struct Map2 {
    LD a, b, c, d;
};

// Exact half-step map of one plane with signed strength kk over length s
// (Sec. 4 quadrupole maps; kk > 0 focusing, kk < 0 defocusing). Below
// |kk s^2| < 1e-8 the Taylor series in u = kk s^2 to u^3 is used.
__device__ Map2 plane_map(LD kk, LD s) {
    LD u = kk * s * s;
    if (fabs(u.v) < 1e-8) {
        LD cc = 1.0 - u * 0.5 + u * u * (1.0 / 24.0) - u * u * u * (1.0 / 720.0);
        LD sn = s * (1.0 - u * (1.0 / 6.0) + u * u * (1.0 / 120.0) - u * u * u * (1.0 / 5040.0));
        return Map2{cc, sn, -(kk * sn), cc};
    }
    if (kk.v > 0) {
        LD r = dsqrt(kk);
        LD th = r * s;
        LD ct = dcos(th), st = dsin(th);
        return Map2{ct, st / r, -(r * st), ct};
    }
    LD r = dsqrt(-kk);
    LD th = r * s;
    LD ch = dcosh(th), sh = dsinh(th);
    return Map2{ch, sh / r, r * sh, ch};
}

template <int NC>
__global__ void k_element_consts(ElemTable tab, int n_elem, const double* __restrict__ elem_in,
                                 double* __restrict__ ec, double inv_g2) {
    const int e = blockIdx.x;
    const int c = threadIdx.x;
    if (e >= n_elem || c >= NC) return;
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
    o[(EC_AX + 0) * NC] = ldchan(ax.a, c);
    o[(EC_AX + 1) * NC] = ldchan(ax.b, c);
    o[(EC_AX + 2) * NC] = ldchan(ax.c, c);
    o[(EC_AX + 3) * NC] = ldchan(ax.d, c);
    o[(EC_AY + 0) * NC] = ldchan(ay.a, c);
    o[(EC_AY + 1) * NC] = ldchan(ay.b, c);
    o[(EC_AY + 2) * NC] = ldchan(ay.c, c);
    o[(EC_AY + 3) * NC] = ldchan(ay.d, c);
    o[EC_SLIP * NC] = ldchan(slip, c);
}

hipError_t launch_element_consts(dpic_ctx* cx) {
    ElemTable tab{};
    for (int e = 0; e < cx->n_elem; ++e) {
        tab.kind[e] = cx->kind[e];
        tab.nsteps[e] = cx->n_steps[e];
    }
    const double inv_g2 = 1.0 / (cx->gamma0 * cx->gamma0);
    dim3 grid(cx->n_elem), block(cx->NC < 64 ? 64 : cx->NC);
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_element_consts<1>, grid, block, 0, cx->stream, tab, cx->n_elem, cx->ws.elem_in, cx->ws.ec, inv_g2); break;
        case 8: hipLaunchKernelGGL(k_element_consts<8>, grid, block, 0, cx->stream, tab, cx->n_elem, cx->ws.elem_in, cx->ws.ec, inv_g2); break;
        default: hipLaunchKernelGGL(k_element_consts<16>, grid, block, 0, cx->stream, tab, cx->n_elem, cx->ws.elem_in, cx->ws.ec, inv_g2); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- beam init
struct SigmaDual {
    double s[6][16];  // [coord][channel]: sigma_j value and its seed row
};

template <int NC>
__global__ void k_init_beam(const double* __restrict__ xi, int64_t n, int64_t cap, SigmaDual sig,
                            double* __restrict__ st, int32_t* __restrict__ pid) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= n) return;
#pragma unroll
    for (int j = 0; j < 6; ++j) st[((int64_t)j * cap + p) * NC + c] = sig.s[j][c] * xi[p * 6 + j];
    if (c == 0) pid[p] = (int32_t)p;
}

hipError_t launch_init_beam(dpic_ctx* cx, const double* xi, const double* sig_dual) {
    SigmaDual sd{};
    for (int j = 0; j < 6; ++j)
        for (int c = 0; c < cx->NC; ++c) sd.s[j][c] = sig_dual[j * cx->NC + c];
    const int64_t threads = cx->n * cx->NC;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    if (threads == 0) return hipSuccess;
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_init_beam<1>, grid, block, 0, cx->stream, xi, cx->n, cx->dims.n_particles, sd, cx->ws.st, cx->ws.pid); break;
        case 8: hipLaunchKernelGGL(k_init_beam<8>, grid, block, 0, cx->stream, xi, cx->n, cx->dims.n_particles, sd, cx->ws.st, cx->ws.pid); break;
        default: hipLaunchKernelGGL(k_init_beam<16>, grid, block, 0, cx->stream, xi, cx->n, cx->dims.n_particles, sd, cx->ws.st, cx->ws.pid); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused step
struct PartArgs {
    double* st;
    int64_t n, cap;
    const double* ec;
    int e_cur, e_next;
    const double* E;
    double* rho;
    int nx, ny, nz;
    double lo0, lo1, lo2, ih0, ih1, ih2;
    double kperp, kpar, q;
    unsigned long long* cnt;
};

struct Cic {
    int ix, iy, iz;
    LD fx, fy, fz;
    bool inside;
};

// Cell and dual fractional offset per dimension: s = (u - lo)/h, cell floor(s),
// inside iff 0 <= s < n-1 in every dimension.
__device__ __forceinline__ Cic cic_of(LD x, LD y, LD z, const PartArgs& a) {
    Cic r;
    const double sx = (x.v - a.lo0) * a.ih0;
    const double sy = (y.v - a.lo1) * a.ih1;
    const double sz = (z.v - a.lo2) * a.ih2;
    r.inside = (sx >= 0.0) && (sx < (double)(a.nx - 1)) && (sy >= 0.0) && (sy < (double)(a.ny - 1)) &&
               (sz >= 0.0) && (sz < (double)(a.nz - 1));
    const double flx = floor(sx), fly = floor(sy), flz = floor(sz);
    r.ix = (int)flx;
    r.iy = (int)fly;
    r.iz = (int)flz;
    r.fx = LD{sx - flx, x.t * a.ih0};
    r.fy = LD{sy - fly, y.t * a.ih1};
    r.fz = LD{sz - flz, z.t * a.ih2};
    return r;
}

template <int NC>
__device__ __forceinline__ void half_map(LD& x, LD& px, LD& y, LD& py, LD& z, const LD& d,
                                         const double* __restrict__ e, int c) {
    LD a = ldload(e + (EC_AX + 0) * NC, c), b = ldload(e + (EC_AX + 1) * NC, c);
    LD cc = ldload(e + (EC_AX + 2) * NC, c), dd = ldload(e + (EC_AX + 3) * NC, c);
    LD nx = a * x + b * px;
    LD npx = cc * x + dd * px;
    x = nx;
    px = npx;
    a = ldload(e + (EC_AY + 0) * NC, c);
    b = ldload(e + (EC_AY + 1) * NC, c);
    cc = ldload(e + (EC_AY + 2) * NC, c);
    dd = ldload(e + (EC_AY + 3) * NC, c);
    LD ny = a * y + b * py;
    LD npy = cc * y + dd * py;
    y = ny;
    py = npy;
    LD slip = ldload(e + EC_SLIP * NC, c);
    z = z + slip * d;
}

template <int NC, int F>
__global__ __launch_bounds__(256) void k_particles(PartArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    const bool valid = p < a.n;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    if (valid) {
        const int64_t cs = a.cap * NC;
        double* sp = a.st + p * NC;
        LD x = ldload(sp, c), px = ldload(sp + cs, c), y = ldload(sp + 2 * cs, c);
        LD py = ldload(sp + 3 * cs, c), z = ldload(sp + 4 * cs, c), d = ldload(sp + 5 * cs, c);
        const int64_t sxy = (int64_t)a.nx * a.ny;
        if (F & PF_KICK) {
            Cic g = cic_of(x, y, z, a);
            if (g.inside) {
                const LD wx0 = 1.0 - g.fx, wy0 = 1.0 - g.fy, wz0 = 1.0 - g.fz;
                const int64_t n0 = ((int64_t)g.iz * a.ny + g.iy) * a.nx + g.ix;
                LD ex = ldc(0.0), ey = ldc(0.0), ez = ldc(0.0);
#pragma unroll
                for (int kz = 0; kz < 2; ++kz) {
                    const LD wz = kz ? g.fz : wz0;
#pragma unroll
                    for (int ky = 0; ky < 2; ++ky) {
                        const LD wyz = (ky ? g.fy : wy0) * wz;
#pragma unroll
                        for (int kx = 0; kx < 2; ++kx) {
                            const LD w = (kx ? g.fx : wx0) * wyz;
                            const double* ep = a.E + (n0 + kx + ky * a.nx + kz * sxy) * 3 * NC;
                            ex = fmad(w, ldload(ep, c), ex);
                            ey = fmad(w, ldload(ep + NC, c), ey);
                            ez = fmad(w, ldload(ep + 2 * NC, c), ez);
                        }
                    }
                }
                const LD tau = ldload(a.ec + (size_t)a.e_cur * EC_N * NC + EC_TAU * NC, c);
                px = px + tau * (ex * a.kperp);
                py = py + tau * (ey * a.kperp);
                d = d + tau * (ez * a.kpar);
            }
        }
        if (F & PF_HALF_CUR) half_map<NC>(x, px, y, py, z, d, a.ec + (size_t)a.e_cur * EC_N * NC, c);
        if (F & PF_HALF_NEXT) half_map<NC>(x, px, y, py, z, d, a.ec + (size_t)a.e_next * EC_N * NC, c);
        if (F & (PF_DEPOSIT | PF_COUNT)) {
            Cic g = cic_of(x, y, z, a);
            if (g.inside) {
                if (F & PF_DEPOSIT) {
                    const LD wx0 = 1.0 - g.fx, wy0 = 1.0 - g.fy, wz0 = 1.0 - g.fz;
                    const int64_t n0 = ((int64_t)g.iz * a.ny + g.iy) * a.nx + g.ix;
#pragma unroll
                    for (int kz = 0; kz < 2; ++kz) {
                        const LD wz = kz ? g.fz : wz0;
#pragma unroll
                        for (int ky = 0; ky < 2; ++ky) {
                            const LD wyz = (ky ? g.fy : wy0) * wz;
#pragma unroll
                            for (int kx = 0; kx < 2; ++kx) {
                                const LD w = (kx ? g.fx : wx0) * wyz;
                                const int64_t node = n0 + kx + ky * a.nx + kz * sxy;
                                unsafeAtomicAdd(a.rho + node * NC + c, ldchan(w, c) * a.q);
                            }
                        }
                    }
                }
            } else if (c == 0) {
                atomicAdd(a.cnt + CNT_OUTSIDE, 1ull);
            }
            e0 = fabs(x.v);
            e1 = fabs(y.v);
            e2 = fabs(z.v);
        }
        sp[0 * cs + c] = ldchan(x, c);
        sp[1 * cs + c] = ldchan(px, c);
        sp[2 * cs + c] = ldchan(y, c);
        sp[3 * cs + c] = ldchan(py, c);
        sp[4 * cs + c] = ldchan(z, c);
        sp[5 * cs + c] = ldchan(d, c);
    }
    if (F & (PF_DEPOSIT | PF_COUNT)) {
        // wavefront max of the extents (all 64 lanes take part), one atomic per wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            e0 = fmax(e0, __shfl_xor(e0, off, 64));
            e1 = fmax(e1, __shfl_xor(e1, off, 64));
            e2 = fmax(e2, __shfl_xor(e2, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMax(a.cnt + CNT_EXT_X, (unsigned long long)__double_as_longlong(e0));
            atomicMax(a.cnt + CNT_EXT_Y, (unsigned long long)__double_as_longlong(e1));
            atomicMax(a.cnt + CNT_EXT_Z, (unsigned long long)__double_as_longlong(e2));
        }
    }
}

template <int NC>
static hipError_t launch_particles_nc(dpic_ctx* cx, int flags, const PartArgs& a) {
    const int64_t threads = a.n * NC;
    if (threads == 0) return hipSuccess;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    hipStream_t s = cx->stream;
    switch (flags) {
        case PF_HALF_NEXT | PF_DEPOSIT:
            hipLaunchKernelGGL((k_particles<NC, PF_HALF_NEXT | PF_DEPOSIT>), grid, block, 0, s, a); break;
        case PF_KICK | PF_HALF_CUR | PF_HALF_NEXT | PF_DEPOSIT:
            hipLaunchKernelGGL((k_particles<NC, PF_KICK | PF_HALF_CUR | PF_HALF_NEXT | PF_DEPOSIT>), grid, block, 0, s, a); break;
        case PF_KICK | PF_HALF_CUR:
            hipLaunchKernelGGL((k_particles<NC, PF_KICK | PF_HALF_CUR>), grid, block, 0, s, a); break;
        case PF_HALF_NEXT | PF_COUNT:
            hipLaunchKernelGGL((k_particles<NC, PF_HALF_NEXT | PF_COUNT>), grid, block, 0, s, a); break;
        case PF_HALF_CUR | PF_HALF_NEXT | PF_COUNT:
            hipLaunchKernelGGL((k_particles<NC, PF_HALF_CUR | PF_HALF_NEXT | PF_COUNT>), grid, block, 0, s, a); break;
        case PF_HALF_CUR:
            hipLaunchKernelGGL((k_particles<NC, PF_HALF_CUR>), grid, block, 0, s, a); break;
        case PF_DEPOSIT:
            hipLaunchKernelGGL((k_particles<NC, PF_DEPOSIT>), grid, block, 0, s, a); break;
        case PF_KICK:
            hipLaunchKernelGGL((k_particles<NC, PF_KICK>), grid, block, 0, s, a); break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_particles(dpic_ctx* cx, int flags, int e_cur, int e_next) {
    PartArgs a;
    a.st = cx->ws.st;
    a.n = cx->n;
    a.cap = cx->dims.n_particles;
    a.ec = cx->ws.ec;
    a.e_cur = e_cur;
    a.e_next = e_next;
    a.E = cx->ws.E;
    a.rho = cx->ws.rho;
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
    a.cnt = cx->ws.counters;
    switch (cx->NC) {
        case 1: return launch_particles_nc<1>(cx, flags, a);
        case 8: return launch_particles_nc<8>(cx, flags, a);
        default: return launch_particles_nc<16>(cx, flags, a);
    }
}

// ---------------------------------------------------------------- read-back
// st [6][cap][NC] in storage order -> st2 [n][6][NC] in original particle order
template <int NC>
__global__ void k_canonical(const double* __restrict__ st, const int32_t* __restrict__ pid, int64_t n,
                            int64_t cap, double* __restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= n) return;
    const int64_t q = pid[p];
#pragma unroll
    for (int j = 0; j < 6; ++j) out[(q * 6 + j) * NC + c] = st[((int64_t)j * cap + p) * NC + c];
}

hipError_t launch_canonical_state(dpic_ctx* cx) {
    const int64_t threads = cx->n * cx->NC;
    if (threads == 0) return hipSuccess;
    dim3 block(256), grid((unsigned)((threads + 255) / 256));
    switch (cx->NC) {
        case 1: hipLaunchKernelGGL(k_canonical<1>, grid, block, 0, cx->stream, cx->ws.st, cx->ws.pid, cx->n, cx->dims.n_particles, cx->ws.st2); break;
        case 8: hipLaunchKernelGGL(k_canonical<8>, grid, block, 0, cx->stream, cx->ws.st, cx->ws.pid, cx->n, cx->dims.n_particles, cx->ws.st2); break;
        default: hipLaunchKernelGGL(k_canonical<16>, grid, block, 0, cx->stream, cx->ws.st, cx->ws.pid, cx->n, cx->dims.n_particles, cx->ws.st2); break;
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
