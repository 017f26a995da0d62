// The paper's own PIC instance (Sec. 4): a 2D beam in a rectangular
// perfectly conducting pipe with the sine-series Poisson solver, every
// quantity a dual number. The C ABI is declared in include/dpic2d.h.
//
// Lanes: NC consecutive lanes per particle (or grid node), lane c holding
// the value and channel c of every dual (the LD rules of common.hpp).
// Solve: the sine projection and its inverse, four passes over the interior
// nodes:
//   T = Sx rho, C = (4/(nx ny)) T Sy / (eps0 (alpha_l^2 + beta_m^2)),
//   U = Sx C,   phi = U Sy,
// with S the (symmetric) sine matrices. On power-of-two grids each pass is
// the O(n log n) sine transform (an FFT of the odd extension, as the
// spectral solver of Sec. 4 has it); otherwise a dense product with S.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/dpic2d.h"
#include "common.hpp"

namespace dpic2d {

using dpic::LD;
using dpic::ldc;
using dpic::ldchan;
using dpic::ldload;
using dpic::Map2;

constexpr int EC2_TAU = 0, EC2_AX = 1, EC2_AY = 5, EC2_N = 9;
constexpr int THREADS = 256;
constexpr int MOM2_BLOCKS = 256;
constexpr double EPS0 = 8.8541878128e-12;

struct Elem2 {
    int kind[DPIC_MAX_ELEMENTS];
    int nsteps[DPIC_MAX_ELEMENTS];
};

template <int NC>
__global__ void k2_elem(Elem2 tab, int n_elem, const double* __restrict__ elem_in, double* __restrict__ ec) {
    const int e = blockIdx.x, c = threadIdx.x;
    if (e >= n_elem || c >= NC) return;
    const LD L = ldload(elem_in + (e * 2 + 0) * NC, c);
    const LD k = ldload(elem_in + (e * 2 + 1) * NC, c);
    const double ns = (double)tab.nsteps[e];
    const LD tau = LD{L.v / ns, L.t / ns};
    const LD s = tau * 0.5;
    Map2 ax, ay;
    if (tab.kind[e] == 1) {
        ax = dpic::plane_map(k, s);
        ay = dpic::plane_map(-k, s);
    } else {
        ax = Map2{ldc(1.0), s, ldc(0.0), ldc(1.0)};
        ay = ax;
    }
    double* o = ec + (size_t)e * EC2_N * NC + c;
    o[EC2_TAU * NC] = ldchan(tau, c);
    const LD m[8] = {ax.a, ax.b, ax.c, ax.d, ay.a, ay.b, ay.c, ay.d};
#pragma unroll
    for (int i = 0; i < 8; ++i) o[(EC2_AX + i) * NC] = ldchan(m[i], c);
}

struct Sig4 {
    double s[4][16];
};

template <int NC>
__global__ void k2_init(const double* __restrict__ xi, int64_t n, int64_t cap, Sig4 sg, double* __restrict__ st) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= n) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) st[((int64_t)j * cap + p) * NC + c] = sg.s[j][c] * xi[p * 4 + j];
}

enum { F2_KICK = 1, F2_MAP = 2, F2_DEPOSIT = 4 };

struct Push2 {
    double* st;
    int64_t n, cap;
    const double* map;  // element constants of the current element (EC2_N duals)
    const double* E;    // [nx+1][ny+1][2][NC]
    double* rho;        // [nx+1][ny+1][NC]
    unsigned long long* lost;
    int nx, ny;
    double a, b, ihx, ihy, kap, qd;  // qd: charge per length per macroparticle / (hx hy)
};

struct Cell2 {
    int ix, iy;
    double sx, sy;
    bool inside;
};

__device__ __forceinline__ Cell2 cell2(double x, double y, const Push2& a) {
    Cell2 r;
    r.sx = (x + 0.5 * a.a) * a.ihx;
    r.sy = (y + 0.5 * a.b) * a.ihy;
    r.inside = r.sx >= 0.0 && r.sx < (double)a.nx && r.sy >= 0.0 && r.sy < (double)a.ny;
    r.ix = (int)floor(r.sx);
    r.iy = (int)floor(r.sy);
    return r;
}

template <int NC, int F>
__global__ __launch_bounds__(THREADS) void k2_push(Push2 a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid / NC;
    const int c = (int)(gid % NC);
    if (p >= a.n) return;
    const int64_t cs = a.cap * NC;
    double* sp = a.st + p * NC;
    LD x = ldload(sp, c), px = ldload(sp + cs, c), y = ldload(sp + 2 * cs, c), py = ldload(sp + 3 * cs, c);
    const int ly = a.ny + 1;
    if (F & F2_KICK) {
        const Cell2 g = cell2(x.v, y.v, a);
        if (g.inside) {
            const LD fx = LD{g.sx - g.ix, x.t * a.ihx}, fy = LD{g.sy - g.iy, y.t * a.ihy};
            LD ex = ldc(0.0), ey = ldc(0.0);
#pragma unroll
            for (int kx = 0; kx < 2; ++kx)
#pragma unroll
                for (int ky = 0; ky < 2; ++ky) {
                    const LD w = (kx ? fx : 1.0 - fx) * (ky ? fy : 1.0 - fy);
                    const double* e = a.E + ((int64_t)(g.ix + kx) * ly + g.iy + ky) * 2 * NC;
                    ex = dpic::fmad(w, ldload(e, c), ex);
                    ey = dpic::fmad(w, ldload(e + NC, c), ey);
                }
            const LD tau = ldload(a.map + EC2_TAU * NC, c);
            px = px + tau * (ex * a.kap);
            py = py + tau * (ey * a.kap);
        }
    }
    if (F & F2_MAP) {
        const double* m = a.map;
        const LD xa = ldload(m + (EC2_AX + 0) * NC, c), xb = ldload(m + (EC2_AX + 1) * NC, c);
        const LD xc = ldload(m + (EC2_AX + 2) * NC, c), xd = ldload(m + (EC2_AX + 3) * NC, c);
        const LD ya = ldload(m + (EC2_AY + 0) * NC, c), yb = ldload(m + (EC2_AY + 1) * NC, c);
        const LD yc = ldload(m + (EC2_AY + 2) * NC, c), yd = ldload(m + (EC2_AY + 3) * NC, c);
        const LD nx = xa * x + xb * px, npx = xc * x + xd * px;
        const LD ny = ya * y + yb * py, npy = yc * y + yd * py;
        x = nx;
        px = npx;
        y = ny;
        py = npy;
    }
    if (F & F2_DEPOSIT) {
        const Cell2 g = cell2(x.v, y.v, a);
        if (g.inside) {
            const LD fx = LD{g.sx - g.ix, x.t * a.ihx}, fy = LD{g.sy - g.iy, y.t * a.ihy};
#pragma unroll
            for (int kx = 0; kx < 2; ++kx)
#pragma unroll
                for (int ky = 0; ky < 2; ++ky) {
                    const LD w = (kx ? fx : 1.0 - fx) * (ky ? fy : 1.0 - fy);
                    unsafeAtomicAdd(a.rho + ((int64_t)(g.ix + kx) * ly + g.iy + ky) * NC + c, ldchan(w * a.qd, c));
                }
        } else if (c == 0) {
            atomicAdd(a.lost, 1ull);
        }
    }
    sp[0 * cs + c] = ldchan(x, c);
    sp[1 * cs + c] = ldchan(px, c);
    sp[2 * cs + c] = ldchan(y, c);
    sp[3 * cs + c] = ldchan(py, c);
}

// sine tables S[l][i] = sin(pi (l+1)(i+1)/n) (interior indices), and
// ginv[l][m] = 4 / (nx ny eps0 (alpha_l^2 + beta_m^2))
__global__ void k2_tables(double* __restrict__ Sx, double* __restrict__ Sy, double* __restrict__ ginv, int nx, int ny,
                          double a, double b) {
    const int nx1 = nx - 1, ny1 = ny - 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nx1 * nx1) {
        const int l = i / nx1, q = i % nx1;
        Sx[i] = sinpi((double)((l + 1) * (q + 1)) / (double)nx);
    }
    if (i < ny1 * ny1) {
        const int l = i / ny1, q = i % ny1;
        Sy[i] = sinpi((double)((l + 1) * (q + 1)) / (double)ny);
    }
    if (i < nx1 * ny1) {
        const int l = i / ny1, m = i % ny1;
        const double al = (l + 1) * M_PI / a, be = (m + 1) * M_PI / b;
        ginv[i] = 4.0 / ((double)nx * (double)ny * EPS0 * (al * al + be * be));
    }
}

// One dense pass over [rows][cols][NC] arrays with leading dimension ld and
// an origin offset (off, off) inside them.
//   DIM 0: out[r][q] = sum_k S[r][k] in[k][q]
//   DIM 1: out[r][q] = scale[r][q] sum_k in[r][k] S[q][k]   (scale optional)
template <int NC, int DIM>
__global__ void k2_pass(const double* __restrict__ in, int in_ld, int in_off, const double* __restrict__ S, int nk,
                        double* __restrict__ out, int out_ld, int out_off, int rows, int cols,
                        const double* __restrict__ scale) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(gid % NC);
    const int64_t e = gid / NC;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), q = (int)(e % cols);
    double acc = 0.0;
    if (DIM == 0) {
        for (int k = 0; k < nk; ++k)
            acc = fma(S[(int64_t)r * nk + k], in[((int64_t)(k + in_off) * in_ld + q + in_off) * NC + c], acc);
    } else {
        for (int k = 0; k < nk; ++k)
            acc = fma(in[((int64_t)(r + in_off) * in_ld + k + in_off) * NC + c], S[(int64_t)q * nk + k], acc);
        if (scale) acc *= scale[(int64_t)r * cols + q];
    }
    out[((int64_t)(r + out_off) * out_ld + q + out_off) * NC + c] = acc;
}

// Type-I discrete sine transform along one axis, O(n log n): the line
// z_i (i = 1..n-1; z_0 = z_n = 0) is extended to the odd sequence of length
// M = 2n (y_t = z_t, y_{M-t} = -z_t), whose M-point FFT is
// Y_l = -2i sum_i z_i sin(pi l i / n); so X_l = sum_i z_i sin(pi l i / n) =
// i Y_l / 2 for l = 1..n-1. The real channels c and c + NC/2 travel as one
// complex line (the transform is real-linear), so one FFT gives both. One
// workgroup of n threads per (line, channel pair); radix-2 in LDS, n a
// power of two. Element (line, i) sits at
// ((line * ls + i * es + off) * NC + channel) on either side; the output is
// multiplied by scale[line * sls + (l - 1)] when scale is given.
struct DstArgs {
    const double* in;
    int64_t in_ls, in_es, in_off;
    double* out;
    int64_t out_ls, out_es, out_off;
    const double* scale;
    int64_t sls;
    int n, log2m;
};

template <int NC>
__global__ void k2_dst(DstArgs a) {
    constexpr int NCH = NC == 1 ? 1 : NC / 2;  // complex channels
    __shared__ double yr[512], yi[512];
    const int M = 2 * a.n;
    const int64_t line = blockIdx.x / NCH;
    const int c = (int)(blockIdx.x % NCH);
    // odd extension, stored at bit-reversed positions
    for (int t = threadIdx.x; t < M; t += blockDim.x) {
        double vr = 0.0, vi = 0.0;
        const int i = t < a.n ? t : M - t;  // 1..n-1 for the nonzero entries
        if (i != 0 && t != a.n) {
            const int64_t e = (line * a.in_ls + i * a.in_es + a.in_off) * NC;
            vr = a.in[e + c];
            if (NC > 1) vi = a.in[e + c + NCH];
            if (t > a.n) {
                vr = -vr;
                vi = -vi;
            }
        }
        const int rt = (int)(__brev((unsigned)t) >> (32 - a.log2m));
        yr[rt] = vr;
        yi[rt] = vi;
    }
    __syncthreads();
    for (int len = 2; len <= M; len <<= 1) {
        const int half = len >> 1;
        for (int k = threadIdx.x; k < M / 2; k += blockDim.x) {
            const int j = k % half, base = (k / half) * len;
            double sn, cs;
            sincospi(-2.0 * (double)j / (double)len, &sn, &cs);
            const double ur = yr[base + j], ui = yi[base + j];
            const double xr = yr[base + j + half], xi = yi[base + j + half];
            const double tr = xr * cs - xi * sn, ti = xr * sn + xi * cs;
            yr[base + j] = ur + tr;
            yi[base + j] = ui + ti;
            yr[base + j + half] = ur - tr;
            yi[base + j + half] = ui - ti;
        }
        __syncthreads();
    }
    for (int l = 1 + threadIdx.x; l < a.n; l += blockDim.x) {
        double xr = -0.5 * yi[l], xi = 0.5 * yr[l];  // X = i Y / 2
        if (a.scale) {
            const double s = a.scale[line * a.sls + (l - 1)];
            xr *= s;
            xi *= s;
        }
        const int64_t e = (line * a.out_ls + l * a.out_es + a.out_off) * NC;
        a.out[e + c] = xr;
        if (NC > 1) a.out[e + c + NCH] = xi;
    }
}

template <int NC>
__global__ void k2_field(const double* __restrict__ phi, double* __restrict__ E, int nx, int ny, double fx, double fy) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(gid % NC);
    const int64_t node = gid / NC;
    const int ly = ny + 1;
    if (node >= (int64_t)(nx + 1) * ly) return;
    const int i = (int)(node / ly), j = (int)(node % ly);
    auto P = [&](int ii, int jj) -> double {  // odd continuation beyond the walls
        double sg = 1.0;
        if (ii < 0) { ii = -ii; sg = -sg; }
        if (ii > nx) { ii = 2 * nx - ii; sg = -sg; }
        if (jj < 0) { jj = -jj; sg = -sg; }
        if (jj > ny) { jj = 2 * ny - jj; sg = -sg; }
        return sg * phi[((int64_t)ii * ly + jj) * NC + c];
    };
    E[(node * 2 + 0) * NC + c] = fx * (P(i + 1, j) - P(i - 1, j));
    E[(node * 2 + 1) * NC + c] = fy * (P(i, j + 1) - P(i, j - 1));
}

template <int NC>
__global__ __launch_bounds__(THREADS) void k2_mom_partial(const double* __restrict__ st, int64_t n, int64_t cap,
                                                          double* __restrict__ part) {
    constexpr int PPB = THREADS / NC;
    const int c = threadIdx.x % NC;
    const int64_t cs = cap * NC;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * PPB + threadIdx.x / NC; p < n; p += (int64_t)gridDim.x * PPB) {
        const double* sp = st + p * NC;
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
            const LD u = ldload(sp + (2 * pl) * cs, c), q = ldload(sp + (2 * pl + 1) * cs, c);
            acc[pl * 3 + 0] += ldchan(u * u, c);
            acc[pl * 3 + 1] += ldchan(u * q, c);
            acc[pl * 3 + 2] += ldchan(q * q, c);
        }
    }
    __shared__ double red[THREADS][6];
#pragma unroll
    for (int m = 0; m < 6; ++m) red[threadIdx.x][m] = acc[m];
    __syncthreads();
    if ((int)threadIdx.x < NC) {
        for (int m = 0; m < 6; ++m) {
            double s = 0.0;
            for (int t = threadIdx.x; t < THREADS; t += NC) s += red[t][m];
            part[((size_t)blockIdx.x * 6 + m) * NC + threadIdx.x] = s;
        }
    }
}

template <int NC>
__global__ void k2_mom_final(const double* __restrict__ part, int nblocks, double inv_n, double* __restrict__ emit) {
    __shared__ double sm[6 * NC];
    for (int i = threadIdx.x; i < 6 * NC; i += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * 6 * NC + i];
        sm[i] = s * inv_n;
    }
    __syncthreads();
    const int c = threadIdx.x;
    if (c >= NC) return;
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
        const LD uu = ldload(sm + (pl * 3 + 0) * NC, c), up = ldload(sm + (pl * 3 + 1) * NC, c);
        const LD pp = ldload(sm + (pl * 3 + 2) * NC, c);
        emit[pl * NC + c] = ldchan(dpic::dsqrt(uu * pp - up * up), c);
    }
}

__global__ void k2_zero(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace dpic2d

// ---------------------------------------------------------------- context
struct dpic2d_ctx {
    dpic2d_dims dims{};
    int NC = 1, ntan = 0, nx = 0, ny = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // workspace
    double *st = nullptr, *rho = nullptr, *phi = nullptr, *E = nullptr, *T = nullptr, *U = nullptr;
    double *Sx = nullptr, *Sy = nullptr, *ginv = nullptr, *ec = nullptr, *elem_in = nullptr;
    unsigned long long* lost = nullptr;
    double *part = nullptr, *emit = nullptr;
    // state
    bool beam_set = false, pipe_set = false, lattice_set = false, params_set = false, beam_init = false;
    double gamma0 = 1, beta0 = 0, kap = 0, current = 0, a = 0, b = 0;
    int n_elem = 0, n_periods = 1;
    std::vector<int> kind, n_steps, L_param, k_param, schedule;
    std::vector<double> L, k, p, seed;
    int64_t n = 0, steps_done = 0;
};

namespace {

using namespace dpic2d;

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int fail(dpic2d_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail((c), DPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int check(const dpic2d_dims* d) {
    if (!d || d->flags != 0) return DPIC_EINVAL;
    if (d->n_particles < 1 || d->n_particles > (int64_t)0x7fffffff) return DPIC_EINVAL;
    if (d->ntan < 0 || d->ntan > 15) return DPIC_EUNSUPPORTED;
    if (d->nx < 4 || d->nx > 256 || d->ny < 4 || d->ny > 256) return DPIC_EUNSUPPORTED;
    return DPIC_OK;
}

size_t layout(const dpic2d_dims& d, char* base, dpic2d_ctx* c) {
    const size_t NC = (size_t)dpic::channels_for(d.ntan);
    const size_t cap = (size_t)d.n_particles;
    const size_t nodes = (size_t)(d.nx + 1) * (d.ny + 1);
    const size_t inner = (size_t)(d.nx - 1) * (d.ny - 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return base ? (void*)(base + o) : nullptr;
    };
    dpic2d_ctx t;
    t.st = (double*)take(4 * cap * NC * 8);
    t.rho = (double*)take(nodes * NC * 8);
    t.phi = (double*)take(nodes * NC * 8);
    t.E = (double*)take(nodes * 2 * NC * 8);
    t.T = (double*)take(inner * NC * 8);
    t.U = (double*)take(inner * NC * 8);
    t.Sx = (double*)take((size_t)(d.nx - 1) * (d.nx - 1) * 8);
    t.Sy = (double*)take((size_t)(d.ny - 1) * (d.ny - 1) * 8);
    t.ginv = (double*)take(inner * 8);
    t.ec = (double*)take((size_t)DPIC_MAX_ELEMENTS * EC2_N * NC * 8);
    t.elem_in = (double*)take((size_t)DPIC_MAX_ELEMENTS * 2 * NC * 8);
    t.lost = (unsigned long long*)take(8);
    t.part = (double*)take((size_t)MOM2_BLOCKS * 6 * NC * 8);
    t.emit = (double*)take(2 * NC * 8);
    if (c) {
        c->st = t.st; c->rho = t.rho; c->phi = t.phi; c->E = t.E; c->T = t.T; c->U = t.U;
        c->Sx = t.Sx; c->Sy = t.Sy; c->ginv = t.ginv; c->ec = t.ec; c->elem_in = t.elem_in;
        c->lost = t.lost; c->part = t.part; c->emit = t.emit;
    }
    return off;
}

hipError_t zero(dpic2d_ctx* c, double* p, int64_t n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k2_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n);
    return hipGetLastError();
}

#define NC_SWITCH(c, CALL)                  \
    switch ((c)->NC) {                      \
        case 1: { constexpr int NC = 1; CALL; } break;  \
        case 8: { constexpr int NC = 8; CALL; } break;  \
        default: { constexpr int NC = 16; CALL; } break; \
    }

int refresh(dpic2d_ctx* c) {
    if (!c->beam_set || !c->lattice_set) return DPIC_OK;
    for (int e = 0; e < c->n_elem; ++e)
        if ((c->L_param[e] >= 0 || c->k_param[e] >= 0) && !c->params_set) return DPIC_OK;
    const int NCc = c->NC, nt = c->ntan;
    const int np = (int)c->p.size();
    std::vector<double> in((size_t)DPIC_MAX_ELEMENTS * 2 * NCc, 0.0);
    for (int e = 0; e < c->n_elem; ++e) {
        double* Ld = &in[(size_t)(e * 2) * NCc];
        double* kd = &in[(size_t)(e * 2 + 1) * NCc];
        const int lp = c->L_param[e], kp = c->k_param[e];
        if (lp >= np || kp >= np) return fail(c, DPIC_EINVAL, "element %d binds a parameter beyond %d", e, np);
        Ld[0] = lp >= 0 ? c->p[lp] : c->L[e];
        if (lp >= 0)
            for (int t = 0; t < nt; ++t) Ld[1 + t] = c->seed[(size_t)lp * nt + t];
        if (c->kind[e] == 1) {
            kd[0] = kp >= 0 ? c->p[kp] : c->k[e];
            if (kp >= 0)
                for (int t = 0; t < nt; ++t) kd[1 + t] = c->seed[(size_t)kp * nt + t];
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->elem_in, in.data(), in.size() * 8, hipMemcpyHostToDevice, c->stream));
    Elem2 tab{};
    for (int e = 0; e < c->n_elem; ++e) {
        tab.kind[e] = c->kind[e];
        tab.nsteps[e] = c->n_steps[e];
    }
    NC_SWITCH(c, hipLaunchKernelGGL((k2_elem<NC>), dim3(c->n_elem), dim3(64), 0, c->stream, tab, c->n_elem, c->elem_in, c->ec));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

bool ready(const dpic2d_ctx* c) {
    if (!c->beam_set || !c->lattice_set || !c->pipe_set || !c->beam_init) return false;
    for (int e = 0; e < c->n_elem; ++e)
        if ((c->L_param[e] >= 0 || c->k_param[e] >= 0) && !c->params_set) return false;
    return true;
}

Push2 push_args(dpic2d_ctx* c, int e) {
    Push2 a;
    a.st = c->st;
    a.n = c->n;
    a.cap = c->dims.n_particles;
    a.map = c->ec + (size_t)e * EC2_N * c->NC;
    a.E = c->E;
    a.rho = c->rho;
    a.lost = c->lost;
    a.nx = c->nx;
    a.ny = c->ny;
    a.a = c->a;
    a.b = c->b;
    a.ihx = c->nx / c->a;
    a.ihy = c->ny / c->b;
    a.kap = c->kap;
    const double hx = c->a / c->nx, hy = c->b / c->ny;
    a.qd = c->n > 0 ? c->current / (c->beta0 * 299792458.0) / (double)c->n / (hx * hy) : 0.0;
    return a;
}

hipError_t push(dpic2d_ctx* c, int flags, int e) {
    if (c->n == 0) return hipSuccess;
    const Push2 a = push_args(c, e);
    const int64_t threads = c->n * c->NC;
    const dim3 grid((unsigned)((threads + THREADS - 1) / THREADS)), block(THREADS);
    switch (flags) {
        case F2_MAP | F2_DEPOSIT: NC_SWITCH(c, hipLaunchKernelGGL((k2_push<NC, F2_MAP | F2_DEPOSIT>), grid, block, 0, c->stream, a)); break;
        case F2_KICK | F2_MAP: NC_SWITCH(c, hipLaunchKernelGGL((k2_push<NC, F2_KICK | F2_MAP>), grid, block, 0, c->stream, a)); break;
        case F2_MAP: NC_SWITCH(c, hipLaunchKernelGGL((k2_push<NC, F2_MAP>), grid, block, 0, c->stream, a)); break;
        case F2_DEPOSIT: NC_SWITCH(c, hipLaunchKernelGGL((k2_push<NC, F2_DEPOSIT>), grid, block, 0, c->stream, a)); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2i(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

// One sine-transform pass over nlines lines of interior length n - 1.
hipError_t dst_pass(dpic2d_ctx* c, int n, int64_t nlines, const double* in, int64_t in_ls, int64_t in_es,
                    int64_t in_off, double* out, int64_t out_ls, int64_t out_es, int64_t out_off, const double* scale,
                    int64_t sls) {
    DstArgs a{in, in_ls, in_es, in_off, out, out_ls, out_es, out_off, scale, sls, n, ilog2i(2 * n)};
    const int nch = c->NC == 1 ? 1 : c->NC / 2;
    const dim3 grid((unsigned)(nlines * nch)), block((unsigned)std::min(n, 256));
    NC_SWITCH(c, hipLaunchKernelGGL((k2_dst<NC>), grid, block, 0, c->stream, a));
    return hipGetLastError();
}

hipError_t solve(dpic2d_ctx* c) {
    const int nx1 = c->nx - 1, ny1 = c->ny - 1, ly = c->ny + 1;
    if (pow2(c->nx) && pow2(c->ny)) {
        // rho[i][j] (nodes, i = x) -> T[l][q]: sine transform along x of the
        // interior rows q (node j = q + 1); T -> U[l][m] along y, scaled by
        // ginv; U -> T along x; T -> phi (interior nodes) along y
        hipError_t e;
        if ((e = dst_pass(c, c->nx, ny1, c->rho, 1, ly, 1, c->T, 1, ny1, -ny1, nullptr, 0)) != hipSuccess) return e;
        if ((e = dst_pass(c, c->ny, nx1, c->T, ny1, 1, -1, c->U, ny1, 1, -1, c->ginv, ny1)) != hipSuccess) return e;
        if ((e = dst_pass(c, c->nx, ny1, c->U, 1, ny1, -ny1, c->T, 1, ny1, -ny1, nullptr, 0)) != hipSuccess) return e;
        return dst_pass(c, c->ny, nx1, c->T, ny1, 1, -1, c->phi, ly, 1, ly, nullptr, 0);
    }
    const int64_t inner = (int64_t)nx1 * ny1 * c->NC;
    const dim3 grid((unsigned)((inner + 255) / 256)), block(256);
    NC_SWITCH(c, {
        // T = Sx rho (interior), C = scale * T Sy, U = Sx C, phi = U Sy
        hipLaunchKernelGGL((k2_pass<NC, 0>), grid, block, 0, c->stream, c->rho, ly, 1, c->Sx, nx1, c->T, ny1, 0, nx1, ny1, nullptr);
        hipLaunchKernelGGL((k2_pass<NC, 1>), grid, block, 0, c->stream, c->T, ny1, 0, c->Sy, ny1, c->U, ny1, 0, nx1, ny1, c->ginv);
        hipLaunchKernelGGL((k2_pass<NC, 0>), grid, block, 0, c->stream, c->U, ny1, 0, c->Sx, nx1, c->T, ny1, 0, nx1, ny1, nullptr);
        hipLaunchKernelGGL((k2_pass<NC, 1>), grid, block, 0, c->stream, c->T, ny1, 0, c->Sy, ny1, c->phi, ly, 1, nx1, ny1, nullptr);
    });
    return hipGetLastError();
}

hipError_t field(dpic2d_ctx* c) {
    const int64_t n = (int64_t)(c->nx + 1) * (c->ny + 1) * c->NC;
    const double fx = -0.5 * c->nx / c->a, fy = -0.5 * c->ny / c->b;
    NC_SWITCH(c, hipLaunchKernelGGL((k2_field<NC>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->phi,
                                    c->E, c->nx, c->ny, fx, fy));
    return hipGetLastError();
}

size_t nodes(const dpic2d_ctx* c) { return (size_t)(c->nx + 1) * (c->ny + 1); }

}  // namespace

extern "C" {

int dpic2d_query_workspace(const dpic2d_dims* d, size_t* bytes) {
    int r = check(d);
    if (r != DPIC_OK) return r;
    if (!bytes) return DPIC_EINVAL;
    *bytes = layout(*d, nullptr, nullptr);
    return DPIC_OK;
}

int dpic2d_create(const dpic2d_dims* d, void* ws, size_t bytes, void* stream, dpic2d_ctx** out) {
    int r = check(d);
    if (r != DPIC_OK) return r;
    if (!ws || !out || (uintptr_t)ws % ALIGN || bytes < layout(*d, nullptr, nullptr)) return DPIC_EINVAL;
    dpic2d_ctx* c = new (std::nothrow) dpic2d_ctx();
    if (!c) return DPIC_EINVAL;
    c->dims = *d;
    c->ntan = d->ntan;
    c->NC = dpic::channels_for(d->ntan);
    c->nx = d->nx;
    c->ny = d->ny;
    c->stream = (hipStream_t)stream;
    layout(*d, (char*)ws, c);
    *out = c;
    return DPIC_OK;
}

int dpic2d_destroy(dpic2d_ctx* c) {
    if (!c) return DPIC_EINVAL;
    delete c;
    return DPIC_OK;
}

int dpic2d_last_error(const dpic2d_ctx* c, char* buf, size_t len) {
    if (!c || !buf || !len) return DPIC_EINVAL;
    snprintf(buf, len, "%s", c->err.c_str());
    return DPIC_OK;
}

int dpic2d_set_beam(dpic2d_ctx* c, double kinetic_eV, double rest_eV, double charge_e, double current_A) {
    if (!c) return DPIC_EINVAL;
    if (!(kinetic_eV > 0) || !(rest_eV > 0) || !isfinite(charge_e) || !isfinite(current_A) || !isfinite(kinetic_eV) ||
        !isfinite(rest_eV))
        return fail(c, DPIC_EINVAL, "beam: energies must be positive and all values finite");
    c->gamma0 = 1.0 + kinetic_eV / rest_eV;
    c->beta0 = sqrt(1.0 - 1.0 / (c->gamma0 * c->gamma0));
    c->kap = (charge_e / rest_eV) / (c->beta0 * c->beta0 * c->gamma0 * c->gamma0 * c->gamma0);
    c->current = current_A;
    c->beam_set = true;
    return refresh(c);
}

int dpic2d_set_pipe(dpic2d_ctx* c, double a, double b) {
    if (!c) return DPIC_EINVAL;
    if (!(a > 0) || !(b > 0) || !isfinite(a) || !isfinite(b)) return fail(c, DPIC_EINVAL, "pipe: widths must be > 0");
    c->a = a;
    c->b = b;
    const int m = std::max(std::max((c->nx - 1) * (c->nx - 1), (c->ny - 1) * (c->ny - 1)), (c->nx - 1) * (c->ny - 1));
    hipLaunchKernelGGL(k2_tables, dim3((m + 255) / 256), dim3(256), 0, c->stream, c->Sx, c->Sy, c->ginv, c->nx, c->ny, a, b);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, zero(c, c->phi, (int64_t)nodes(c) * c->NC));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pipe_set = true;
    return DPIC_OK;
}

int dpic2d_set_lattice(dpic2d_ctx* c, int n_elem, const int* kind, const int* n_steps, const double* L, const double* k,
                       const int* L_param, const int* k_param, int n_periods) {
    if (!c) return DPIC_EINVAL;
    if (n_elem < 1 || n_elem > DPIC_MAX_ELEMENTS || !kind || !n_steps || n_periods < 1)
        return fail(c, DPIC_EINVAL, "lattice: need 1..%d elements and n_periods >= 1", DPIC_MAX_ELEMENTS);
    int64_t total = 0;
    for (int e = 0; e < n_elem; ++e) {
        const int lp = L_param ? L_param[e] : -1, kp = k_param ? k_param[e] : -1;
        if ((kind[e] != 0 && kind[e] != 1) || n_steps[e] < 1 || lp < -1 || lp >= DPIC_MAX_PARAMS || kp < -1 ||
            kp >= DPIC_MAX_PARAMS || (lp < 0 && (!L || !isfinite(L[e]))) || (kind[e] == 1 && kp < 0 && (!k || !isfinite(k[e]))))
            return fail(c, DPIC_EINVAL, "lattice: bad element %d", e);
        total += n_steps[e];
    }
    if (total * n_periods > 100000000) return fail(c, DPIC_EINVAL, "lattice: schedule too long");
    c->n_elem = n_elem;
    c->n_periods = n_periods;
    c->kind.assign(kind, kind + n_elem);
    c->n_steps.assign(n_steps, n_steps + n_elem);
    c->L.assign(n_elem, 0.0);
    c->k.assign(n_elem, 0.0);
    c->L_param.assign(n_elem, -1);
    c->k_param.assign(n_elem, -1);
    for (int e = 0; e < n_elem; ++e) {
        if (L) c->L[e] = L[e];
        if (k) c->k[e] = k[e];
        if (L_param) c->L_param[e] = L_param[e];
        if (k_param) c->k_param[e] = k_param[e];
    }
    c->schedule.clear();
    for (int pr = 0; pr < n_periods; ++pr)
        for (int e = 0; e < n_elem; ++e)
            for (int s = 0; s < n_steps[e]; ++s) c->schedule.push_back(e);
    c->lattice_set = true;
    return refresh(c);
}

int dpic2d_set_params(dpic2d_ctx* c, int np, const double* p, const double* seed) {
    if (!c) return DPIC_EINVAL;
    if (np < 0 || np > DPIC_MAX_PARAMS || (np > 0 && !p)) return fail(c, DPIC_EINVAL, "params: 0..%d values", DPIC_MAX_PARAMS);
    const int nt = c->ntan;
    c->p.assign(p, p + np);
    c->seed.assign((size_t)np * nt, 0.0);
    for (int j = 0; j < np; ++j) {
        if (!isfinite(p[j])) return fail(c, DPIC_EINVAL, "params: p[%d] not finite", j);
        for (int t = 0; t < nt; ++t) c->seed[(size_t)j * nt + t] = seed ? seed[(size_t)j * nt + t] : (j == t ? 1.0 : 0.0);
    }
    c->params_set = true;
    return refresh(c);
}

int dpic2d_init_beam(dpic2d_ctx* c, int64_t n, const double* xi, const double sigma[4], const double* sigma_seed) {
    if (!c || !sigma) return DPIC_EINVAL;
    if (n < 0 || n > c->dims.n_particles) return fail(c, DPIC_EINVAL, "init_beam: n outside 0..capacity");
    if (n > 0 && !xi) return fail(c, DPIC_EINVAL, "init_beam: xi is NULL");
    Sig4 sg{};
    for (int j = 0; j < 4; ++j) {
        if (!isfinite(sigma[j])) return fail(c, DPIC_EINVAL, "init_beam: sigma[%d] not finite", j);
        sg.s[j][0] = sigma[j];
        if (sigma_seed)
            for (int t = 0; t < c->ntan; ++t) sg.s[j][1 + t] = sigma_seed[(size_t)j * c->ntan + t];
    }
    c->n = n;
    if (n > 0) {
        const int64_t threads = n * c->NC;
        NC_SWITCH(c, hipLaunchKernelGGL((k2_init<NC>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, c->stream,
                                        xi, n, c->dims.n_particles, sg, c->st));
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, zero(c, (double*)c->lost, 1));
    c->steps_done = 0;
    c->beam_init = true;
    return DPIC_OK;
}

int dpic2d_step(dpic2d_ctx* c, int n) {
    if (!c) return DPIC_EINVAL;
    if (n < 0) return fail(c, DPIC_EINVAL, "step: n < 0");
    if (!ready(c)) return fail(c, DPIC_ESTATE, "step: beam, pipe, lattice, parameters and initial beam must be set");
    if (c->steps_done + n > (int64_t)c->schedule.size()) return fail(c, DPIC_EINVAL, "step: past the end of the schedule");
    const bool sc = c->current != 0.0;
    for (int64_t s = c->steps_done; s < c->steps_done + n; ++s) {
        const int e = c->schedule[s];
        if (sc) {
            HIPCHK(c, zero(c, c->rho, (int64_t)nodes(c) * c->NC));
            HIPCHK(c, push(c, F2_MAP | F2_DEPOSIT, e));
            HIPCHK(c, solve(c));
            HIPCHK(c, field(c));
            HIPCHK(c, push(c, F2_KICK | F2_MAP, e));
        } else {
            HIPCHK(c, push(c, F2_MAP | F2_DEPOSIT, e));  // deposit only counts: no space charge is used
            HIPCHK(c, push(c, F2_MAP, e));
        }
    }
    c->steps_done += n;
    return DPIC_OK;
}

int dpic2d_read_emittance(dpic2d_ctx* c, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    if (!c->beam_init || c->n == 0) return fail(c, DPIC_ESTATE, "read_emittance: no beam");
    const int64_t want = (c->n * c->NC + THREADS - 1) / THREADS;
    const int nb = (int)std::min<int64_t>(std::max<int64_t>(want, 1), MOM2_BLOCKS);
    NC_SWITCH(c, {
        hipLaunchKernelGGL((k2_mom_partial<NC>), dim3(nb), dim3(THREADS), 0, c->stream, c->st, c->n, c->dims.n_particles, c->part);
        hipLaunchKernelGGL((k2_mom_final<NC>), dim3(1), dim3(64), 0, c->stream, c->part, nb, 1.0 / (double)c->n, c->emit);
    });
    HIPCHK(c, hipGetLastError());
    std::vector<double> h((size_t)2 * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->emit, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int pl = 0; pl < 2; ++pl)
        for (int ch = 0; ch <= c->ntan; ++ch) out[pl * (c->ntan + 1) + ch] = h[(size_t)pl * c->NC + ch];
    return DPIC_OK;
}

int dpic2d_read_particles(dpic2d_ctx* c, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "read_particles: no beam");
    const size_t cap = (size_t)c->dims.n_particles, NCc = c->NC;
    std::vector<double> h(4 * cap * NCc);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->st, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t p = 0; p < c->n; ++p)
        for (int j = 0; j < 4; ++j)
            for (int ch = 0; ch <= c->ntan; ++ch) out[((size_t)p * 4 + j) * (c->ntan + 1) + ch] = h[((size_t)j * cap + p) * NCc + ch];
    return DPIC_OK;
}

int dpic2d_stage(dpic2d_ctx* c, int stage) {
    if (!c) return DPIC_EINVAL;
    if (!c->pipe_set || !c->beam_set) return fail(c, DPIC_ESTATE, "stage: beam and pipe must be set");
    switch (stage) {
        case 0:
            if (!c->beam_init) return fail(c, DPIC_ESTATE, "stage deposit: no beam");
            HIPCHK(c, zero(c, c->rho, (int64_t)nodes(c) * c->NC));
            HIPCHK(c, push(c, F2_DEPOSIT, 0));
            return DPIC_OK;
        case 1: HIPCHK(c, solve(c)); return DPIC_OK;
        case 2: HIPCHK(c, field(c)); return DPIC_OK;
        default: return fail(c, DPIC_EINVAL, "stage: unknown stage %d", stage);
    }
}

static int grid2(dpic2d_ctx* c, int which, double** dev, size_t* rows) {
    switch (which) {
        case DPIC2D_GRID_RHO: *dev = c->rho; *rows = nodes(c); return DPIC_OK;
        case DPIC2D_GRID_PHI: *dev = c->phi; *rows = nodes(c); return DPIC_OK;
        case DPIC2D_GRID_E: *dev = c->E; *rows = nodes(c) * 2; return DPIC_OK;
        default: return DPIC_EINVAL;
    }
}

int dpic2d_read_grid(dpic2d_ctx* c, int which, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    double* dev;
    size_t rows;
    if (grid2(c, which, &dev, &rows) != DPIC_OK) return fail(c, DPIC_EINVAL, "read_grid: unknown array");
    std::vector<double> h(rows * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), dev, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t r = 0; r < rows; ++r)
        for (int ch = 0; ch <= c->ntan; ++ch) out[r * (c->ntan + 1) + ch] = h[r * c->NC + ch];
    return DPIC_OK;
}

int dpic2d_write_grid(dpic2d_ctx* c, int which, const double* in) {
    if (!c || !in) return DPIC_EINVAL;
    double* dev;
    size_t rows;
    if (grid2(c, which, &dev, &rows) != DPIC_OK) return fail(c, DPIC_EINVAL, "write_grid: unknown array");
    std::vector<double> h(rows * c->NC, 0.0);
    for (size_t r = 0; r < rows; ++r)
        for (int ch = 0; ch <= c->ntan; ++ch) h[r * c->NC + ch] = in[r * (c->ntan + 1) + ch];
    HIPCHK(c, hipMemcpyAsync(dev, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

int dpic2d_counters(dpic2d_ctx* c, int64_t* lost, int64_t* steps) {
    if (!c) return DPIC_EINVAL;
    unsigned long long h = 0;
    HIPCHK(c, hipMemcpyAsync(&h, c->lost, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (lost) *lost = (int64_t)h;
    if (steps) *steps = c->steps_done;
    return DPIC_OK;
}

}  // extern "C"
