// Twiss parameters of a line and their parameter derivatives (dual numbers,
// NC = 16 lanes per parameter vector), the matching objective, and the BFGS
// driver of the matching example. C ABI: include/dtwiss.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <vector>

#include "../../include/dtwiss.h"
#include "common.hpp"

namespace dtwiss {

using dpic::LD;
using dpic::ldc;
using dpic::ldchan;
using dpic::Map2;

constexpr int NC = 16;
constexpr int MAX_NB = 65536;

struct Line {
    int n;
    int kind[DPIC_MAX_ELEMENTS];
    int lp[DPIC_MAX_ELEMENTS], kp[DPIC_MAX_ELEMENTS];
    double L[DPIC_MAX_ELEMENTS], k[DPIC_MAX_ELEMENTS];
};

struct Ends {
    double tw0[4];
    int periodic;
    double tgt[4];
    int has_target;
};

// parameter j of vector s as a dual with tangent j (lane c holds channel c)
__device__ __forceinline__ LD param(const double* p, int np, int s, int j, int c) {
    return LD{p[(int64_t)s * np + j], (c == 1 + j) ? 1.0 : 0.0};
}

__device__ void twiss_of(const Map2& m, const LD& b0, const LD& a0, LD& b1, LD& a1) {
    const LD g0 = (1.0 + a0 * a0) / b0;
    b1 = m.a * m.a * b0 - m.a * m.b * a0 * 2.0 + m.b * m.b * g0;
    a1 = -(m.a * m.c * b0) + (m.a * m.d + m.b * m.c) * a0 - m.b * m.d * g0;
}

__device__ void periodic_of(const Map2& m, LD& b, LD& a) {
    const LD cmu = (m.a + m.d) * 0.5;
    LD smu = dpic::dsqrt(1.0 - cmu * cmu);
    if (m.b.v < 0) smu = -smu;
    b = m.b / smu;
    a = (m.a - m.d) / (smu * 2.0);
}

__global__ void k_twiss(Line ln, Ends en, const double* __restrict__ p, int np, int nb, double* __restrict__ tw,
                        double* __restrict__ f) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = gid / NC, c = gid % NC;
    if (s >= nb) return;
    Map2 Mx{ldc(1.0), ldc(0.0), ldc(0.0), ldc(1.0)}, My = Mx;
    for (int e = 0; e < ln.n; ++e) {
        const LD L = ln.lp[e] >= 0 ? param(p, np, s, ln.lp[e], c) : ldc(ln.L[e]);
        Map2 ex, ey;
        if (ln.kind[e] == 1) {
            const LD k = ln.kp[e] >= 0 ? param(p, np, s, ln.kp[e], c) : ldc(ln.k[e]);
            ex = dpic::plane_map(k, L);
            ey = dpic::plane_map(-k, L);
        } else {
            ex = Map2{ldc(1.0), L, ldc(0.0), ldc(1.0)};
            ey = ex;
        }
        Mx = dpic::map_mul(ex, Mx);
        My = dpic::map_mul(ey, My);
    }
    LD t[4];
    if (en.periodic) {
        periodic_of(Mx, t[0], t[1]);
        periodic_of(My, t[2], t[3]);
    } else {
        twiss_of(Mx, ldc(en.tw0[0]), ldc(en.tw0[1]), t[0], t[1]);
        twiss_of(My, ldc(en.tw0[2]), ldc(en.tw0[3]), t[2], t[3]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) tw[((int64_t)s * 4 + q) * NC + c] = ldchan(t[q], c);
    if (en.has_target && f) {
        const LD dbx = t[0] - en.tgt[0], dax = t[1] - en.tgt[1], dby = t[2] - en.tgt[2], day = t[3] - en.tgt[3];
        const LD v = dbx * dbx * (1.0 / (en.tgt[0] * en.tgt[0])) + dax * dax + dby * dby * (1.0 / (en.tgt[2] * en.tgt[2])) +
                     day * day;
        f[(int64_t)s * NC + c] = ldchan(v, c);
    }
}

struct Bufs {
    double *p, *tw, *f;
};

size_t layout(int nb, char* base, Bufs* b) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return base ? (double*)(base + o) : nullptr;
    };
    Bufs t;
    t.p = take((size_t)nb * DPIC_MAX_PARAMS * 8);
    t.tw = take((size_t)nb * 4 * NC * 8);
    t.f = take((size_t)nb * NC * 8);
    if (b) *b = t;
    return off;
}

int make_line(int n_elem, const int* kind, const double* L, const double* k, const int* lp, const int* kp, int np, Line* ln) {
    if (n_elem < 1 || n_elem > DPIC_MAX_ELEMENTS || !kind) return DPIC_EINVAL;
    ln->n = n_elem;
    for (int e = 0; e < n_elem; ++e) {
        ln->kind[e] = kind[e];
        ln->lp[e] = lp ? lp[e] : -1;
        ln->kp[e] = kp ? kp[e] : -1;
        ln->L[e] = L ? L[e] : 0.0;
        ln->k[e] = k ? k[e] : 0.0;
        if ((kind[e] != 0 && kind[e] != 1) || ln->lp[e] >= np || ln->kp[e] >= np || ln->lp[e] < -1 || ln->kp[e] < -1)
            return DPIC_EINVAL;
        if (ln->lp[e] < 0 && (!L || !isfinite(L[e]))) return DPIC_EINVAL;
        if (kind[e] == 1 && ln->kp[e] < 0 && (!k || !isfinite(k[e]))) return DPIC_EINVAL;
    }
    return DPIC_OK;
}

// Evaluate nb vectors (host in, host out); twiss [nb][4][1+np], f [nb][1+np].
int eval(void* ws, size_t bytes, hipStream_t st, const Line& ln, const Ends& en, int np, int nb, const double* p,
         double* twiss, double* f) {
    if (nb < 1 || nb > MAX_NB || np < 0 || np > 15) return DPIC_EINVAL;
    if (!ws || bytes < layout(nb, nullptr, nullptr) || (uintptr_t)ws % 256) return DPIC_EINVAL;
    Bufs b;
    layout(nb, (char*)ws, &b);
    if (np > 0 && hipMemcpyAsync(b.p, p, (size_t)nb * np * 8, hipMemcpyHostToDevice, st) != hipSuccess) return DPIC_EHIP;
    hipLaunchKernelGGL(k_twiss, dim3((nb * NC + 255) / 256), dim3(256), 0, st, ln, en, b.p, np, nb, b.tw, b.f);
    if (hipGetLastError() != hipSuccess) return DPIC_EHIP;
    std::vector<double> h((size_t)nb * 4 * NC), hf((size_t)nb * NC);
    if (hipMemcpyAsync(h.data(), b.tw, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess) return DPIC_EHIP;
    if (en.has_target && hipMemcpyAsync(hf.data(), b.f, hf.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
        return DPIC_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DPIC_EHIP;
    for (int s = 0; s < nb; ++s) {
        for (int q = 0; q < 4; ++q)
            for (int ch = 0; ch <= np; ++ch) twiss[((size_t)s * 4 + q) * (np + 1) + ch] = h[((size_t)s * 4 + q) * NC + ch];
        if (f && en.has_target)
            for (int ch = 0; ch <= np; ++ch) f[(size_t)s * (np + 1) + ch] = hf[(size_t)s * NC + ch];
    }
    return DPIC_OK;
}

}  // namespace dtwiss

extern "C" {

int dtwiss_query_workspace(int nb, size_t* bytes) {
    if (nb < 1 || nb > dtwiss::MAX_NB || !bytes) return DPIC_EINVAL;
    *bytes = dtwiss::layout(nb, nullptr, nullptr);
    return DPIC_OK;
}

int dtwiss_eval(void* ws, size_t bytes, void* stream, int n_elem, const int* kind, const double* L, const double* k,
                const int* L_param, const int* k_param, int np, int nb, const double* p, const double* twiss0,
                const double* target, double* twiss, double* f) {
    using namespace dtwiss;
    if (!twiss || (np > 0 && !p)) return DPIC_EINVAL;
    Line ln;
    int r = make_line(n_elem, kind, L, k, L_param, k_param, np, &ln);
    if (r != DPIC_OK) return r;
    Ends en{};
    en.periodic = twiss0 == nullptr;
    for (int q = 0; q < 4; ++q) {
        en.tw0[q] = twiss0 ? twiss0[q] : 0.0;
        en.tgt[q] = target ? target[q] : 1.0;
    }
    en.has_target = target != nullptr;
    if (twiss0 && (!(twiss0[0] > 0) || !(twiss0[2] > 0))) return DPIC_EINVAL;
    if (target && (!(target[0] > 0) || !(target[2] > 0))) return DPIC_EINVAL;
    return eval(ws, bytes, (hipStream_t)stream, ln, en, np, nb, p, twiss, f);
}

int dtwiss_match(void* ws, size_t bytes, void* stream, int n_elem, const int* kind, const double* L, const double* k,
                 const int* L_param, const int* k_param, int np, const double* p0, const double* twiss0,
                 const double* target, double tol, int max_eval, double* p_out, double* f_out, int* n_eval,
                 double* history) {
    using namespace dtwiss;
    if (!p0 || !twiss0 || !target || !p_out || np < 1 || np > 15 || max_eval < 2) return DPIC_EINVAL;
    Line ln;
    int r = make_line(n_elem, kind, L, k, L_param, k_param, np, &ln);
    if (r != DPIC_OK) return r;
    Ends en{};
    en.periodic = 0;
    en.has_target = 1;
    for (int q = 0; q < 4; ++q) {
        en.tw0[q] = twiss0[q];
        en.tgt[q] = target[q];
    }
    const hipStream_t st = (hipStream_t)stream;
    int evals = 0;
    int err = DPIC_OK;
    std::vector<double> tw(4 * (np + 1)), fv(np + 1);
    // f and its gradient at x (one evaluation)
    auto fg = [&](const std::vector<double>& x, std::vector<double>* g) -> double {
        if (err != DPIC_OK) return INFINITY;
        err = eval(ws, bytes, st, ln, en, np, 1, x.data(), tw.data(), fv.data());
        if (history && evals < max_eval) history[evals] = fv[0];
        ++evals;
        if (g)
            for (int j = 0; j < np; ++j) (*g)[j] = fv[1 + j];
        return fv[0];
    };
    std::vector<double> x(p0, p0 + np);
    double fx;
    std::vector<double> g(np), gn(np), d(np), xn(np), H((size_t)np * np, 0.0);
    for (int i = 0; i < np; ++i) H[(size_t)i * np + i] = 1.0;
    fx = fg(x, &g);
    while (evals < max_eval && fx >= tol && err == DPIC_OK) {
        double gd = 0.0;
        for (int i = 0; i < np; ++i) {
            double s = 0.0;
            for (int j = 0; j < np; ++j) s -= H[(size_t)i * np + j] * g[j];
            d[i] = s;
            gd += g[i] * s;
        }
        if (gd >= 0) {  // not a descent direction: restart from steepest descent
            std::fill(H.begin(), H.end(), 0.0);
            for (int i = 0; i < np; ++i) H[(size_t)i * np + i] = 1.0, d[i] = -g[i];
            gd = 0.0;
            for (int i = 0; i < np; ++i) gd -= g[i] * g[i];
        }
        double t = 1.0, fn = fx;
        while (evals < max_eval) {
            for (int i = 0; i < np; ++i) xn[i] = x[i] + t * d[i];
            fn = fg(xn, &gn);
            if (fn <= fx + 1e-4 * t * gd || t < 1e-12) break;
            t *= 0.5;
        }
        // BFGS inverse-Hessian update with s = xn - x, y = gn - g
        std::vector<double> s(np), y(np), Hy(np);
        double ys = 0.0;
        for (int i = 0; i < np; ++i) {
            s[i] = xn[i] - x[i];
            y[i] = gn[i] - g[i];
            ys += y[i] * s[i];
        }
        if (ys > 1e-300) {
            const double rr = 1.0 / ys;
            double yHy = 0.0;
            for (int i = 0; i < np; ++i) {
                double v = 0.0;
                for (int j = 0; j < np; ++j) v += H[(size_t)i * np + j] * y[j];
                Hy[i] = v;
                yHy += y[i] * v;
            }
            // H <- H - r (Hy s^T + s (Hy)^T) + (r^2 yHy + r) s s^T  (H symmetric)
            for (int i = 0; i < np; ++i)
                for (int j = 0; j < np; ++j)
                    H[(size_t)i * np + j] += -rr * (Hy[i] * s[j] + s[i] * Hy[j]) + (rr * rr * yHy + rr) * s[i] * s[j];
        }
        x = xn;
        fx = fn;
        g = gn;
    }
    if (err != DPIC_OK) return err;
    for (int j = 0; j < np; ++j) p_out[j] = x[j];
    if (f_out) *f_out = fx;
    if (n_eval) *n_eval = evals;
    return DPIC_OK;
}

}  // extern "C"
