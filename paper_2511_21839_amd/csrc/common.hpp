// Shared device/host definitions of the dpic HIP library (gfx950).
//
// Dual numbers on the GPU (Sec. 2 algebra) use a lane-per-channel layout:
// a particle (or grid node) owns a group of NC consecutive lanes, lane c
// holding channel c of every dual quantity. Every lane also carries the value
// so that all arithmetic is lane-local: a product F G is (f g, g f_c + f g_c)
// in lane c without any cross-lane traffic. Lane 0's derivative slot is kept
// at zero, so the rules never need a per-lane branch; the value is written
// from lane 0 on store.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpic {

// ---------------------------------------------------------------- dual lane
struct LD {
    double v;  // value (uniform across the lane group)
    double t;  // this lane's derivative channel (0 in lane 0)
};

__device__ __forceinline__ LD ldc(double v) { return LD{v, 0.0}; }
__device__ __forceinline__ LD operator+(LD a, LD b) { return LD{a.v + b.v, a.t + b.t}; }
__device__ __forceinline__ LD operator-(LD a, LD b) { return LD{a.v - b.v, a.t - b.t}; }
__device__ __forceinline__ LD operator-(LD a) { return LD{-a.v, -a.t}; }
__device__ __forceinline__ LD operator+(LD a, double s) { return LD{a.v + s, a.t}; }
__device__ __forceinline__ LD operator+(double s, LD a) { return LD{a.v + s, a.t}; }
__device__ __forceinline__ LD operator-(double s, LD a) { return LD{s - a.v, -a.t}; }
__device__ __forceinline__ LD operator-(LD a, double s) { return LD{a.v - s, a.t}; }
// product rule
__device__ __forceinline__ LD operator*(LD a, LD b) { return LD{a.v * b.v, fma(a.v, b.t, a.t * b.v)}; }
__device__ __forceinline__ LD operator*(LD a, double s) { return LD{a.v * s, a.t * s}; }
__device__ __forceinline__ LD operator*(double s, LD a) { return LD{a.v * s, a.t * s}; }
// quotient rule: (f/g, (f_c - (f/g) g_c) / g)
__device__ __forceinline__ LD operator/(LD a, LD b) {
    double q = a.v / b.v;
    return LD{q, (a.t - q * b.t) / b.v};
}
// acc + a b
__device__ __forceinline__ LD fmad(LD a, LD b, LD acc) {
    return LD{fma(a.v, b.v, acc.v), fma(a.v, b.t, fma(a.t, b.v, acc.t))};
}
// function rule h(F) = (h(f), h'(f) f_c)
__device__ __forceinline__ LD dsqrt(LD a) {
    double s = sqrt(a.v);
    return LD{s, a.t * (0.5 / s)};
}
__device__ __forceinline__ LD dsin(LD a) { return LD{sin(a.v), cos(a.v) * a.t}; }
__device__ __forceinline__ LD dcos(LD a) { return LD{cos(a.v), -sin(a.v) * a.t}; }
__device__ __forceinline__ LD dsinh(LD a) { return LD{sinh(a.v), cosh(a.v) * a.t}; }
__device__ __forceinline__ LD dcosh(LD a) { return LD{cosh(a.v), sinh(a.v) * a.t}; }

// Load channel c of a dual stored with channel stride NC at p (p[0] is the value).
__device__ __forceinline__ LD ldload(const double* p, int c) {
    double v = p[0];
    double t = p[c];
    return LD{v, c ? t : 0.0};
}
// The channel this lane stores.
__device__ __forceinline__ double ldchan(LD a, int c) { return c ? a.t : a.v; }

// ---------------------------------------------------------------- maps
struct Map2 {
    LD a, b, c, d;
};

// Exact map of one plane with signed strength kk over length s (Sec. 4
// quadrupole maps; kk > 0 focusing, kk < 0 defocusing, kk = 0 a drift).
// Below |kk s^2| < 1e-8 the Taylor series in u = kk s^2 to u^3 is used.
__device__ inline Map2 plane_map(LD kk, LD s) {
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

__device__ inline Map2 map_mul(const Map2& B, const Map2& A) {  // B A
    return Map2{B.a * A.a + B.b * A.c, B.a * A.b + B.b * A.d, B.c * A.a + B.d * A.c, B.c * A.b + B.d * A.d};
}

// ---------------------------------------------------------------- layout
// Element constants: per element EC_N duals, each NC doubles. A "map block"
// is 9 consecutive duals: the (x, px) 2x2 map row-major, the (y, py) map,
// and the z slip coefficient (z += slip * delta).
enum ElemSlot {
    EC_TAU = 0,    // full step tau = L / n_steps
    EC_HALF = 1,   // map block of M1(tau/2)
    EC_SAME = 10,  // map block of M1(tau/2) M1(tau/2) (two half steps of this element)
    EC_NEXT = 19,  // map block of M1'(tau'/2) M1(tau/2) (this element, then the next one)
    EC_N = 28
};
enum MapSlot { MB_AX = 0, MB_AY = 4, MB_SLIP = 8, MB_N = 9 };

// Particle-kernel stage flags.
enum PartFlags {
    PF_KICK = 1,     // gather E with CIC weights and apply the kick of the current element
    PF_MAP = 2,      // apply one map block (a half step, or two fused half steps)
    PF_DEPOSIT = 4,  // CIC deposit at the resulting position (implies counting)
    PF_COUNT = 8,    // count out-of-box particles and track the extent
    PF_EHALO = 16,   // tiled kernel: E tile with the transverse drift allowance (see particles.hip)
    PF_KEYS = 32,    // with PF_DEPOSIT: write each particle's tile key for the sort that follows
    PF_SCATTER = 64  // tiled kernel: store each particle in its sorted slot of the second state buffer
};

// CNT_NONFINITE: 0 while every stored state value is finite, else
// NONFINITE_BASE - (first step whose particle launch stored a NaN or Inf)
enum CounterSlot { CNT_OUTSIDE = 0, CNT_EXT_X = 1, CNT_EXT_Y = 2, CNT_EXT_Z = 3, CNT_NONFINITE = 4, CNT_N = 8 };
constexpr unsigned long long NONFINITE_BASE = 1ull << 62;

constexpr int MOM_N = 15;  // 3 planes x 5 moments

// ---------------------------------------------------------------- grid cells
// Cell of a position on the node grid: s = (u - lo) / h per dimension, cell
// floor(s), inside iff 0 <= s < n - 1 in every dimension (all 8 corner nodes
// of the cell exist). Every kernel that decides in or out uses this.
struct CellPos {
    double sx, sy, sz;
    int ix, iy, iz;
    bool inside;
};

__device__ __forceinline__ CellPos grid_cell(double x, double y, double z, double lo0, double lo1, double lo2,
                                             double ih0, double ih1, double ih2, int nx, int ny, int nz) {
    CellPos r;
    r.sx = (x - lo0) * ih0;
    r.sy = (y - lo1) * ih1;
    r.sz = (z - lo2) * ih2;
    r.inside = (r.sx >= 0.0) && (r.sx < (double)(nx - 1)) && (r.sy >= 0.0) && (r.sy < (double)(ny - 1)) &&
               (r.sz >= 0.0) && (r.sz < (double)(nz - 1));
    r.ix = (int)floor(r.sx);
    r.iy = (int)floor(r.sy);
    r.iz = (int)floor(r.sz);
    return r;
}

__host__ __device__ constexpr int channels_for(int ntan) { return ntan == 0 ? 1 : (ntan <= 7 ? 8 : 16); }

}  // namespace dpic
