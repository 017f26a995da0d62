// C ABI of the dpic library: argument checking, workspace layout, the step
// schedule and host<->device marshalling. All arithmetic of the method runs in
// the kernels of particles.hip, solver.hip and moments.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "context.hpp"

using namespace dpic;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int fail(dpic_ctx* c, int code, const char* fmt, ...) {
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

bool grid_ok(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }

int check_dims(const dpic_dims* d) {
    if (!d) return DPIC_EINVAL;
    if (d->n_particles < 1 || d->n_particles > (int64_t)0x7fffffff) return DPIC_EINVAL;
    if (d->flags != 0) return DPIC_EINVAL;
    if (d->ntan < 0 || d->ntan > 15) return DPIC_EUNSUPPORTED;
    if (!grid_ok(d->nx) || !grid_ok(d->ny) || !grid_ok(d->nz)) return DPIC_EUNSUPPORTED;
    return DPIC_OK;
}

// Event pairs around stage launches (optional timing).
void timer_begin(dpic_ctx* c, int stage, hipEvent_t* out_end) {
    *out_end = nullptr;
    if (!c->stage_timing) return;
    auto& pool = c->ev_pool[stage];
    size_t i = c->ev_used[stage]++;
    if (i >= pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            c->ev_used[stage]--;
            return;
        }
        pool.emplace_back(a, b);
    }
    (void)hipEventRecord(pool[i].first, c->stream);
    *out_end = pool[i].second;
}

void timer_end(dpic_ctx* c, int stage, hipEvent_t end) {
    if (!end) return;
    (void)hipEventRecord(end, c->stream);
    c->stage_launches[stage]++;
}

enum { T_PART = 0, T_SOLVE = 1, T_FIELD = 2, T_SORT = 3 };

int run_particles(dpic_ctx* c, int flags, int e_tau, const double* map) {
    hipEvent_t end;
    timer_begin(c, T_PART, &end);
    HIPCHK(c, launch_particles(c, flags, e_tau, map, c->sort_every > 0 && c->chunks_valid));
    timer_end(c, T_PART, end);
    return DPIC_OK;
}

// Map block that ends step s: the second half step of element e(s) fused with
// the first half step of e(s+1), or the lone half step on the last step of a call.
const double* closing_map(const dpic_ctx* c, int64_t s, bool last) {
    const int e = c->schedule[s];
    if (last) return element_map_block(c, e, EC_HALF);
    const int en = c->schedule[s + 1];
    return element_map_block(c, e, en == e ? EC_SAME : EC_NEXT);
}

int run_solve_field(dpic_ctx* c);

// One unfused step s: half map + deposit, solve, field, kick + half map.
// When e_store is given, the step's field is copied there (adjoint replay).
int single_step(dpic_ctx* c, int64_t s, double* e_store) {
    const int e = c->schedule[s];
    const double* half = element_map_block(c, e, EC_HALF);
    int r;
    if (c->bunch_charge != 0.0) {
        if ((r = run_particles(c, PF_MAP | PF_DEPOSIT, e, half)) != DPIC_OK) return r;
        if ((r = run_solve_field(c)) != DPIC_OK) return r;
        if (e_store)
            HIPCHK(c, hipMemcpyAsync(e_store, c->ws.E, (size_t)c->dims.nx * c->dims.ny * c->dims.nz * 3 * c->NC * sizeof(double),
                                     hipMemcpyDeviceToDevice, c->stream));
        return run_particles(c, PF_KICK | PF_MAP, e, half);
    }
    if ((r = run_particles(c, PF_MAP | PF_COUNT, e, half)) != DPIC_OK) return r;
    return run_particles(c, PF_MAP, e, half);
}

int run_solve_field(dpic_ctx* c) {
    hipEvent_t end;
    timer_begin(c, T_SOLVE, &end);
    HIPCHK(c, launch_solve(c));
    timer_end(c, T_SOLVE, end);
    timer_begin(c, T_FIELD, &end);
    HIPCHK(c, launch_field(c));
    timer_end(c, T_FIELD, end);
    return DPIC_OK;
}

int run_sort(dpic_ctx* c) {
    hipEvent_t end;
    timer_begin(c, T_SORT, &end);
    HIPCHK(c, launch_sort(c));
    timer_end(c, T_SORT, end);
    return DPIC_OK;
}

bool consts_possible(const dpic_ctx* c) {
    if (!c->beam_set || !c->lattice_set) return false;
    for (int e = 0; e < c->n_elem; ++e)
        if (c->L_param[e] >= 0 || c->k_param[e] >= 0)
            if (!c->params_set) return false;
    return true;
}

// Upload element L and k duals (value + seed rows of the bound parameters) and
// compute the per-element constants on the device.
int refresh_elements(dpic_ctx* c) {
    if (!consts_possible(c)) return DPIC_OK;
    const int NC = c->NC, nt = c->ntan;
    std::vector<double> in((size_t)c->n_elem * 2 * NC, 0.0);
    for (int e = 0; e < c->n_elem; ++e) {
        double* Ld = &in[(size_t)(e * 2 + 0) * NC];
        double* kd = &in[(size_t)(e * 2 + 1) * NC];
        const int lp = c->L_param[e], kp = c->k_param[e];
        if (lp >= 0) {
            if (lp >= (int)c->p.size()) return fail(c, DPIC_EINVAL, "element %d binds L to parameter %d of %zu", e, lp, c->p.size());
            Ld[0] = c->p[lp];
            for (int t = 0; t < nt; ++t) Ld[1 + t] = c->seed[(size_t)lp * nt + t];
        } else {
            Ld[0] = c->L[e];
        }
        if (c->kind[e] == 1) {
            if (kp >= 0) {
                if (kp >= (int)c->p.size()) return fail(c, DPIC_EINVAL, "element %d binds k to parameter %d of %zu", e, kp, c->p.size());
                kd[0] = c->p[kp];
                for (int t = 0; t < nt; ++t) kd[1 + t] = c->seed[(size_t)kp * nt + t];
            } else {
                kd[0] = c->k[e];
            }
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->ws.elem_in, in.data(), in.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_element_consts(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

bool elements_ready(const dpic_ctx* c) { return consts_possible(c); }

// copy a device array with channel stride NC into host [rows][1+ntan]
void repack_out(const std::vector<double>& dev, size_t rows, int NC, int nt, double* out) {
    for (size_t r = 0; r < rows; ++r)
        for (int ch = 0; ch <= nt; ++ch) out[r * (nt + 1) + ch] = dev[r * NC + ch];
}

bool all_finite(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

}  // namespace

namespace dpic {

size_t workspace_layout(const dpic_dims& d, char* base, Workspace* ws) {
    const int NC = channels_for(d.ntan);
    const int NCC = NC == 1 ? 1 : NC / 2;
    const size_t cap = (size_t)d.n_particles;
    const size_t nx = d.nx, ny = d.ny, nz = d.nz;
    const size_t Mx = 2 * nx, My = 2 * ny, Mz = 2 * nz;
    const size_t W = Mx * NCC;
    size_t fft = std::max({nz * ny * W, nz * My * W, (nz + 2) * My * W, (nz + 2) * (ny + 2) * W, Mx * My * Mz});
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return base ? base + o : nullptr;
    };
    Workspace w;
    w.st = (double*)take(6 * cap * NC * sizeof(double));
    w.st2 = (double*)take(6 * cap * NC * sizeof(double));
    w.pid = (int32_t*)take(cap * sizeof(int32_t));
    w.pid2 = (int32_t*)take(cap * sizeof(int32_t));
    w.key = (uint32_t*)take(cap * sizeof(uint32_t));
    size_t nbins = 1;
    for (size_t nd : {nx, ny, nz}) nbins *= (nd - 1 + TILE_EDGE - 1) / TILE_EDGE;
    nbins += 1;
    const size_t sort_blocks = (cap + SORT_PB - 1) / SORT_PB;
    const size_t ncount = nbins * sort_blocks;
    w.counts = (uint32_t*)take(ncount * sizeof(uint32_t));
    w.seg = (uint32_t*)take(((ncount + 1023) / 1024 + 1) * sizeof(uint32_t));
    w.chunks = (int4*)take((nbins + (cap + TILE_CHUNK - 1) / TILE_CHUNK + 1) * sizeof(int4));
    w.nchunks = (uint32_t*)take(sizeof(uint32_t));
    w.rho = (double*)take(nx * ny * nz * NC * sizeof(double));
    w.phi = (double*)take((nx + 2) * (ny + 2) * (nz + 2) * NC * sizeof(double));
    w.E = (double*)take(nx * ny * nz * 3 * NC * sizeof(double));
    w.buf0 = (double2*)take(fft * sizeof(double2));
    w.buf1 = (double2*)take(fft * sizeof(double2));
    w.ghat = (double*)take((nx + 1) * (ny + 1) * (nz + 1) * sizeof(double));
    w.tw = (double2*)take((Mx + My + Mz) * sizeof(double2));
    w.ec = (double*)take((size_t)DPIC_MAX_ELEMENTS * EC_N * NC * sizeof(double));
    w.elem_in = (double*)take((size_t)DPIC_MAX_ELEMENTS * 2 * NC * sizeof(double));
    w.counters = (unsigned long long*)take(CNT_N * sizeof(unsigned long long));
    w.mom_part = (double*)take((size_t)MOM_BLOCKS * MOM_N * NC * sizeof(double));
    w.mom = (double*)take((size_t)MOM_N * NC * sizeof(double));
    w.emit = (double*)take((size_t)6 * NC * sizeof(double));
    w.bytes = off;
    if (ws) *ws = w;
    return off;
}

size_t adjoint_layout(const dpic_dims& d, int nmax, int K, char* base, AdjointWs* out) {
    const size_t cap = (size_t)d.n_particles;
    const size_t nodes = (size_t)d.nx * d.ny * d.nz;
    const size_t nck = ((size_t)nmax + K - 1) / K;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return base ? (double*)(base + o) : nullptr;
    };
    AdjointWs a;
    a.K = K;
    a.nmax = nmax;
    a.ckpt = take(nck * 6 * cap * sizeof(double));
    a.xi = take(6 * cap * sizeof(double));
    a.states = take((size_t)K * 6 * cap * sizeof(double));
    a.fields = take((size_t)K * 3 * nodes * sizeof(double));
    a.lam = take(6 * cap * sizeof(double));
    a.gacc = take((size_t)DPIC_MAX_ELEMENTS * 10 * sizeof(double));
    a.ec_dual = take((size_t)DPIC_MAX_ELEMENTS * EC_N * 16 * sizeof(double));
    a.elem_in_dual = take((size_t)DPIC_MAX_ELEMENTS * 2 * 16 * sizeof(double));
    a.grad = take(((size_t)DPIC_MAX_PARAMS + 6) * sizeof(double));
    if (out) *out = a;
    return off;
}

}  // namespace dpic

extern "C" {

int dpic_version(void) { return 10000; }

int dpic_query_workspace(const dpic_dims* dims, size_t* bytes) {
    int r = check_dims(dims);
    if (r != DPIC_OK) return r;
    if (!bytes) return DPIC_EINVAL;
    *bytes = workspace_layout(*dims, nullptr, nullptr);
    return DPIC_OK;
}

int dpic_create(const dpic_dims* dims, void* workspace_dev, size_t workspace_bytes, void* hip_stream, dpic_ctx** out) {
    int r = check_dims(dims);
    if (r != DPIC_OK) return r;
    if (!out || !workspace_dev) return DPIC_EINVAL;
    if (((uintptr_t)workspace_dev) % ALIGN != 0) return DPIC_EINVAL;
    const size_t need = workspace_layout(*dims, nullptr, nullptr);
    if (workspace_bytes < need) return DPIC_EINVAL;
    dpic_ctx* c = new (std::nothrow) dpic_ctx();
    if (!c) return DPIC_EINVAL;
    c->dims = *dims;
    c->ntan = dims->ntan;
    c->NC = channels_for(dims->ntan);
    c->stream = (hipStream_t)hip_stream;
    workspace_layout(*dims, (char*)workspace_dev, &c->ws);
    *out = c;
    return DPIC_OK;
}

int dpic_destroy(dpic_ctx* c) {
    if (!c) return DPIC_EINVAL;
    for (auto& pool : c->ev_pool)
        for (auto& pr : pool) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete c;
    return DPIC_OK;
}

int dpic_last_error(const dpic_ctx* c, char* buf, size_t len) {
    if (!c || !buf || len == 0) return DPIC_EINVAL;
    snprintf(buf, len, "%s", c->err.c_str());
    return DPIC_OK;
}

int dpic_set_beam(dpic_ctx* c, double kinetic_eV, double rest_eV, double charge_e, double bunch_charge_C) {
    if (!c) return DPIC_EINVAL;
    if (!(kinetic_eV > 0) || !(rest_eV > 0) || !isfinite(kinetic_eV) || !isfinite(rest_eV) || !isfinite(charge_e) ||
        !isfinite(bunch_charge_C))
        return fail(c, DPIC_EINVAL, "beam: energies must be positive and all values finite");
    c->gamma0 = 1.0 + kinetic_eV / rest_eV;
    c->beta0 = sqrt(1.0 - 1.0 / (c->gamma0 * c->gamma0));
    const double q_over_mc2 = charge_e / rest_eV;  // (q/e) / (mc^2 / e) in 1/V
    c->kperp = q_over_mc2 / (c->beta0 * c->beta0 * c->gamma0 * c->gamma0);
    c->kpar = q_over_mc2 / (c->beta0 * c->beta0 * c->gamma0);
    c->bunch_charge = bunch_charge_C;
    c->beam_set = true;
    if (c->grid_set) {
        HIPCHK(c, launch_green(c));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return refresh_elements(c);
}

int dpic_set_grid(dpic_ctx* c, const double lo[3], const double hi[3]) {
    if (!c || !lo || !hi) return DPIC_EINVAL;
    if (!c->beam_set) return fail(c, DPIC_ESTATE, "set_grid needs set_beam first (the kernel depends on gamma0)");
    const int n[3] = {c->dims.nx, c->dims.ny, c->dims.nz};
    for (int d = 0; d < 3; ++d) {
        if (!isfinite(lo[d]) || !isfinite(hi[d]) || !(hi[d] > lo[d]))
            return fail(c, DPIC_EINVAL, "grid: need finite lo < hi in dimension %d", d);
        c->lo[d] = lo[d];
        c->hi[d] = hi[d];
        c->h[d] = (hi[d] - lo[d]) / (double)(n[d] - 1);
    }
    HIPCHK(c, launch_green(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->grid_set = true;
    c->chunks_valid = false;
    return DPIC_OK;
}

int dpic_set_lattice(dpic_ctx* c, int n_elem, const int* kind, const int* n_steps, const double* L, const double* k,
                     const int* L_param, const int* k_param, int n_periods) {
    if (!c) return DPIC_EINVAL;
    if (n_elem < 1 || n_elem > DPIC_MAX_ELEMENTS || !kind || !n_steps || n_periods < 1)
        return fail(c, DPIC_EINVAL, "lattice: need 1..%d elements and n_periods >= 1", DPIC_MAX_ELEMENTS);
    int64_t total = 0;
    for (int e = 0; e < n_elem; ++e) {
        if (kind[e] != 0 && kind[e] != 1) return fail(c, DPIC_EINVAL, "lattice: element %d kind %d", e, kind[e]);
        if (n_steps[e] < 1) return fail(c, DPIC_EINVAL, "lattice: element %d has %d steps", e, n_steps[e]);
        const int lp = L_param ? L_param[e] : -1, kp = k_param ? k_param[e] : -1;
        if (lp < -1 || lp >= DPIC_MAX_PARAMS || kp < -1 || kp >= DPIC_MAX_PARAMS)
            return fail(c, DPIC_EINVAL, "lattice: element %d parameter index out of range", e);
        if (lp < 0 && (!L || !isfinite(L[e]))) return fail(c, DPIC_EINVAL, "lattice: element %d needs a fixed L", e);
        if (kind[e] == 1 && kp < 0 && (!k || !isfinite(k[e])))
            return fail(c, DPIC_EINVAL, "lattice: element %d needs a fixed k", e);
        total += n_steps[e];
    }
    total *= n_periods;
    if (total > (int64_t)100000000) return fail(c, DPIC_EINVAL, "lattice: schedule too long");
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
    return refresh_elements(c);
}

int dpic_set_params(dpic_ctx* c, int np, const double* p, const double* seed) {
    if (!c) return DPIC_EINVAL;
    if (np < 0 || np > DPIC_MAX_PARAMS || (np > 0 && !p)) return fail(c, DPIC_EINVAL, "params: 0..%d values", DPIC_MAX_PARAMS);
    const int nt = c->ntan;
    c->p.assign(p, p + np);
    c->seed.assign((size_t)np * nt, 0.0);
    for (int j = 0; j < np; ++j) {
        if (!isfinite(p[j])) return fail(c, DPIC_EINVAL, "params: p[%d] not finite", j);
        for (int t = 0; t < nt; ++t) {
            const double v = seed ? seed[(size_t)j * nt + t] : (j == t ? 1.0 : 0.0);
            if (!isfinite(v)) return fail(c, DPIC_EINVAL, "params: seed[%d][%d] not finite", j, t);
            c->seed[(size_t)j * nt + t] = v;
        }
    }
    c->params_set = true;
    return refresh_elements(c);
}

int dpic_init_beam(dpic_ctx* c, int64_t n, const double* xi_dev, const double sigma[6], const double* sigma_seed) {
    if (!c || !sigma) return DPIC_EINVAL;
    if (n < 0 || n > c->dims.n_particles) return fail(c, DPIC_EINVAL, "init_beam: n=%lld outside 0..capacity", (long long)n);
    if (n > 0 && !xi_dev) return fail(c, DPIC_EINVAL, "init_beam: xi_dev is NULL");
    const int NC = c->NC, nt = c->ntan;
    std::vector<double> sd((size_t)6 * NC, 0.0);
    for (int j = 0; j < 6; ++j) {
        if (!isfinite(sigma[j])) return fail(c, DPIC_EINVAL, "init_beam: sigma[%d] not finite", j);
        sd[(size_t)j * NC] = sigma[j];
        if (sigma_seed)
            for (int t = 0; t < nt; ++t) sd[(size_t)j * NC + 1 + t] = sigma_seed[(size_t)j * nt + t];
    }
    c->n = n;
    HIPCHK(c, launch_init_beam(c, xi_dev, sd.data()));
    if (c->adj.bound && n > 0)  // the adjoint needs xi for d/dsigma
        HIPCHK(c, hipMemcpyAsync(c->adj.xi, xi_dev, (size_t)n * 6 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_zero(c, (double*)c->ws.counters, CNT_N));
    HIPCHK(c, launch_zero(c, c->ws.rho, (size_t)c->dims.nx * c->dims.ny * c->dims.nz * NC));
    c->steps_done = 0;
    c->beam_init = true;
    c->chunks_valid = false;
    return DPIC_OK;
}

int dpic_step(dpic_ctx* c, int n) {
    if (!c) return DPIC_EINVAL;
    if (n < 0) return fail(c, DPIC_EINVAL, "step: n < 0");
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "step: call init_beam first");
    if (!elements_ready(c)) return fail(c, DPIC_ESTATE, "step: beam, lattice and parameters must be set");
    const bool sc = c->bunch_charge != 0.0;
    if (sc && !c->grid_set) return fail(c, DPIC_ESTATE, "step: space charge needs set_grid");
    if (n == 0) return DPIC_OK;
    if (c->steps_done + n > (int64_t)c->schedule.size())
        return fail(c, DPIC_EINVAL, "step: %d steps from %lld exceed the schedule of %zu", n, (long long)c->steps_done,
                    c->schedule.size());
    const int64_t s0 = c->steps_done, s1 = s0 + n;
    int r;
    if (sc && c->sort_every > 0 && !c->chunks_valid)
        if ((r = run_sort(c)) != DPIC_OK) return r;
    if (c->adj.bound) {
        // reverse-mode forward: unfused steps (the backward replays the same
        // sequence), a checkpoint every K steps, no re-sorting (the adjoint
        // follows the stored particle order)
        if (s1 > c->adj.nmax) return fail(c, DPIC_EINVAL, "step: the adjoint workspace covers %d steps", c->adj.nmax);
        HIPCHK(c, launch_zero(c, c->ws.rho, (size_t)c->dims.nx * c->dims.ny * c->dims.nz * c->NC));
        const size_t sbytes = (size_t)6 * c->dims.n_particles * sizeof(double);
        for (int64_t s = s0; s < s1; ++s) {
            if (s % c->adj.K == 0)
                HIPCHK(c, hipMemcpyAsync(c->adj.ckpt + (size_t)(s / c->adj.K) * 6 * c->dims.n_particles, c->ws.st,
                                         sbytes, hipMemcpyDeviceToDevice, c->stream));
            if ((r = single_step(c, s, nullptr)) != DPIC_OK) return r;
        }
        c->steps_done = s1;
        return DPIC_OK;
    }
    if (sc) {
        HIPCHK(c, launch_zero(c, c->ws.rho, (size_t)c->dims.nx * c->dims.ny * c->dims.nz * c->NC));
        const double* first = element_map_block(c, c->schedule[s0], EC_HALF);
        if ((r = run_particles(c, PF_MAP | PF_DEPOSIT, c->schedule[s0], first)) != DPIC_OK) return r;
        for (int64_t s = s0; s < s1; ++s) {
            if ((r = run_solve_field(c)) != DPIC_OK) return r;
            const bool last = (s == s1 - 1);
            const int flags = PF_KICK | PF_MAP | (last ? 0 : PF_DEPOSIT);
            if ((r = run_particles(c, flags, c->schedule[s], closing_map(c, s, last))) != DPIC_OK) return r;
            if (c->sort_every > 0 && !last && ((s + 1) % c->sort_every) == 0)
                if ((r = run_sort(c)) != DPIC_OK) return r;
        }
    } else {
        const double* first = element_map_block(c, c->schedule[s0], EC_HALF);
        if ((r = run_particles(c, PF_MAP | PF_COUNT, c->schedule[s0], first)) != DPIC_OK) return r;
        for (int64_t s = s0; s < s1; ++s) {
            const bool last = (s == s1 - 1);
            const int flags = PF_MAP | (last ? 0 : PF_COUNT);
            if ((r = run_particles(c, flags, c->schedule[s], closing_map(c, s, last))) != DPIC_OK) return r;
        }
    }
    c->steps_done = s1;
    return DPIC_OK;
}

int dpic_read_moments(dpic_ctx* c, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "read_moments: no beam");
    HIPCHK(c, launch_moments(c));
    std::vector<double> h((size_t)MOM_N * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->ws.mom, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    repack_out(h, MOM_N, c->NC, c->ntan, out);
    if (!all_finite(out, (size_t)MOM_N * (c->ntan + 1))) return fail(c, DPIC_ENONFINITE, "read_moments: non-finite moment");
    return DPIC_OK;
}

int dpic_read_emittance(dpic_ctx* c, int centred, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "read_emittance: no beam");
    HIPCHK(c, launch_moments(c));
    std::vector<double> h((size_t)6 * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->ws.emit, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> part(h.begin() + (centred ? 3 * c->NC : 0), h.begin() + (centred ? 6 : 3) * c->NC);
    repack_out(part, 3, c->NC, c->ntan, out);
    if (!all_finite(out, (size_t)3 * (c->ntan + 1))) return fail(c, DPIC_ENONFINITE, "read_emittance: non-finite emittance");
    return DPIC_OK;
}

int dpic_read_particles(dpic_ctx* c, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "read_particles: no beam");
    if (c->n == 0) return DPIC_OK;
    HIPCHK(c, launch_canonical_state(c));
    std::vector<double> h((size_t)c->n * 6 * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->ws.st2, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    repack_out(h, (size_t)c->n * 6, c->NC, c->ntan, out);
    return DPIC_OK;
}

int dpic_counters(dpic_ctx* c, int64_t* out_of_box, int64_t* steps_done, double* extent) {
    if (!c) return DPIC_EINVAL;
    unsigned long long h[CNT_N];
    HIPCHK(c, hipMemcpyAsync(h, c->ws.counters, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (out_of_box) *out_of_box = (int64_t)h[CNT_OUTSIDE];
    if (steps_done) *steps_done = c->steps_done;
    if (extent)
        for (int d = 0; d < 3; ++d) memcpy(&extent[d], &h[CNT_EXT_X + d], sizeof(double));
    return DPIC_OK;
}

int dpic_stage(dpic_ctx* c, int stage) {
    if (!c) return DPIC_EINVAL;
    switch (stage) {
        case DPIC_STAGE_DEPOSIT:
            if (!c->beam_init || !c->grid_set) return fail(c, DPIC_ESTATE, "stage deposit: needs beam and grid");
            HIPCHK(c, launch_zero(c, c->ws.rho, (size_t)c->dims.nx * c->dims.ny * c->dims.nz * c->NC));
            HIPCHK(c, launch_particles(c, PF_DEPOSIT, 0, nullptr, false));
            return DPIC_OK;
        case DPIC_STAGE_SOLVE:
            if (!c->grid_set) return fail(c, DPIC_ESTATE, "stage solve: needs grid");
            HIPCHK(c, launch_solve(c));
            return DPIC_OK;
        case DPIC_STAGE_FIELD:
            if (!c->grid_set) return fail(c, DPIC_ESTATE, "stage field: needs grid");
            HIPCHK(c, launch_field(c));
            return DPIC_OK;
        default:
            return fail(c, DPIC_EINVAL, "stage: unknown stage %d", stage);
    }
}

static int grid_geom(const dpic_ctx* c, int which, double** dev, size_t* rows, int* per_row) {
    const size_t nx = c->dims.nx, ny = c->dims.ny, nz = c->dims.nz;
    switch (which) {
        case DPIC_GRID_RHO: *dev = c->ws.rho; *rows = nx * ny * nz; *per_row = 1; return DPIC_OK;
        case DPIC_GRID_PHI: *dev = c->ws.phi; *rows = (nx + 2) * (ny + 2) * (nz + 2); *per_row = 1; return DPIC_OK;
        case DPIC_GRID_E: *dev = c->ws.E; *rows = nx * ny * nz * 3; *per_row = 1; return DPIC_OK;
        default: return DPIC_EINVAL;
    }
}

int dpic_read_grid(dpic_ctx* c, int which, double* out) {
    if (!c || !out) return DPIC_EINVAL;
    double* dev;
    size_t rows;
    int per;
    if (grid_geom(c, which, &dev, &rows, &per) != DPIC_OK) return fail(c, DPIC_EINVAL, "read_grid: unknown array %d", which);
    std::vector<double> h(rows * c->NC);
    HIPCHK(c, hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    repack_out(h, rows, c->NC, c->ntan, out);
    return DPIC_OK;
}

int dpic_write_grid(dpic_ctx* c, int which, const double* in) {
    if (!c || !in) return DPIC_EINVAL;
    double* dev;
    size_t rows;
    int per;
    if (grid_geom(c, which, &dev, &rows, &per) != DPIC_OK) return fail(c, DPIC_EINVAL, "write_grid: unknown array %d", which);
    const int NC = c->NC, nt = c->ntan;
    std::vector<double> h(rows * NC, 0.0);
    for (size_t r = 0; r < rows; ++r)
        for (int ch = 0; ch <= nt; ++ch) h[r * NC + ch] = in[r * (nt + 1) + ch];
    HIPCHK(c, hipMemcpyAsync(dev, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

// checkpoint layout: int64 header[2] = {n, steps_done}, pid[cap] (int32), state [6][cap][NC]
int dpic_state_bytes(const dpic_ctx* c, size_t* bytes) {
    if (!c || !bytes) return DPIC_EINVAL;
    const size_t cap = (size_t)c->dims.n_particles;
    *bytes = align_up(16 + cap * sizeof(int32_t)) + 6 * cap * c->NC * sizeof(double);
    return DPIC_OK;
}

int dpic_save_state(dpic_ctx* c, void* dev_buf) {
    if (!c || !dev_buf) return DPIC_EINVAL;
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "save_state: no beam");
    const size_t cap = (size_t)c->dims.n_particles;
    int64_t hdr[2] = {c->n, c->steps_done};
    char* b = (char*)dev_buf;
    HIPCHK(c, hipMemcpyAsync(b, hdr, sizeof hdr, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + 16, c->ws.pid, cap * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + align_up(16 + cap * sizeof(int32_t)), c->ws.st, 6 * cap * c->NC * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DPIC_OK;
}

int dpic_load_state(dpic_ctx* c, const void* dev_buf) {
    if (!c || !dev_buf) return DPIC_EINVAL;
    const size_t cap = (size_t)c->dims.n_particles;
    int64_t hdr[2];
    const char* b = (const char*)dev_buf;
    HIPCHK(c, hipMemcpyAsync(hdr, b, sizeof hdr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hdr[0] < 0 || hdr[0] > c->dims.n_particles || hdr[1] < 0)
        return fail(c, DPIC_EINVAL, "load_state: buffer does not hold a checkpoint of this context");
    HIPCHK(c, hipMemcpyAsync(c->ws.pid, b + 16, cap * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws.st, b + align_up(16 + cap * sizeof(int32_t)), 6 * cap * c->NC * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->n = hdr[0];
    c->steps_done = hdr[1];
    c->beam_init = true;
    c->chunks_valid = false;
    return DPIC_OK;
}

int dpic_set_option(dpic_ctx* c, int option, int64_t value) {
    if (!c) return DPIC_EINVAL;
    switch (option) {
        case DPIC_OPT_SORT_EVERY:
            if (value < 0) return fail(c, DPIC_EINVAL, "sort_every must be >= 0");
            c->sort_every = value;
            return DPIC_OK;
        case DPIC_OPT_STAGE_TIMING:
            c->stage_timing = value != 0;
            return DPIC_OK;
        default:
            return fail(c, DPIC_EINVAL, "unknown option %d", option);
    }
}

int dpic_stage_times(dpic_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms) return DPIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < DPIC_N_STAGE_TIMERS; ++s) {
        double tot = 0.0;
        for (size_t i = 0; i < c->ev_used[s]; ++i) {
            float t = 0.f;
            HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[s][i].first, c->ev_pool[s][i].second));
            tot += t;
        }
        ms[s] = tot;
        if (launches) launches[s] = c->stage_launches[s];
        c->ev_used[s] = 0;
        c->stage_launches[s] = 0;
    }
    return DPIC_OK;
}

int dpic_adjoint_query(const dpic_dims* dims, int n_steps, int checkpoint_every, size_t* bytes) {
    int r = check_dims(dims);
    if (r != DPIC_OK) return r;
    if (!bytes || dims->ntan != 0 || n_steps < 1 || checkpoint_every < 1) return DPIC_EINVAL;
    *bytes = adjoint_layout(*dims, n_steps, checkpoint_every, nullptr, nullptr);
    return DPIC_OK;
}

int dpic_adjoint_bind(dpic_ctx* c, void* adj_dev, size_t bytes, int n_steps, int checkpoint_every) {
    if (!c || !adj_dev) return DPIC_EINVAL;
    if (c->ntan != 0) return fail(c, DPIC_EINVAL, "adjoint: the context must be value-only (ntan = 0)");
    if (n_steps < 1 || checkpoint_every < 1) return fail(c, DPIC_EINVAL, "adjoint: n_steps and checkpoint_every >= 1");
    if (((uintptr_t)adj_dev) % ALIGN != 0) return fail(c, DPIC_EINVAL, "adjoint: workspace not 256-byte aligned");
    if (bytes < adjoint_layout(c->dims, n_steps, checkpoint_every, nullptr, nullptr))
        return fail(c, DPIC_EINVAL, "adjoint: workspace too small");
    adjoint_layout(c->dims, n_steps, checkpoint_every, (char*)adj_dev, &c->adj);
    c->adj.bound = true;
    c->beam_init = false;  // the initial normals must be captured by init_beam
    return DPIC_OK;
}

int dpic_adjoint_backward(dpic_ctx* c, const double w[3], double* grad_params, double* grad_sigma) {
    if (!c || !w) return DPIC_EINVAL;
    if (!c->adj.bound) return fail(c, DPIC_ESTATE, "backward: no adjoint workspace bound");
    if (!c->beam_init) return fail(c, DPIC_ESTATE, "backward: no forward run to differentiate");
    const int np = (int)c->p.size();
    if (np > 15) return fail(c, DPIC_EUNSUPPORTED, "backward: at most 15 parameters");
    for (int k = 0; k < 3; ++k)
        if (!isfinite(w[k])) return fail(c, DPIC_EINVAL, "backward: non-finite weight");
    const bool sc = c->bunch_charge != 0.0;
    const size_t cap = (size_t)c->dims.n_particles;
    const size_t nodes = (size_t)c->dims.nx * c->dims.ny * c->dims.nz;
    unsigned long long cnt[CNT_N];
    HIPCHK(c, hipMemcpyAsync(cnt, c->ws.counters, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, launch_adj_terminal(c, w));
    HIPCHK(c, launch_zero(c, c->adj.gacc, (size_t)DPIC_MAX_ELEMENTS * 10));
    const int64_t nf = c->steps_done;
    const int K = c->adj.K;
    int r;
    for (int64_t g = (nf + K - 1) / K - 1; g >= 0; --g) {
        const int64_t sa = g * K, sb = std::min<int64_t>(sa + K, nf);
        // replay the segment from its checkpoint, keeping each step's start state and field
        HIPCHK(c, hipMemcpyAsync(c->ws.st, c->adj.ckpt + (size_t)g * 6 * cap, 6 * cap * sizeof(double),
                                 hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, launch_zero(c, c->ws.rho, nodes));
        for (int64_t s = sa; s < sb; ++s) {
            HIPCHK(c, hipMemcpyAsync(c->adj.states + (size_t)(s - sa) * 6 * cap, c->ws.st, 6 * cap * sizeof(double),
                                     hipMemcpyDeviceToDevice, c->stream));
            if ((r = single_step(c, s, c->adj.fields + (size_t)(s - sa) * 3 * nodes)) != DPIC_OK) return r;
        }
        for (int64_t s = sb - 1; s >= sa; --s)
            HIPCHK(c, launch_adj_step(c, c->schedule[s], c->adj.states + (size_t)(s - sa) * 6 * cap,
                                      c->adj.fields + (size_t)(s - sa) * 3 * nodes, sc));
    }
    // element constants with one tangent per parameter (identity seeds)
    std::vector<double> in((size_t)c->n_elem * 2 * 16, 0.0);
    for (int e = 0; e < c->n_elem; ++e) {
        double* Ld = &in[(size_t)(e * 2 + 0) * 16];
        double* kd = &in[(size_t)(e * 2 + 1) * 16];
        const int lp = c->L_param[e], kp = c->k_param[e];
        Ld[0] = lp >= 0 ? c->p[lp] : c->L[e];
        if (lp >= 0) Ld[1 + lp] = 1.0;
        if (c->kind[e] == 1) {
            kd[0] = kp >= 0 ? c->p[kp] : c->k[e];
            if (kp >= 0) kd[1 + kp] = 1.0;
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->adj.elem_in_dual, in.data(), in.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_element_consts_into(c, 16, c->adj.elem_in_dual, c->adj.ec_dual));
    c->adj.ncd = 16;
    HIPCHK(c, launch_adj_finish(c, np));
    std::vector<double> g(DPIC_MAX_PARAMS + 6);
    HIPCHK(c, hipMemcpyAsync(g.data(), c->adj.grad, g.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws.counters, cnt, sizeof cnt, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (grad_params)
        for (int j = 0; j < np; ++j) grad_params[j] = g[j];
    if (grad_sigma)
        for (int j = 0; j < 6; ++j) grad_sigma[j] = g[DPIC_MAX_PARAMS + j];
    c->beam_init = false;  // the particle state now holds a replayed segment
    for (int j = 0; j < np; ++j)
        if (!isfinite(g[j])) return fail(c, DPIC_ENONFINITE, "backward: non-finite gradient");
    return DPIC_OK;
}

}  // extern "C"
