// Host-side context of the dpic library and the launchers each kernel file
// exports to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dpic.h"
#include "common.hpp"

namespace dpic {

struct Workspace {
    double* st = nullptr;      // particle state [6][cap][NC]
    double* st2 = nullptr;     // second state buffer (sort target, read-back staging)
    int32_t* pid = nullptr;    // original index of each stored particle
    int32_t* pid2 = nullptr;
    uint32_t* key = nullptr;     // sort keys
    uint32_t* counts = nullptr;  // per (bin, block) counts, then offsets
    uint32_t* seg = nullptr;     // scan segment sums
    int4* chunks = nullptr;      // tiled work list (tile, first, count, -)
    uint32_t* nchunks = nullptr;
    double* rho = nullptr;     // node charges [nz][ny][nx][NC]
    double* phi = nullptr;     // potential [nz+2][ny+2][nx+2][NC]
    double* E = nullptr;       // field [nz][ny][nx][3][NC]
    double2* buf0 = nullptr;   // FFT work arrays
    double2* buf1 = nullptr;
    double* ghat = nullptr;    // transform of G on the (nx+1)(ny+1)(nz+1) octant
    double2* tw = nullptr;     // twiddles exp(-2 pi i m / M) for M = 2nx, 2ny, 2nz
    double* ec = nullptr;      // element constants [MAX_ELEM][EC_N][NC]
    double* elem_in = nullptr; // uploaded element L and k duals [MAX_ELEM][2][NC]
    unsigned long long* counters = nullptr;
    double* mom_part = nullptr;  // moment partial sums [MOM_BLOCKS][MOM_N][NC]
    double* mom = nullptr;       // moments [MOM_N][NC]
    double* emit = nullptr;      // emittance [2][3][NC] (raw, centred)
    size_t bytes = 0;
};

constexpr int MOM_BLOCKS = 512;
constexpr int NUM_TILE_BINS_MAX = 4096;
constexpr int TILE_EDGE = 4;                             // cells per tile edge
constexpr int TILE_HALO = 1;                             // drift allowance (cells) of the LDS deposit
constexpr int TILE_R = TILE_EDGE + 2 * TILE_HALO + 1;    // LDS nodes per dimension
constexpr int TILE_CHUNK = 1024;                         // particles per tiled workgroup
constexpr int SORT_PB = 1024;                            // particles per sort block

size_t workspace_layout(const dpic_dims& d, char* base, Workspace* ws);

// Reverse-mode workspace (caller-owned, bound by dpic_adjoint_bind).
struct AdjointWs {
    bool bound = false;
    int K = 0;                     // checkpoint interval (steps)
    int nmax = 0;                  // steps the checkpoints cover
    int ncd = 16;                  // channels of the dual element table
    double* ckpt = nullptr;        // [ceil(nmax/K)][6][cap] state at steps 0, K, 2K, ...
    double* xi = nullptr;          // [cap][6] initial standard normals, original order
    double* states = nullptr;      // [K][6][cap] replayed state at each step's start
    double* fields = nullptr;      // [K][nz][ny][nx][3] replayed field of each step
    double* lam = nullptr;         // [6][cap] adjoint of the state
    double* gacc = nullptr;        // [MAX_ELEM][10] dJ/dA (9 map entries), dJ/dtau per element
    double* ec_dual = nullptr;     // [MAX_ELEM][EC_N][16] element constants with parameter tangents
    double* elem_in_dual = nullptr;
    double* grad = nullptr;        // [MAX_PARAMS + 6]
};

size_t adjoint_layout(const dpic_dims& d, int nmax, int K, char* base, AdjointWs* out);

}  // namespace dpic

struct dpic_ctx {
    dpic_dims dims{};
    int NC = 1;
    int ntan = 0;
    hipStream_t stream = nullptr;
    dpic::Workspace ws;
    std::string err;

    // beam
    bool beam_set = false;
    double gamma0 = 1, beta0 = 0, kperp = 0, kpar = 0, bunch_charge = 0;
    // grid
    bool grid_set = false;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    // lattice
    bool lattice_set = false;
    int n_elem = 0, n_periods = 1;
    std::vector<int> kind, n_steps, L_param, k_param;
    std::vector<double> L, k;
    std::vector<int> schedule;  // element index of every step
    // parameters
    bool params_set = false;
    std::vector<double> p, seed;  // seed [np][ntan]
    // beam state
    bool beam_init = false;
    int64_t n = 0;
    int64_t steps_done = 0;
    // options
    int64_t sort_every = 20;
    bool chunks_valid = false;  // the tiled work list matches the stored order
    bool stage_timing = false;
    dpic::AdjointWs adj;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[DPIC_N_STAGE_TIMERS];
    size_t ev_used[DPIC_N_STAGE_TIMERS] = {0, 0, 0, 0};
    int64_t stage_launches[DPIC_N_STAGE_TIMERS] = {0, 0, 0, 0};
};

namespace dpic {

// ---- launchers (particles.hip)
hipError_t launch_element_consts(dpic_ctx* c);
hipError_t launch_element_consts_into(dpic_ctx* c, int NC, const double* elem_in, double* ec);
hipError_t launch_init_beam(dpic_ctx* c, const double* xi, const double* sig_dual /*[6][NC] host-marshalled*/);
// flags: PF_*; e_tau: element whose step size the kick uses; map: map block
// to apply (element_map_block) or nullptr without PF_MAP.
hipError_t launch_particles(dpic_ctx* c, int flags, int e_tau, const double* map, bool tiled);
const double* element_map_block(const dpic_ctx* c, int e, int slot);
hipError_t launch_canonical_state(dpic_ctx* c);  // st -> st2 in original order
hipError_t launch_zero(dpic_ctx* c, double* p, size_t n);

// ---- launchers (sort.hip)
bool sort_geometry(const dpic_ctx* c, int* tiles, int* nbins);
hipError_t launch_sort(dpic_ctx* c);  // also rebuilds the tiled work list

// ---- launchers (solver.hip)
hipError_t launch_green(dpic_ctx* c);
hipError_t launch_solve(dpic_ctx* c);
hipError_t launch_conv(dpic_ctx* c, double* in, const int nin[3], double* out, const int nout[3], int shift, int NC);
hipError_t launch_field(dpic_ctx* c);

// ---- launchers (moments.hip)
hipError_t launch_moments(dpic_ctx* c);

// ---- launchers (adjoint.hip)
hipError_t launch_adj_terminal(dpic_ctx* c, const double w[3]);
hipError_t launch_adj_step(dpic_ctx* c, int e, const double* st0, const double* E, bool space_charge);
hipError_t launch_adj_finish(dpic_ctx* c, int np);

}  // namespace dpic
