// Host-side context of the dpic library and the launchers each kernel file
// exports to the C-ABI layer.
//
// A context holds B >= 1 independent settings (lattice parameter points and
// beams) that share the grid, the beam energy, the bunch charge and the
// lattice structure. Every stage launch covers all settings: particle
// storage is one array whose setting b occupies slots [off_b, off_b + n_b),
// off_b a multiple of SEG, and every grid array carries a leading setting
// index. With B = 1 the layout is the plain single-run layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/dpic.h"
#include "common.hpp"

namespace dpic {

constexpr int SEG = 1024;  // storage segment: settings start on segment boundaries

// Per-setting device record (the particle kernels take a setting's arrays
// from here, which keeps their bases out of the kernel arguments).
struct SettingDev {
    int64_t off;    // first storage slot (multiple of SEG)
    int64_t n;      // macroparticles
    int64_t delta;  // off minus the particles of earlier settings: packed row = slot - delta
    double q;       // charge per macroparticle, bunch charge / n
    const double* E;           // the setting's field [nz][ny][nx][3][NC]
    double* rho;               // its node charges [nz][ny][nx][NC]
    unsigned long long* cnt;   // its counters [CNT_N]
    const double* ec;          // its element constants [MAX_ELEM][EC_N][NC]
};

struct Workspace {
    double* st = nullptr;      // particle state [6][cap][NC]
    double* st2 = nullptr;     // second state buffer (sort target, read-back staging)
    int32_t* pid = nullptr;    // packed original row of each stored particle
    int32_t* pid2 = nullptr;
    uint32_t* key = nullptr;     // sort keys
    uint32_t* hist = nullptr;    // sort: [B][nbins] bin totals, zero between sorts
    uint32_t* bins = nullptr;    // sort: [B][nbins] first slots; [B][nbins] claim cursors
    int4* chunks = nullptr;      // tiled work list (tile, first, count, setting) of the order in st
    uint32_t* nchunks = nullptr;
    int4* chunks2 = nullptr;     // the work list of the order in st2 (written by a sort's counts)
    uint32_t* nchunks2 = nullptr;
    uint32_t* nitems = nullptr;  // [B] work items of each setting (batched sorts)
    SettingDev* set = nullptr;   // [B]
    int32_t* owner = nullptr;    // [cap / SEG] setting of each storage segment
    double* sig = nullptr;       // [B][6][NC] initial beam sizes as duals
    double* rho = nullptr;     // node charges [B][nz][ny][nx][NC]
    double* phi = nullptr;     // potential [B][nz+2][ny+2][nx+2][NC]
    double* E = nullptr;       // field [B][nz][ny][nx][3][NC]
    double2* buf0 = nullptr;   // FFT work arrays (B settings)
    double2* buf1 = nullptr;
    double* ghat = nullptr;    // transform of G on the (nx+1)(ny+1)(nz+1) octant (shared)
    double2* tw = nullptr;     // twiddles exp(-2 pi i m / M) for M = 2nx, 2ny, 2nz
    double* ec = nullptr;      // element constants [B][MAX_ELEM][EC_N][NC]
    double* elem_in = nullptr; // uploaded element L and k duals [B][MAX_ELEM][2][NC]
    unsigned long long* counters = nullptr;  // [B][CNT_N]
    double* mom_part = nullptr;  // moment partial sums [B][mom_blocks][MOM_N][NC]
    double* mom = nullptr;       // moments [B][MOM_N][NC]
    double* emit = nullptr;      // emittance [B][2][3][NC] (raw, centred)
    size_t bytes = 0;
};

constexpr int MOM_BLOCKS = 512;
constexpr int NUM_TILE_BINS_MAX = 4096;
constexpr int TILE_EDGE = 4;                             // cells per tile edge
// LDS tiles of a work item: its tile's cells plus a drift allowance of one
// cell on each side for the deposit tile; the E tile (three components per
// node) has it at most in x and y, where particles drift most between
// re-sorts (per step about 1/200 of a cell transversely, 1/1000 in z).
constexpr int TILE_HALO = 1;                             // drift allowance (cells)
constexpr int TILE_R = TILE_EDGE + 2 * TILE_HALO + 1;    // deposit tile nodes per dimension
constexpr int TILE_RZ_E = TILE_EDGE + 1;                 // E tile nodes in z
constexpr int TILE_CHUNK = 1024;                         // default particles per tiled work item
constexpr int64_t SORT_AUTO_CADENCE = 5;                 // automatic cadence: re-sort every 5 steps
constexpr int64_t SORT_AUTO_MIN_PARTICLES = 32768;       // ... from this many particles (all settings) up
constexpr int CHUNK_MIN = 128;                           // smallest work item (sizes the work list)
// One setting's work list: items of `chunk` particles while at least chunk x
// (resident workgroups) particles remain after an item's start, then halving
// sizes over GUIDE_LEVELS zones (never below CHUNK_MIN), so that the items
// that start last are short.
#ifndef DPIC_GUIDE_LEVELS
#define DPIC_GUIDE_LEVELS 2
#endif
constexpr int GUIDE_LEVELS = DPIC_GUIDE_LEVELS;
constexpr int CHUNK_MAX = 8192;
constexpr int SORT_PB = SEG;                             // particles per sort block
constexpr int MAX_BATCH = 4096;

inline int batch_of(const dpic_dims& d) { return d.nbatch > 0 ? d.nbatch : 1; }
// moment partial rows per setting
inline int mom_blocks_for(int B) {
    const int m = 4096 / B;
    return m > MOM_BLOCKS ? MOM_BLOCKS : (m < 1 ? 1 : m);
}

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

// One captured run of dpic_step(n) from step s0 and the host state it leaves.
struct GraphEntry {
    int64_t s0 = 0;
    int n = 0;
    bool swapped_in = false, chunks_in = false;
    bool adj = false;  // captured with the adjoint bound (checkpointed single steps)
    uint64_t layout = 0;
    hipGraphExec_t exec = nullptr;
    bool swapped_out = false, chunks_out = false;
};

// One captured adjoint sweep (terminal adjoint, segment replays and adjoint
// steps) of dpic_adjoint_backward after nf forward steps with weights w.
struct BwdGraph {
    int64_t nf = 0;
    double w[3] = {0.0, 0.0, 0.0};
    bool swapped = false, chunks = false;
    uint64_t layout = 0;
    hipGraphExec_t exec = nullptr;
};

}  // namespace dpic

struct dpic_ctx {
    dpic_dims dims{};
    int NC = 1;
    int ntan = 0;
    int B = 1;
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
    int np = 0;
    std::vector<double> p;     // [B][np]
    std::vector<double> seed;  // [np][ntan], shared by the settings
    // beam state
    bool beam_init = false;
    int64_t n = 0;                    // particles over all settings
    int64_t used = 0;                 // storage slots in use (off + n of the last setting)
    std::vector<int64_t> nb, off;     // per setting
    int64_t steps_done = 0;
    int64_t cur_step = 0;             // schedule step of the particle launch being enqueued
    bool swapped = false;             // ws.st holds the second state buffer
    // options
    int64_t sort_every = -1;  // re-sort cadence; -1 automatic (sort_cadence in capi.hip)
    int64_t chunk = dpic::TILE_CHUNK;  // particles per tiled work item
    int part_slots = 512;              // resident workgroups of the tiled particle kernel
    int64_t part_blocks = 0;           // workgroups of the tiled particle kernel (0: resident capacity)
    bool chunks_valid = false;  // the tiled work list matches the stored order
    bool keys_ready = false;    // ws.key holds every particle's tile key (written by the last particle launch)
    bool hist_clean = false;    // ws.hist is all zero (every sort's planning clears it)
    int stage_timing = 0;  // 0 off, 1 every stage, 2 the particle stage only
    bool use_graph = false;
    bool check_finite = false;  // dpic_step synchronises and reports non-finite state values
    bool deterministic = false; // fixed-order deposit, no re-sorting: bit-identical runs
    bool sorted_order = false;  // the stored order may come from a sort (not the packed original order)
    int cu_count = 0;
    int device = 0;  // the device current at dpic_create
    dpic::AdjointWs adj;
    // captured runs
    uint64_t layout_gen = 1;
    hipStream_t cap_stream = nullptr;
    std::vector<dpic::GraphEntry> graphs;
    std::vector<dpic::BwdGraph> bgraphs;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[DPIC_N_STAGE_TIMERS];
    size_t ev_used[DPIC_N_STAGE_TIMERS] = {0, 0, 0, 0};
    int64_t stage_launches[DPIC_N_STAGE_TIMERS] = {0, 0, 0, 0};
};

namespace dpic {

inline size_t grid_nodes(const dpic_ctx* c) { return (size_t)c->dims.nx * c->dims.ny * c->dims.nz; }
inline size_t ec_stride(const dpic_ctx* c) { return (size_t)DPIC_MAX_ELEMENTS * EC_N * c->NC; }
// offset of a map block (or of the step tau) inside one setting's element table
inline int ec_offset(const dpic_ctx* c, int e, int slot) { return (e * EC_N + slot) * c->NC; }

// ---- launchers (particles.hip)
hipError_t launch_element_consts(dpic_ctx* c);
// element constants of nb settings with NC channels from elem_in [nb][MAX_ELEM][2][NC]
hipError_t launch_element_consts_into(dpic_ctx* c, int NC, int nb, const double* elem_in, double* ec);
hipError_t launch_init_beam(dpic_ctx* c, const double* xi);
// flags: PF_*; e_tau: element whose step size the kick uses; map_off: map
// block to apply (ec_offset) when PF_MAP is set.
// write_keys: also write each particle's tile key (PF_KEYS); scatter: store
// each particle in its sorted slot of the second buffer (PF_SCATTER, after
// launch_sort_counts over the previous launch's keys).
hipError_t launch_particles(dpic_ctx* c, int flags, int e_tau, int map_off, bool tiled, bool write_keys = false,
                            bool scatter = false);
hipError_t launch_canonical_state(dpic_ctx* c);  // st -> st2 in packed original order
hipError_t launch_deposit_det(dpic_ctx* c);      // rho in a fixed summation order (deposit_det.hip)
hipError_t launch_unsort(dpic_ctx* c);           // st -> st2 (and pid -> pid2) in packed original order slots
int particle_resident_blocks(dpic_ctx* c);       // resident tiled-kernel workgroups on the device
hipError_t launch_zero(dpic_ctx* c, double* p, size_t n);

// ---- launchers (sort.hip)
bool sort_geometry(const dpic_ctx* c, int* tiles, int* nbins);
size_t max_chunks(const dpic_ctx* c);
hipError_t launch_sort(dpic_ctx* c);  // also rebuilds the tiled work list
// The sort in two parts around a particle launch that stores the state in
// sorted order itself: bin totals, first slots and the work list of the
// sorted order (into chunks2) from the stored keys, then (after that launch)
// the buffer swap.
hipError_t launch_sort_counts(dpic_ctx* c);
hipError_t launch_sort_finish(dpic_ctx* c, bool scattered);
// st, pid and the work list with their second buffers (a sort's swap)
inline void swap_sorted_buffers(Workspace& w) {
    std::swap(w.st, w.st2);
    std::swap(w.pid, w.pid2);
    std::swap(w.chunks, w.chunks2);
    std::swap(w.nchunks, w.nchunks2);
}

// ---- launchers (solver.hip)
hipError_t launch_green(dpic_ctx* c);
hipError_t launch_solve(dpic_ctx* c);
// nb settings of real [z][y][x][NC] windows, back to back
hipError_t launch_conv(dpic_ctx* c, double* in, const int nin[3], double* out, const int nout[3], int shift, int NC,
                       int nb);
hipError_t launch_field(dpic_ctx* c);

// ---- launchers (moments.hip)
hipError_t launch_moments(dpic_ctx* c);

// ---- launchers (adjoint.hip)
hipError_t launch_adj_terminal(dpic_ctx* c, const double w[3]);
hipError_t launch_adj_step(dpic_ctx* c, int e, const double* st0, const double* E, bool space_charge);
hipError_t launch_adj_finish(dpic_ctx* c, int np);

}  // namespace dpic
