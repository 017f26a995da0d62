/*
 * dpic.h -- C ABI of the forward-mode differentiable 3D particle-in-cell
 * space-charge step on one AMD MI355X (gfx950).
 *
 * The method (arXiv 2511.21839, Sec. 4): macroparticles are advanced by the
 * second-order split-operator map M1(tau/2) M2(tau) M1(tau/2), where M1 is the
 * exact external map of a drift or hard-edge quadrupole and M2 the
 * space-charge kick computed from a grid potential. Every particle coordinate,
 * grid charge, potential and field value is a first-order dual number
 * F = (f, f_x1, ..., f_xn) (Sec. 2), so one run yields the result and its
 * derivatives with respect to n parameters (lattice lengths and strengths,
 * initial beam sizes).
 *
 * Conventions
 *  - Every function returns an int: DPIC_OK (0) or a negative DPIC_E* code.
 *    No function throws or aborts across the ABI. dpic_last_error() gives a
 *    message for the last failing call on a context.
 *  - Pointers named *_dev are device pointers; all others are host pointers,
 *    read or written only during the call.
 *  - The caller owns all device memory: one workspace buffer, sized by
 *    dpic_query_workspace(), bound at dpic_create() and never freed by the
 *    library. The library allocates no device memory.
 *  - All GPU work is enqueued on the stream bound at dpic_create() (a
 *    hipStream_t passed as void*; NULL means the default stream). Calls that
 *    return data to the host synchronise that stream; the others are
 *    asynchronous.
 *  - A context is not thread-safe; use one context per stream.
 *  - Dual numbers are stored with a channel stride NC = 1 (ntan = 0),
 *    8 (ntan <= 7) or 16 (ntan <= 15); channel 0 is the value, channel
 *    1 + t the derivative with respect to tangent t, the rest zero.
 *  - Units: SI (m, V, C); momenta are normalised, px/p0, py/p0 and
 *    delta = (p - p0)/p0; z is the lab-frame distance from the bunch centre.
 *  - Batches: a context runs B = dims.nbatch independent settings at once
 *    (each its own lattice parameter values, particle count and initial beam;
 *    grid, beam energy, bunch charge and lattice structure shared). Every
 *    stage is one launch over all settings. Setting b's particles take
 *    storage slots from a multiple of 1024, so the capacity must cover
 *    sum over b < B-1 of roundup(n_b, 1024), plus n_{B-1}. Outputs that are
 *    per setting carry a leading [B] index; with B = 1 it is omitted from
 *    the layouts below.
 */
#ifndef DPIC_H
#define DPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPIC_OK 0
#define DPIC_EINVAL (-1)       /* bad argument or size */
#define DPIC_ESTATE (-2)       /* call out of order (e.g. step before init) */
#define DPIC_EHIP (-3)         /* a HIP runtime call failed */
#define DPIC_ENONFINITE (-4)   /* a non-finite value was found */
#define DPIC_EUNSUPPORTED (-5) /* ntan > 15 or a grid size other than 8/16/32/64 */

#define DPIC_MAX_ELEMENTS 64
#define DPIC_MAX_PARAMS 64

typedef struct dpic_ctx dpic_ctx;

/* Problem dimensions, fixed for the lifetime of a context. */
typedef struct dpic_dims {
    int64_t n_particles; /* capacity: storage slots for all settings         */
    int32_t ntan;        /* number of tangents (derivative channels), 0..15  */
    int32_t nx, ny, nz;  /* grid nodes per dimension, each in {8,16,32,64}   */
    int32_t flags;       /* reserved, must be 0                              */
    int32_t nbatch;      /* settings run together, 1..4096 (0 means 1)       */
} dpic_dims;

/* Library version as major*10000 + minor*100 + patch. */
int dpic_version(void);

/* Bytes of device workspace a context with these dimensions needs. */
int dpic_query_workspace(const dpic_dims* dims, size_t* bytes);

/*
 * Bind caller-owned device memory (at least the queried size, 256-byte
 * aligned) and a HIP stream to a new context. The context owns host metadata
 * only; dpic_destroy() frees that and never the workspace.
 */
int dpic_create(const dpic_dims* dims, void* workspace_dev, size_t workspace_bytes,
                void* hip_stream, dpic_ctx** out);
int dpic_destroy(dpic_ctx* ctx);

/* Copy the message of the last failing call (NUL-terminated, truncated). */
int dpic_last_error(const dpic_ctx* ctx, char* buf, size_t len);

/*
 * Reference particle and bunch: kinetic and rest energy in eV, particle
 * charge in units of e, total bunch charge in C (0 switches space charge
 * off). gamma0 = 1 + T / mc^2. The space-charge kick (Sec. 4, map M2) is read
 * in 3D as Delta(px/p0) = tau q E_x / (m c^2 beta0^2 gamma0^2) (same for y)
 * and Delta(delta) = tau q E_z / (m c^2 beta0^2 gamma0), E the rest-frame
 * field; for a long beam this is the paper's perveance kick.
 */
int dpic_set_beam(dpic_ctx* ctx, double kinetic_eV, double rest_eV, double charge_e,
                  double bunch_charge_C);

/*
 * Fixed grid box [lo, hi] per dimension (never differentiated). Nodes sit at
 * lo + i h, h = (hi - lo) / (n - 1). A particle is inside iff
 * 0 <= (u - lo)/h < n - 1 in every dimension; outside particles deposit
 * nothing, feel no kick and are counted. Builds the transform of the
 * open-boundary Green's function on the doubled grid; needs dpic_set_beam()
 * first (the rest-frame kernel depends on gamma0).
 */
int dpic_set_grid(dpic_ctx* ctx, const double lo[3], const double hi[3]);

/*
 * One lattice period of n_elem elements, repeated n_periods times.
 * kind[e]: 0 drift, 1 hard-edge quadrupole (Sec. 4 maps; k > 0 focuses x).
 * n_steps[e]: integration steps per element (tau = L / n_steps, Sec. 4).
 * L[e], k[e]: values used when L_param[e] / k_param[e] is -1; otherwise the
 * element takes parameter L_param[e] / k_param[e] of dpic_set_params(),
 * shared by every period.
 */
int dpic_set_lattice(dpic_ctx* ctx, int n_elem, const int* kind, const int* n_steps,
                     const double* L, const double* k, const int* L_param,
                     const int* k_param, int n_periods);

/*
 * Parameter values p[np] and their derivative seeds seed[np][ntan] (row j is
 * the derivative of p[j] with respect to each tangent, Sec. 2 seeding
 * X_i = (x_i, 0, .., 1, .., 0)); seed == NULL means identity (p[j] carries
 * tangent j for j < ntan). Recomputes the per-element dual step sizes and
 * half-step maps on the device. Every setting of a batch takes these values.
 */
int dpic_set_params(dpic_ctx* ctx, int np, const double* p, const double* seed);

/*
 * Per-setting parameter values p[nb][np] (nb must equal the context's B) with
 * the seeds seed[np][ntan] (or NULL = identity) shared by all settings.
 */
int dpic_set_params_batch(dpic_ctx* ctx, int nb, int np, const double* p, const double* seed);

/*
 * Initial beam zeta_j = sigma_j xi_j for n <= capacity particles.
 * xi_dev: device array [n][6] of standard normals (caller draws them).
 * sigma[6]: rms sizes of x, px/p0, y, py/p0, z, delta.
 * sigma_seed[6][ntan] or NULL: derivative of sigma_j per tangent, so the
 * initial tangents are sigma_seed[j][t] * xi_j.
 * Resets the step counter and the diagnostic counters. Needs B = 1.
 */
int dpic_init_beam(dpic_ctx* ctx, int64_t n, const double* xi_dev, const double sigma[6],
                   const double* sigma_seed);

/*
 * Initial beams of all nb = B settings: setting b has n[b] >= 0 particles,
 * its normals are rows [sum_{b'<b} n[b'], + n[b]) of the packed device array
 * xi_dev [sum n][6], its sizes sigma[b][6]; sigma_seed[6][ntan] (or NULL) is
 * shared. The bunch charge is split over each setting's own n[b]. Fails with
 * DPIC_EINVAL when the settings do not fit the capacity (see Batches).
 */
int dpic_init_beam_batch(dpic_ctx* ctx, int nb, const int64_t* n, const double* xi_dev, const double* sigma,
                         const double* sigma_seed);

/*
 * Advance n steps along the lattice schedule (asynchronous). Each step is
 * M1(tau/2), deposit, solve, field, gather + kick, M1(tau/2). Fails with
 * DPIC_EINVAL past the end of the schedule.
 */
int dpic_step(dpic_ctx* ctx, int n);

/*
 * Raw dual moments over each setting's particles, host out[B][3][5][1+ntan]: planes
 * (x,px), (y,py), (z,delta); moments <u^2>, <u p>, <p^2>, <u>, <p> with 1/N
 * sums (Sec. 4). Synchronises the stream.
 */
int dpic_read_moments(dpic_ctx* ctx, double* out);

/*
 * Emittances as duals, host out[B][3][1+ntan]: eps = sqrt(<u^2><p^2> - <u p>^2)
 * with raw moments (Sec. 4) when centred == 0, central moments otherwise.
 * A setting without particles reports zeros. Synchronises the stream.
 */
int dpic_read_emittance(dpic_ctx* ctx, int centred, double* out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the emittances
 * of dpic_read_emittance, written to caller device memory
 * out_dev[B][3][1+ntan] (raw when centred == 0, central moments otherwise;
 * zeros for an empty setting) and enqueued asynchronously on the bound
 * stream: no host transfer and no synchronisation. The moment partial sums,
 * moments and emittance duals go to a static device array of the library
 * (4 MiB per device, held until the process ends) instead of the context
 * workspace; nothing is allocated. Contexts that need more than 4 MiB
 * (B * NC * (15 * blocks + 21) doubles, blocks <= 512 partial-sum blocks per
 * setting, at most 4096 / B) get DPIC_EINVAL. Every call on one GPU shares
 * that array: calls that overlap on one GPU (other streams, other threads)
 * race. No non-finite check (that needs the host; dpic_read_emittance does it).
 */
int dpic_read_emittance_noalloc(dpic_ctx* ctx, int centred, double* out_dev);

/*
 * Particle state in the original particle order, host out[n][6][1+ntan]
 * (settings back to back in the packed order of dpic_init_beam_batch).
 * Synchronises the stream.
 */
int dpic_read_particles(dpic_ctx* ctx, double* out);

/*
 * Diagnostics, host: particle-steps found outside the box, steps done, and
 * max |x|, |y|, |z| seen at deposit time (extent may be NULL); summed and
 * maximised over the settings. Synchronises the stream.
 */
int dpic_counters(dpic_ctx* ctx, int64_t* out_of_box, int64_t* steps_done, double* extent);
/* Out-of-box particle-steps per setting, host out_of_box[B]. Synchronises. */
int dpic_batch_counters(dpic_ctx* ctx, int64_t* out_of_box);

/* Stage-level access for parity checks and diagnostics ------------------ */
#define DPIC_GRID_RHO 0 /* node charges  [B][nz][ny][nx][1+ntan]         */
#define DPIC_GRID_PHI 1 /* potential     [B][nz+2][ny+2][nx+2][1+ntan], node i at i+1 */
#define DPIC_GRID_E 2   /* rest-frame E  [B][nz][ny][nx][3][1+ntan]      */

#define DPIC_STAGE_DEPOSIT 0 /* clear rho, deposit the current particles    */
#define DPIC_STAGE_SOLVE 1   /* rho -> phi (consumes rho: it is left zeroed) */
#define DPIC_STAGE_FIELD 2   /* phi -> E                                    */

/* Run one stage on the current state (asynchronous). */
int dpic_stage(dpic_ctx* ctx, int stage);
/* Copy a grid array to / from host memory in the layouts above (synchronous). */
int dpic_read_grid(dpic_ctx* ctx, int which, double* out);
int dpic_write_grid(dpic_ctx* ctx, int which, const double* in);

/*
 * Checkpoint: bytes needed, then copy the particle state, particle order,
 * per-setting particle counts and step counter to / from caller device
 * memory (synchronous). The buffer ends with the particle state in storage
 * order, [6][capacity][NC] doubles (coordinate, storage slot, channel); the
 * header and the particle order come before it.
 */
int dpic_state_bytes(const dpic_ctx* ctx, size_t* bytes);
int dpic_save_state(dpic_ctx* ctx, void* dev_buf);
int dpic_load_state(dpic_ctx* ctx, const void* dev_buf);

/*
 * Options:
 *  DPIC_OPT_SORT_EVERY = re-sort particles by grid tile every k steps, for
 *    the tiled particle kernel (k > 0); 0 = never (storage-order kernel,
 *    deposit by global atomics); -1 = automatic, the default: every 5 steps
 *    from 32768 particles (all settings together) up, or while the adjoint
 *    is bound, else never (with fewer particles the storage-order kernel
 *    is faster). Other values are EINVAL; dpic_get_option returns -1 while
 *    automatic;
 *  DPIC_OPT_STAGE_TIMING = 1 records HIP events around every stage launch of
 *    dpic_step, 2 around the particle stage only (fewer event records in the
 *    stream: each leaves the GPU idle for a few microseconds), 3 around the
 *    plain particle launches only (not the launch that also writes the sort
 *    keys nor the one that stores the particles in sorted order); read with
 *    dpic_stage_times; other values are EINVAL;
 *  DPIC_OPT_CHUNK = particles per work item of the tiled particle kernel
 *    (a multiple of 64 in 128..8192, default 1024). With one setting the
 *    items that start once fewer than chunk x (the kernel's resident
 *    workgroups) particles remain hold chunk / 2, so that the last items of
 *    a launch are short; batches use chunk throughout;
 *  DPIC_OPT_PART_BLOCKS = workgroups of the persistent tiled particle kernel
 *    (0 = four times the device's resident capacity for it, the default;
 *    never more than the work list can hold);
 *  DPIC_OPT_GRAPH = 1 captures each distinct dpic_step(n) call (same start
 *    step, same n, same batch layout) in a HIP graph on first use and replays
 *    it afterwards, and likewise the adjoint sweep of dpic_adjoint_backward
 *    (same number of forward steps, same weights); ignored while stage
 *    timing is on. Replays see new parameter values and beams (device
 *    memory); changing the beam, grid, lattice, particle counts or the
 *    adjoint binding, or loading a state, drops the captured graphs. The
 *    stream bound at dpic_create may be the null stream: capture runs on a
 *    stream the context creates;
 *  DPIC_OPT_CHECK_FINITE = 1 makes dpic_step synchronise at its end and
 *    return DPIC_ENONFINITE when any particle launch since dpic_init_beam
 *    stored a NaN or Inf in the state of any setting (the message names the
 *    first such step); every particle launch records that step in device
 *    memory whatever the option, and dpic_read_moments and
 *    dpic_read_emittance return DPIC_ENONFINITE from it too (after writing
 *    their output). Default 0: dpic_step stays asynchronous;
 *  DPIC_OPT_DETERMINISTIC = 1 makes the forward steps bit-reproducible: the
 *    same context inputs give bit-identical states, moments and emittances on
 *    every run, eager or graph-replayed. The charge deposit (Sec. 4,
 *    cloud-in-cell assignment of rho and its derivative arrays) then runs
 *    as a sorted segmented reduction with a fixed summation order instead of
 *    floating-point atomics, and particles are never re-sorted (the sort
 *    cadence is ignored and the tiled kernels are not used). Switching the
 *    mode on, or loading a state while it is on, moves the stored particles
 *    back into their original order (a re-sort's order depends on the timing
 *    of atomics). Results agree with the default mode to rounding (the
 *    summation order differs); the step costs several times the default's.
 *    The adjoint sweep of dpic_adjoint_backward still accumulates with
 *    atomics, and dpic_autotune returns DPIC_ESTATE in this mode.
 *    DPIC_STAGE_DEPOSIT follows the mode but counts no out-of-box particles
 *    in it. Default 0.
 */
#define DPIC_OPT_SORT_EVERY 1
#define DPIC_OPT_STAGE_TIMING 2
#define DPIC_OPT_CHUNK 3
#define DPIC_OPT_PART_BLOCKS 4
#define DPIC_OPT_GRAPH 5
#define DPIC_OPT_CHECK_FINITE 6
#define DPIC_OPT_DETERMINISTIC 7
int dpic_set_option(dpic_ctx* ctx, int option, int64_t value);
int dpic_get_option(const dpic_ctx* ctx, int option, int64_t* value);

/*
 * Autotuner: times trial_steps steps from the current state for candidate
 * sort cadences (0, 5, 10, 12, 20, 40 steps), then work-item sizes, then
 * persistent grid sizes (coordinate search in that order), restores the
 * state and the counters after every trial, and keeps the fastest setting;
 * a candidate replaces the current one only when its trial is at least 2%
 * faster. scratch_dev: caller device memory of at least
 * dpic_state_bytes(). best[3] (host, may be NULL) receives
 * {sort_every, chunk, part_blocks}; ms_best the time of the winning trial.
 * Needs space charge on and no adjoint bound; synchronises.
 */
int dpic_autotune(dpic_ctx* ctx, void* scratch_dev, size_t scratch_bytes, int trial_steps, int64_t* best,
                  double* ms_best);

/*
 * Accumulated stage times since the last call, host ms[DPIC_N_STAGE_TIMERS]
 * and launch counts; synchronises. Order: particle push/deposit, solve,
 * field, sort.
 */
#define DPIC_N_STAGE_TIMERS 4
int dpic_stage_times(dpic_ctx* ctx, double* ms, int64_t* launches);

/*
 * Reverse mode: gradients of J = w0 eps_x + w1 eps_y + w2 eps_z (raw
 * emittances of the final beam, Sec. 4) with respect to the parameters of
 * dpic_set_params (at most 15) and the six initial beam sizes, at a cost that
 * does not grow with their number. Works on value-only contexts (ntan = 0)
 * with one setting (B = 1; otherwise DPIC_EUNSUPPORTED).
 *
 * dpic_adjoint_query: device bytes for a run of up to n_steps steps with a
 * state checkpoint every checkpoint_every steps (checkpoints, one segment of
 * replayed states and fields, adjoint arrays).
 * dpic_adjoint_bind: attach that caller-owned workspace (256-byte aligned);
 * call before dpic_init_beam, which then keeps a copy of xi. While bound,
 * dpic_step runs unfused steps, stores a checkpoint every checkpoint_every
 * steps and does not re-sort particles after the first sort.
 * dpic_adjoint_backward: after the forward dpic_step calls, sweep the steps
 * in reverse (replaying each segment from its checkpoint) and write
 * grad_params[np] and grad_sigma[6] (host, either may be NULL). The particle
 * state is consumed: call dpic_init_beam before stepping again.
 * Synchronises the stream.
 */
int dpic_adjoint_query(const dpic_dims* dims, int n_steps, int checkpoint_every, size_t* bytes);
int dpic_adjoint_bind(dpic_ctx* ctx, void* adjoint_workspace_dev, size_t bytes, int n_steps, int checkpoint_every);
int dpic_adjoint_backward(dpic_ctx* ctx, const double weights[3], double* grad_params, double* grad_sigma);

#ifdef __cplusplus
}
#endif
#endif /* DPIC_H */
