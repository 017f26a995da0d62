/*
 * dpic2d.h -- C ABI of the paper's own PIC instance on one MI355X: a 2D beam
 * in a rectangular perfectly conducting pipe (Sec. 4), every coordinate,
 * grid charge, potential and field value a first-order dual number.
 *
 * Per step: M1(tau/2) (drift / quadrupole maps of (x, px) and (y, py)),
 * bilinear deposit, the sine-series Poisson solve with phi = 0 on the pipe
 * walls, central-difference field, bilinear gather and kick, M1(tau/2).
 *
 *  - Pipe [0, a] x [0, b] with nx x ny cells; nodes (i a/nx, j b/ny),
 *    i = 0..nx, j = 0..ny. Beam coordinates are measured from the pipe
 *    centre. A particle is inside iff 0 <= (x + a/2) nx/a < nx (same in y);
 *    others deposit nothing, feel no kick and are counted.
 *  - A macroparticle carries lambda / n of the line charge lambda = I /
 *    (beta0 c); node densities are node charges per length / (h_x h_y).
 *  - Solve: rho^lm = 4/(nx ny) sum_ij rho_ij sin(l pi i/nx) sin(m pi j/ny)
 *    over the interior nodes, phi^lm = rho^lm / (eps0 (alpha_l^2 +
 *    beta_m^2)), alpha_l = l pi / a, beta_m = m pi / b, and phi_ij =
 *    sum_lm phi^lm sin sin (Sec. 4 sine expansion and its solution).
 *  - Field: central differences on every node; beyond a wall the sine
 *    series is odd (phi_{-1} = -phi_1).
 *  - Kick: Delta(px/p0) = tau q E_x / (m c^2 beta0^2 gamma0^3), likewise y:
 *    for a uniform round beam of radius r0 this is the paper's x'' =
 *    K x / r0^2 with K = q I / (2 pi eps0 p0 v0^2 gamma0^2).
 *
 * Conventions as in dpic.h (return codes, device/host pointers, one caller-
 * owned workspace, one stream, channel 0 the value and 1 + t tangent t).
 */
#ifndef DPIC2D_H
#define DPIC2D_H

#include <stddef.h>
#include <stdint.h>

#include "dpic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpic2d_ctx dpic2d_ctx;

typedef struct dpic2d_dims {
    int64_t n_particles; /* capacity                                     */
    int32_t ntan;        /* tangents, 0..15                              */
    int32_t nx, ny;      /* cells per dimension, 4..256                  */
    int32_t flags;       /* reserved, must be 0                          */
} dpic2d_dims;

#define DPIC2D_GRID_RHO 0 /* node densities [nx+1][ny+1][1+ntan]          */
#define DPIC2D_GRID_PHI 1 /* potential      [nx+1][ny+1][1+ntan]          */
#define DPIC2D_GRID_E 2   /* field          [nx+1][ny+1][2][1+ntan]       */

int dpic2d_query_workspace(const dpic2d_dims* dims, size_t* bytes);
int dpic2d_create(const dpic2d_dims* dims, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                  dpic2d_ctx** out);
int dpic2d_destroy(dpic2d_ctx* ctx);
int dpic2d_last_error(const dpic2d_ctx* ctx, char* buf, size_t len);

/* Reference particle and beam current (A; 0 switches space charge off). */
int dpic2d_set_beam(dpic2d_ctx* ctx, double kinetic_eV, double rest_eV, double charge_e, double current_A);
/* Pipe widths a, b (m). Builds the sine tables. */
int dpic2d_set_pipe(dpic2d_ctx* ctx, double a, double b);
/* Lattice and parameters: as dpic_set_lattice / dpic_set_params. */
int dpic2d_set_lattice(dpic2d_ctx* ctx, int n_elem, const int* kind, const int* n_steps, const double* L,
                       const double* k, const int* L_param, const int* k_param, int n_periods);
int dpic2d_set_params(dpic2d_ctx* ctx, int np, const double* p, const double* seed);
/* zeta_j = sigma_j xi_j for x, px, y, py: xi_dev [n][4] device, sigma[4],
 * sigma_seed [4][ntan] host or NULL. Resets the step and loss counters. */
int dpic2d_init_beam(dpic2d_ctx* ctx, int64_t n, const double* xi_dev, const double sigma[4],
                     const double* sigma_seed);
/* Advance n steps (asynchronous). */
int dpic2d_step(dpic2d_ctx* ctx, int n);
/* Raw emittances as duals, host out[2][1+ntan] (x, y). Synchronous. */
int dpic2d_read_emittance(dpic2d_ctx* ctx, double* out);
/* Particles in the original order, host out[n][4][1+ntan]. Synchronous. */
int dpic2d_read_particles(dpic2d_ctx* ctx, double* out);
/* Stage access for parity: 0 clear + deposit, 1 solve, 2 field (asynchronous). */
int dpic2d_stage(dpic2d_ctx* ctx, int stage);
int dpic2d_read_grid(dpic2d_ctx* ctx, int which, double* out);
int dpic2d_write_grid(dpic2d_ctx* ctx, int which, const double* in);
/* Particle-steps found outside the pipe at deposit, and steps done. Synchronous. */
int dpic2d_counters(dpic2d_ctx* ctx, int64_t* lost, int64_t* steps_done);

#ifdef __cplusplus
}
#endif
#endif /* DPIC2D_H */
