/*
 * dtwiss.h -- single-particle linear optics on one MI355X: Twiss parameters
 * of a line of drifts and hard-edge quadrupoles and their derivatives with
 * respect to lattice parameters (dual numbers, Sec. 2), and the paper's
 * matching example (Sec. 3): quadrupole strengths that carry given Twiss
 * parameters into target ones, minimised by BFGS using the derivatives.
 *
 * Twiss transport with the plane's transfer matrix m (Sec. 3):
 *   beta1 = m11^2 beta0 - 2 m11 m12 alpha0 + m12^2 gamma0,
 *   alpha1 = -m11 m21 beta0 + (m11 m22 + m12 m21) alpha0 - m12 m22 gamma0,
 *   gamma = (1 + alpha^2)/beta. Each element's matrix is its exact map over
 * its full length (the Sec. 4 quadrupole maps; k > 0 focuses x). With no
 * initial Twiss the line is taken as one periodic cell: cos mu =
 * (M11 + M22)/2, beta = M12 / sin mu, alpha = (M11 - M22)/(2 sin mu).
 * Matching objective (Sec. 3):
 *   f = (bx - bxt)^2/bxt^2 + (ax - axt)^2 + (by - byt)^2/byt^2 + (ay - ayt)^2.
 *
 * Lines are given like dpic_set_lattice (kind, L, k, L_param, k_param; no
 * step counts); parameter j carries tangent j (np <= 15). Conventions as in
 * dpic.h; the caller owns the device workspace.
 */
#ifndef DTWISS_H
#define DTWISS_H

#include <stddef.h>

#include "dpic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Device workspace bytes for evaluations of up to nb parameter vectors. */
int dtwiss_query_workspace(int nb, size_t* bytes);

/*
 * Evaluate nb parameter vectors p [nb][np] (host): twiss [nb][4][1+np]
 * (host: beta_x, alpha_x, beta_y, alpha_y with their derivatives) and, when
 * target [4] is given, f [nb][1+np] (host, may be NULL). twiss0 [4] (host)
 * gives the Twiss at the entry; NULL means the line's periodic solution.
 * Synchronous.
 */
int dtwiss_eval(void* workspace_dev, size_t bytes, void* hip_stream, int n_elem, const int* kind, const double* L,
                const double* k, const int* L_param, const int* k_param, int np, int nb, const double* p,
                const double* twiss0, const double* target, double* twiss, double* f);

/*
 * Minimise the matching objective over the np parameters from p0 [np] with
 * BFGS on the objective and its dual-number gradient (backtracking Armijo
 * line search, inverse-Hessian update), until f < tol or max_eval
 * evaluations. Writes p_out [np], f_out, the evaluation count and, if not
 * NULL, history [max_eval] (f after every evaluation). Synchronous.
 */
int dtwiss_match(void* workspace_dev, size_t bytes, void* hip_stream, int n_elem, const int* kind, const double* L,
                 const double* k, const int* L_param, const int* k_param, int np, const double* p0,
                 const double* twiss0, const double* target, double tol, int max_eval, double* p_out, double* f_out,
                 int* n_eval, double* history);

#ifdef __cplusplus
}
#endif
#endif /* DTWISS_H */
