/*
 * CPU oracle for time-vectorized backward- and forward-Euler integration.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the library.  Shares no code
 * with the HIP library.  All arithmetic is IEEE double.
 *
 * Layouts (all row-major, series-major):
 *   y0      [B][n]
 *   times   uniform: [N+1] shared by all series;
 *           ragged:  the time points of series b at times[offsets[b] .. offsets[b+1]-1]
 *   offsets NULL (uniform) or point offsets [B+1]; series b has
 *           N_b = offsets[b+1] - offsets[b] - 1 >= 0 steps
 *   params  per series [B][P], or one shared [P] when params_shared != 0
 *   y_out   uniform: [B][N+1][n]; ragged: [offsets[B]][n]; y_out at a series'
 *           first point is y0
 *   g       dL/dy in the layout of y_out
 *   dLdp    [B][P], or [P] when params_shared
 *   dLdy0   [B][n]
 *
 * Models (parameter vectors):
 *   ORACLE_LINEAR     h = A y,  p = A [n][n]
 *   ORACLE_VANDERPOL  n = 2, h = (y2, mu (1 - y1^2) y2 - y1), p = (mu)
 *   ORACLE_ROBERTSON  n = 3, rate constants 0.04 s1, 3e7 s2, 1e4 s3, p = (s1, s2, s3)
 *   ORACLE_MLP        h = W3 tanh(W2 tanh(W1 y + b1) + b2) + b3 with hidden width H,
 *                     p = W1[H][n], b1[H], W2[H][H], b2[H], W3[n][H], b3[n]
 *   ORACLE_CHABOCHE   Chaboche viscoplasticity with nu = n - 2 backstresses, state
 *                     (sigma, K, X_1..X_nu), p = (E, n, eta, sigma0, K_inf, tau,
 *                     C_1..C_nu, gamma_1..gamma_nu, edot_a, T) (Section 5.1.1)
 *   ORACLE_NEURON     nu = n / 4 coupled neurons, state (V, m, h, n) per neuron,
 *                     p = 15 per neuron (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf,
 *                     tau_m, h_inf, tau_h, n_inf, tau_n, g_C, T), then I_a (Section 5.1.1)
 *   ORACLE_MDS        mass-damper-spring chain of nu = n / 2 units, state (d_1, v_1, ..,
 *                     d_nu, v_nu), p = (K_1..K_nu, C_1..C_nu, M_1..M_nu, f_a, T) (Section 5.1.1)
 *   ORACLE_FNODE      forced neural ODE h = tanh(W3 tanh(W2 tanh(W1 (y, f(t)) + b1) + b2) + b3),
 *                     p = (W1[n+1][n+1], b1[n+1], W2[n+1][n+1], b2[n+1], W3[n][n+1], b3[n],
 *                     f_a, T), f(t) = f_a sin(2 pi t / T) (Section 5.1.1)
 * State size n <= 64.
 */
#ifndef TVI_ORACLE_H
#define TVI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_LINEAR = 0, ORACLE_VANDERPOL = 1, ORACLE_ROBERTSON = 2, ORACLE_MLP = 3, ORACLE_CHABOCHE = 4,
       ORACLE_NEURON = 5, ORACLE_MDS = 6, ORACLE_FNODE = 7 };
enum { ORACLE_OK = 0, ORACLE_NOT_CONVERGED = 1, ORACLE_SINGULAR = 2, ORACLE_NONFINITE = 3 };

int oracle_param_count(int kind, int n, int hidden);

/* Dense LU with partial pivoting; overwrites A and b; x returned in b. 0 = ok, 1 = singular. */
int oracle_lu_solve(int n, double *A, double *b);

/* f = h(y,t;p) and, when J is not NULL, J = dh/dy (row-major). */
int oracle_rhs(int kind, int n, int hidden, const double *y, double t, const double *p,
               double *f, double *J);

/* gp += (dh/dp)^T w */
int oracle_vjp_p(int kind, int n, int hidden, const double *y, double t, const double *p,
                 const double *w, double *gp);

/* Sequential backward Euler with one dense Newton solve per step.  A step is
 * converged when ||r||_2 <= tol_a or ||r||_2 <= tol_r ||r0||_2.  A step that
 * is not converged after max_newton corrections (NOT_CONVERGED), meets a zero
 * or non-finite pivot (SINGULAR) or a non-finite residual (NONFINITE) stops
 * its series: status[b] gets the code and the states from that step on are
 * NaN.  iters[B] (may be NULL) gets the total number of Newton corrections.
 * Returns 0, or -1 on invalid arguments. */
int oracle_forward(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                   const double *times, const double *y0, const double *params, int params_shared,
                   double tol_a, double tol_r, int max_newton, int threads,
                   double *y_out, int32_t *status, int32_t *iters);

/* Discrete adjoint of the map computed by oracle_forward, given its trajectory y. */
int oracle_adjoint(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                   const double *times, const double *y, const double *params, int params_shared,
                   const double *g, int threads, double *dLdp, double *dLdy0, int32_t *status);

/* Sequential forward Euler: y_k = y_{k-1} + (t_k - t_{k-1}) h(y_{k-1}, t_{k-1}; p).
 * A non-finite state stops its series (NONFINITE; NaN from that step on). */
int oracle_forward_euler(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                         const double *times, const double *y0, const double *params, int params_shared,
                         int threads, double *y_out, int32_t *status);

/* Discrete adjoint of the map computed by oracle_forward_euler, given its trajectory y. */
int oracle_forward_euler_adjoint(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                                 const double *times, const double *y, const double *params, int params_shared,
                                 const double *g, int threads, double *dLdp, double *dLdy0, int32_t *status);

#ifdef __cplusplus
}
#endif
#endif
