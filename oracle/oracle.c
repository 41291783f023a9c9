/*
 * CPU oracle for time-vectorized backward-Euler integration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP
 * library.
 *
 * What it computes is the plain definition of the result the chunked method
 * reaches (Section 2.2, Eq. backward-euler): for every series, the sequence
 * y_1..y_N with
 *
 *     y_k - y_{k-1} - (t_k - t_{k-1}) h(y_k, t_k; p) = 0,
 *
 * found one step at a time by Newton's method started from the previous
 * converged state (Section 2.2, the zero-order-hold starting guess), with a
 * dense LU solve of the discrete Jacobian I - dt j (Section 2.2) at every
 * iteration.  The gradient is the discrete adjoint of that computed map
 * (Appendix A: the same scheme for the forward and the backward problem).
 *
 * The explicit scheme of Section 2.2 (Eq. forward-euler) is here too, as its
 * plain definition: y_k = y_{k-1} + (t_k - t_{k-1}) h(y_{k-1}, t_{k-1}; p),
 * one step after another, with the discrete adjoint of that map.
 *
 * Everything is IEEE double, no fast-math.  Series are independent
 * (Section 2.1) and are distributed over a pthread pool, longest first.
 */
#define _DEFAULT_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NMAX 64
#define HMAX 512

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (ties go to the lowest row index).         */
/* Solves A x = b in place for an n x n row-major A; returns 0 on success,   */
/* 1 when a pivot is zero or not finite.                                     */
/* ------------------------------------------------------------------------ */
static int lu_solve(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = fabs(A[r * n + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0) || !isfinite(best)) return 1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        double inv = 1.0 / A[c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double l = A[r * n + c] * inv;
            if (l == 0.0) continue;
            for (int k = c + 1; k < n; ++k) A[r * n + k] -= l * A[c * n + k];
            b[r] -= l * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

int oracle_lu_solve(int n, double *A, double *b) { return lu_solve(n, A, b); }

/* ------------------------------------------------------------------------ */
/* Model right-hand sides h(y, t; p), their state Jacobians j = dh/dy and     */
/* the parameter vector-Jacobian products (dh/dp)^T w.                        */
/* ------------------------------------------------------------------------ */

int oracle_param_count(int kind, int n, int hidden)
{
    switch (kind) {
    case ORACLE_LINEAR:    return n * n;
    case ORACLE_VANDERPOL: return 1;
    case ORACLE_ROBERTSON: return 3;
    case ORACLE_MLP:       return hidden * n + hidden + hidden * hidden + hidden + n * hidden + n;
    case ORACLE_CHABOCHE:  return n >= 3 ? 8 + 2 * (n - 2) : -1;
    case ORACLE_NEURON:    return (n >= 4 && n % 4 == 0) ? 15 * (n / 4) + 1 : -1;
    case ORACLE_MDS:       return (n >= 2 && n % 2 == 0) ? 3 * (n / 2) + 2 : -1;
    case ORACLE_FNODE:     return 2 * (n + 1) * (n + 1) + 2 * (n + 1) + n * (n + 1) + n + 2;
    default:               return -1;
    }
}

/* MLP forward: a1 = tanh(W1 y + b1), a2 = tanh(W2 a1 + b2), f = W3 a2 + b3. */
static void mlp_forward(int n, int H, const double *th, const double *y,
                        double *a1, double *a2, double *f)
{
    const double *W1 = th, *b1 = W1 + H * n, *W2 = b1 + H, *b2 = W2 + H * H,
                 *W3 = b2 + H, *b3 = W3 + n * H;
    for (int i = 0; i < H; ++i) {
        double s = b1[i];
        for (int k = 0; k < n; ++k) s += W1[i * n + k] * y[k];
        a1[i] = tanh(s);
    }
    for (int i = 0; i < H; ++i) {
        double s = b2[i];
        for (int k = 0; k < H; ++k) s += W2[i * H + k] * a1[k];
        a2[i] = tanh(s);
    }
    for (int i = 0; i < n; ++i) {
        double s = b3[i];
        for (int k = 0; k < H; ++k) s += W3[i * H + k] * a2[k];
        f[i] = s;
    }
}

/* Chaboche viscoplasticity (Section 5.1.1), n_unit = n - 2 backstresses.
 * State (sigma, K, X_1..X_nu); parameters
 *   p = (E, n, eta, sigma0, K_inf, tau, C_1..C_nu, gamma_1..gamma_nu, edot_a, T).
 * With s = sigma - sum X and a = (|s| - K - sigma0) / eta, the plastic rate is
 * ep = <a>^n sign(s) (<> the Macaulay bracket), |ep| = <a>^n, and
 *   dsigma/dt = E (edot(t) - ep),  dK/dt = tau (K_inf - K) |ep|,
 *   dX_i/dt = 2/3 C_i ep - gamma_i X_i |ep|,  edot(t) = edot_a sin(2 pi t / T).
 * The isotropic hardening grows with the plastic rate (the standard form; the
 * printed dK/dt lacks the |ep| factor, under which the paper's parameter table
 * never leaves the elastic range). */
typedef struct {
    double s, sg, a, pa, dpa, ep, edot;
} chaboche_flow;

static chaboche_flow chaboche_eval(int nu, const double *y, double t, const double *p)
{
    chaboche_flow c;
    double sx = 0.0;
    for (int i = 0; i < nu; ++i) sx += y[2 + i];
    c.s = y[0] - sx;
    c.sg = c.s > 0.0 ? 1.0 : (c.s < 0.0 ? -1.0 : 0.0);
    c.a = (fabs(c.s) - y[1] - p[3]) / p[2];
    c.pa = c.a > 0.0 ? pow(c.a, p[1]) : 0.0;                      /* <a>^n              */
    c.dpa = c.a > 0.0 ? p[1] * pow(c.a, p[1] - 1.0) / p[2] : 0.0; /* d<a>^n / d|s|      */
    c.ep = c.pa * c.sg;
    c.edot = p[6 + 2 * nu] * sin(2.0 * M_PI * t / p[7 + 2 * nu]);
    return c;
}

/* Coupled neurons (Section 5.1.1), n_unit = n / 4, state (V_i, m_i, h_i, n_i) per
 * neuron; parameters per neuron (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf, tau_m,
 * h_inf, tau_h, n_inf, tau_n, g_C, T), then the current amplitude I_a. */
enum { NR_C, NR_GNA, NR_ENA, NR_GK, NR_EK, NR_GL, NR_EL, NR_MINF, NR_TM, NR_HINF, NR_TH, NR_NINF, NR_TN,
       NR_GC, NR_T, NR_PER_UNIT };

/* Mass-damper-spring chain (Section 5.1.1) of nu = n / 2 units, state
 * (d_1, v_1, ..., d_nu, v_nu); p = (K_1..K_nu, C_1..C_nu, M_1..M_nu, f_a, T).
 * Unit i is mass M_i joined to its neighbour on the fixed side, i + 1, by the
 * spring K_i and the damper C_i; position nu + 1 is the wall (d = v = 0) and
 * the periodic force acts on the first mass:
 *   dd_i/dt = v_i,
 *   dv_i/dt = [K_i (d_{i+1} - d_i) + C_i (v_{i+1} - v_i)
 *             - K_{i-1} (d_i - d_{i-1}) - C_{i-1} (v_i - v_{i-1})] / M_i + f_i(t),
 * with no i - 1 terms for the first unit, f_1 = f_a sin(2 pi t / T), f_i = 0
 * otherwise.  The spring and damper forces restore (the printed signs would
 * drive the chain away from rest), every force on a mass is divided by that
 * mass, and the printed forcing lacks its time argument. */
static void mds_accel_row(int nu, int i, const double *y, const double *p, double *acc)
{
    const double *K = p, *C = p + nu, *M = p + 2 * nu;
    const double d = y[2 * i], v = y[2 * i + 1];
    const double dn = (i + 1 < nu) ? y[2 * i + 2] : 0.0, vn = (i + 1 < nu) ? y[2 * i + 3] : 0.0;
    double a = K[i] * (dn - d) + C[i] * (vn - v);
    if (i > 0) a -= K[i - 1] * (d - y[2 * i - 2]) + C[i - 1] * (v - y[2 * i - 1]);
    *acc = a / M[i];
}

/* Forced neural ODE (Section 5.1.1) of size n: x = (y, f(t)),
 * a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), h = tanh(W3 a2 + b3), with
 * W1, W2 (n+1) x (n+1), W3 n x (n+1), f(t) = f_a sin(2 pi t / T);
 * p = (W1, b1, W2, b2, W3, b3, f_a, T), matrices row-major. */
typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    double fa, T;
} fnode_params;

static fnode_params fnode_unpack(int n, const double *p)
{
    const int m = n + 1;
    fnode_params q;
    q.W1 = p; q.b1 = q.W1 + m * m; q.W2 = q.b1 + m; q.b2 = q.W2 + m * m; q.W3 = q.b2 + m; q.b3 = q.W3 + n * m;
    q.fa = q.b3[n]; q.T = q.b3[n + 1];
    return q;
}

static void fnode_forward(int n, const fnode_params *q, const double *y, double t, double *x, double *a1,
                          double *a2, double *a3)
{
    const int m = n + 1;
    for (int k = 0; k < n; ++k) x[k] = y[k];
    x[n] = q->fa * sin(2.0 * M_PI * t / q->T);
    for (int i = 0; i < m; ++i) {
        double s = q->b1[i];
        for (int k = 0; k < m; ++k) s += q->W1[i * m + k] * x[k];
        a1[i] = tanh(s);
    }
    for (int i = 0; i < m; ++i) {
        double s = q->b2[i];
        for (int k = 0; k < m; ++k) s += q->W2[i * m + k] * a1[k];
        a2[i] = tanh(s);
    }
    for (int i = 0; i < n; ++i) {
        double s = q->b3[i];
        for (int k = 0; k < m; ++k) s += q->W3[i * m + k] * a2[k];
        a3[i] = tanh(s);
    }
}

/* f = h(y,t;p); if J != NULL also J = dh/dy (row-major n x n). */
static void rhs(int kind, int n, int H, const double *y, double t, const double *p,
                double *f, double *J)
{
    switch (kind) {
    case ORACLE_LINEAR:
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += p[i * n + k] * y[k];
            f[i] = s;
        }
        if (J) memcpy(J, p, sizeof(double) * n * n);
        break;
    case ORACLE_VANDERPOL: {
        double mu = p[0];
        f[0] = y[1];
        f[1] = mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
        if (J) {
            J[0] = 0.0;                          J[1] = 1.0;
            J[2] = -2.0 * mu * y[0] * y[1] - 1.0; J[3] = mu * (1.0 - y[0] * y[0]);
        }
        break;
    }
    case ORACLE_ROBERTSON: {
        double k1 = 0.04 * p[0], k2 = 3.0e7 * p[1], k3 = 1.0e4 * p[2];
        f[0] = -k1 * y[0] + k3 * y[1] * y[2];
        f[1] = k1 * y[0] - k3 * y[1] * y[2] - k2 * y[1] * y[1];
        f[2] = k2 * y[1] * y[1];
        if (J) {
            J[0] = -k1; J[1] = k3 * y[2];                     J[2] = k3 * y[1];
            J[3] = k1;  J[4] = -k3 * y[2] - 2.0 * k2 * y[1];  J[5] = -k3 * y[1];
            J[6] = 0.0; J[7] = 2.0 * k2 * y[1];               J[8] = 0.0;
        }
        break;
    }
    case ORACLE_MLP: {
        double a1[HMAX], a2[HMAX];
        mlp_forward(n, H, p, y, a1, a2, f);
        if (J) {
            /* J = W3 diag(1-a2^2) W2 diag(1-a1^2) W1, built column by column
               as the Jacobian-vector product with each unit vector. */
            const double *W1 = p, *W2 = W1 + H * n + H, *W3 = W2 + H * H + H;
            double u1[HMAX], u2[HMAX];
            for (int c = 0; c < n; ++c) {
                for (int i = 0; i < H; ++i) u1[i] = (1.0 - a1[i] * a1[i]) * W1[i * n + c];
                for (int i = 0; i < H; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < H; ++k) s += W2[i * H + k] * u1[k];
                    u2[i] = (1.0 - a2[i] * a2[i]) * s;
                }
                for (int i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < H; ++k) s += W3[i * H + k] * u2[k];
                    J[i * n + c] = s;
                }
            }
        }
        break;
    }
    case ORACLE_CHABOCHE: {
        const int nu = n - 2;
        const double E = p[0], tau = p[5], Kinf = p[4];
        const double *C = p + 6, *gam = p + 6 + nu;
        const chaboche_flow c = chaboche_eval(nu, y, t, p);
        f[0] = E * (c.edot - c.ep);
        f[1] = tau * (Kinf - y[1]) * c.pa;
        for (int i = 0; i < nu; ++i) f[2 + i] = 2.0 / 3.0 * C[i] * c.ep - gam[i] * y[2 + i] * c.pa;
        if (J) {
            /* d ep and d|ep| with respect to sigma, K and each X_j */
            double dep[NMAX], dab[NMAX];
            dep[0] = c.dpa * c.sg * c.sg; dab[0] = c.dpa * c.sg;
            dep[1] = -c.dpa * c.sg;       dab[1] = -c.dpa;
            for (int j = 0; j < nu; ++j) { dep[2 + j] = -c.dpa * c.sg * c.sg; dab[2 + j] = -c.dpa * c.sg; }
            for (int k = 0; k < n; ++k) {
                J[0 * n + k] = -E * dep[k];
                J[1 * n + k] = tau * (Kinf - y[1]) * dab[k] - ((k == 1) ? tau * c.pa : 0.0);
                for (int i = 0; i < nu; ++i)
                    J[(2 + i) * n + k] = 2.0 / 3.0 * C[i] * dep[k] - gam[i] * y[2 + i] * dab[k]
                                         - ((k == 2 + i) ? gam[i] * c.pa : 0.0);
            }
        }
        break;
    }
    case ORACLE_MDS: {
        const int nu = n / 2;
        const double *K = p, *C = p + nu, *M = p + 2 * nu;
        for (int i = 0; i < nu; ++i) {
            double a;
            mds_accel_row(nu, i, y, p, &a);
            f[2 * i] = y[2 * i + 1];
            f[2 * i + 1] = a + (i == 0 ? p[3 * nu] * sin(2.0 * M_PI * t / p[3 * nu + 1]) : 0.0);
        }
        if (J) {
            memset(J, 0, sizeof(double) * n * n);
            for (int i = 0; i < nu; ++i) {
                double *r = J + (2 * i + 1) * n;
                J[(2 * i) * n + 2 * i + 1] = 1.0;
                r[2 * i] = -K[i] / M[i];
                r[2 * i + 1] = -C[i] / M[i];
                if (i + 1 < nu) { r[2 * i + 2] = K[i] / M[i]; r[2 * i + 3] = C[i] / M[i]; }
                if (i > 0) {
                    r[2 * i] -= K[i - 1] / M[i];
                    r[2 * i + 1] -= C[i - 1] / M[i];
                    r[2 * i - 2] = K[i - 1] / M[i];
                    r[2 * i - 1] = C[i - 1] / M[i];
                }
            }
        }
        break;
    }
    case ORACLE_FNODE: {
        const int m = n + 1;
        const fnode_params q = fnode_unpack(n, p);
        double x[NMAX + 1], a1[NMAX + 1], a2[NMAX + 1];
        fnode_forward(n, &q, y, t, x, a1, a2, f);
        if (J) {
            /* J = diag(1 - h^2) W3 diag(1 - a2^2) W2 diag(1 - a1^2) W1[:, 0:n],
               column by column as Jacobian-vector products with unit vectors */
            double u1[NMAX + 1], u2[NMAX + 1];
            for (int c = 0; c < n; ++c) {
                for (int i = 0; i < m; ++i) u1[i] = (1.0 - a1[i] * a1[i]) * q.W1[i * m + c];
                for (int i = 0; i < m; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < m; ++k) s += q.W2[i * m + k] * u1[k];
                    u2[i] = (1.0 - a2[i] * a2[i]) * s;
                }
                for (int i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int k = 0; k < m; ++k) s += q.W3[i * m + k] * u2[k];
                    J[i * n + c] = (1.0 - f[i] * f[i]) * s;
                }
            }
        }
        break;
    }
    case ORACLE_NEURON: {
        const int nu = n / 4;
        const double Ia = p[NR_PER_UNIT * nu];
        if (J) memset(J, 0, sizeof(double) * n * n);
        for (int i = 0; i < nu; ++i) {
            const double *q = p + NR_PER_UNIT * i;
            const double V = y[4 * i], m = y[4 * i + 1], hh = y[4 * i + 2], nn = y[4 * i + 3];
            double cpl = 0.0;
            for (int j = 0; j < nu; ++j) cpl += V - y[4 * j];
            const double I = Ia * sin(2.0 * M_PI * t / q[NR_T]);
            const double m3 = m * m * m, n4 = nn * nn * nn * nn;
            const double F = -q[NR_GNA] * m3 * hh * (V - q[NR_ENA]) - q[NR_GK] * n4 * (V - q[NR_EK])
                             - q[NR_GL] * (V - q[NR_EL]) + I + q[NR_GC] * cpl;
            f[4 * i] = F / q[NR_C];
            f[4 * i + 1] = (q[NR_MINF] - m) / q[NR_TM];
            f[4 * i + 2] = (q[NR_HINF] - hh) / q[NR_TH];
            f[4 * i + 3] = (q[NR_NINF] - nn) / q[NR_TN];
            if (J) {
                double *r = J + 4 * i * n;
                for (int j = 0; j < nu; ++j) r[4 * j] = (j == i) ? 0.0 : -q[NR_GC] / q[NR_C];
                r[4 * i] = (-q[NR_GNA] * m3 * hh - q[NR_GK] * n4 - q[NR_GL] + q[NR_GC] * (nu - 1)) / q[NR_C];
                r[4 * i + 1] = -3.0 * q[NR_GNA] * m * m * hh * (V - q[NR_ENA]) / q[NR_C];
                r[4 * i + 2] = -q[NR_GNA] * m3 * (V - q[NR_ENA]) / q[NR_C];
                r[4 * i + 3] = -4.0 * q[NR_GK] * nn * nn * nn * (V - q[NR_EK]) / q[NR_C];
                J[(4 * i + 1) * n + 4 * i + 1] = -1.0 / q[NR_TM];
                J[(4 * i + 2) * n + 4 * i + 2] = -1.0 / q[NR_TH];
                J[(4 * i + 3) * n + 4 * i + 3] = -1.0 / q[NR_TN];
            }
        }
        break;
    }
    }
}

/* gp += (dh/dp (y,t;p))^T w */
static void vjp_p(int kind, int n, int H, const double *y, double t, const double *p,
                  const double *w, double *gp)
{
    switch (kind) {
    case ORACLE_CHABOCHE: {
        const int nu = n - 2;
        const double E = p[0], Kinf = p[4], tau = p[5], eda = p[6 + 2 * nu], T = p[7 + 2 * nu];
        const double *C = p + 6, *gam = p + 6 + nu;
        const chaboche_flow c = chaboche_eval(nu, y, t, p);
        /* the weights carried by ep and by |ep| = <a>^n */
        double g_ep = -E * w[0], g_pa = w[1] * tau * (Kinf - y[1]);
        for (int i = 0; i < nu; ++i) {
            g_ep += 2.0 / 3.0 * C[i] * w[2 + i];
            g_pa -= gam[i] * y[2 + i] * w[2 + i];
        }
        const double g_a = g_ep * c.sg + g_pa; /* weight of <a>^n itself */
        if (c.a > 0.0) {
            gp[1] += g_a * c.pa * log(c.a);         /* d<a>^n / dn      */
            gp[2] += g_a * (-p[1] * c.pa / p[2]);  /* d<a>^n / deta    */
            gp[3] += g_a * (-c.dpa);               /* d<a>^n / dsigma0 */
        }
        gp[0] += w[0] * (c.edot - c.ep);
        gp[4] += w[1] * tau * c.pa;
        gp[5] += w[1] * (Kinf - y[1]) * c.pa;
        for (int i = 0; i < nu; ++i) {
            gp[6 + i] += w[2 + i] * 2.0 / 3.0 * c.ep;
            gp[6 + nu + i] -= w[2 + i] * y[2 + i] * c.pa;
        }
        const double ph = 2.0 * M_PI * t / T;
        gp[6 + 2 * nu] += w[0] * E * sin(ph);
        gp[7 + 2 * nu] += w[0] * E * eda * cos(ph) * (-ph / T);
        return;
    }
    case ORACLE_MDS: {
        /* h is linear in K, C, 1/M and f_a: dv_i/dt = a_i + f_i with a_i the
           spring and damper acceleration of mass i */
        const int nu = n / 2;
        const double *M = p + 2 * nu;
        double *gK = gp, *gC = gp + nu, *gM = gp + 2 * nu;
        for (int i = 0; i < nu; ++i) {
            const double wi = w[2 * i + 1] / M[i];
            const double d = y[2 * i], v = y[2 * i + 1];
            const double dn = (i + 1 < nu) ? y[2 * i + 2] : 0.0, vn = (i + 1 < nu) ? y[2 * i + 3] : 0.0;
            gK[i] += wi * (dn - d);
            gC[i] += wi * (vn - v);
            if (i > 0) {
                gK[i - 1] -= wi * (d - y[2 * i - 2]);
                gC[i - 1] -= wi * (v - y[2 * i - 1]);
            }
            double a;
            mds_accel_row(nu, i, y, p, &a);
            gM[i] -= w[2 * i + 1] * a / M[i];
        }
        const double ph = 2.0 * M_PI * t / p[3 * nu + 1];
        gp[3 * nu] += w[1] * sin(ph);
        gp[3 * nu + 1] += w[1] * p[3 * nu] * cos(ph) * (-ph / p[3 * nu + 1]);
        return;
    }
    case ORACLE_FNODE: {
        /* back-propagation of w through the three layers, then into f_a and T
           through the forcing input */
        const int m = n + 1;
        const fnode_params q = fnode_unpack(n, p);
        double x[NMAX + 1], a1[NMAX + 1], a2[NMAX + 1], a3[NMAX], d3[NMAX], d2[NMAX + 1], d1[NMAX + 1];
        fnode_forward(n, &q, y, t, x, a1, a2, a3);
        double *gW1 = gp, *gb1 = gW1 + m * m, *gW2 = gb1 + m, *gb2 = gW2 + m * m, *gW3 = gb2 + m,
               *gb3 = gW3 + n * m;
        for (int i = 0; i < n; ++i) d3[i] = w[i] * (1.0 - a3[i] * a3[i]);
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < m; ++k) gW3[i * m + k] += d3[i] * a2[k];
            gb3[i] += d3[i];
        }
        for (int k = 0; k < m; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += q.W3[i * m + k] * d3[i];
            d2[k] = s * (1.0 - a2[k] * a2[k]);
        }
        for (int i = 0; i < m; ++i) {
            for (int k = 0; k < m; ++k) gW2[i * m + k] += d2[i] * a1[k];
            gb2[i] += d2[i];
        }
        for (int k = 0; k < m; ++k) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += q.W2[i * m + k] * d2[i];
            d1[k] = s * (1.0 - a1[k] * a1[k]);
        }
        double gx = 0.0; /* dL/d(forcing input) */
        for (int i = 0; i < m; ++i) {
            for (int k = 0; k < m; ++k) gW1[i * m + k] += d1[i] * x[k];
            gb1[i] += d1[i];
            gx += q.W1[i * m + n] * d1[i];
        }
        const double ph = 2.0 * M_PI * t / q.T;
        gb3[n] += gx * sin(ph);
        gb3[n + 1] += gx * q.fa * cos(ph) * (-ph / q.T);
        return;
    }
    case ORACLE_NEURON: {
        const int nu = n / 4;
        const double Ia = p[NR_PER_UNIT * nu];
        for (int i = 0; i < nu; ++i) {
            const double *q = p + NR_PER_UNIT * i;
            double *g = gp + NR_PER_UNIT * i;
            const double V = y[4 * i], m = y[4 * i + 1], hh = y[4 * i + 2], nn = y[4 * i + 3];
            double cpl = 0.0;
            for (int j = 0; j < nu; ++j) cpl += V - y[4 * j];
            const double ph = 2.0 * M_PI * t / q[NR_T];
            const double I = Ia * sin(ph);
            const double m3 = m * m * m, n4 = nn * nn * nn * nn;
            const double F = -q[NR_GNA] * m3 * hh * (V - q[NR_ENA]) - q[NR_GK] * n4 * (V - q[NR_EK])
                             - q[NR_GL] * (V - q[NR_EL]) + I + q[NR_GC] * cpl;
            const double wv = w[4 * i] / q[NR_C];
            g[NR_C] -= wv * F / q[NR_C];
            g[NR_GNA] -= wv * m3 * hh * (V - q[NR_ENA]);
            g[NR_ENA] += wv * q[NR_GNA] * m3 * hh;
            g[NR_GK] -= wv * n4 * (V - q[NR_EK]);
            g[NR_EK] += wv * q[NR_GK] * n4;
            g[NR_GL] -= wv * (V - q[NR_EL]);
            g[NR_EL] += wv * q[NR_GL];
            g[NR_GC] += wv * cpl;
            g[NR_T] += wv * Ia * cos(ph) * (-ph / q[NR_T]);
            gp[NR_PER_UNIT * nu] += wv * sin(ph);
            g[NR_MINF] += w[4 * i + 1] / q[NR_TM];
            g[NR_TM] -= w[4 * i + 1] * (q[NR_MINF] - m) / (q[NR_TM] * q[NR_TM]);
            g[NR_HINF] += w[4 * i + 2] / q[NR_TH];
            g[NR_TH] -= w[4 * i + 2] * (q[NR_HINF] - hh) / (q[NR_TH] * q[NR_TH]);
            g[NR_NINF] += w[4 * i + 3] / q[NR_TN];
            g[NR_TN] -= w[4 * i + 3] * (q[NR_NINF] - nn) / (q[NR_TN] * q[NR_TN]);
        }
        return;
    }
    default: break;
    }
    (void)t;
    switch (kind) {
    case ORACLE_LINEAR: /* h_i = sum_k A_ik y_k  ->  dL/dA_ik = w_i y_k */
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) gp[i * n + k] += w[i] * y[k];
        break;
    case ORACLE_VANDERPOL: /* dh/dmu = (0, (1-y1^2) y2) */
        gp[0] += w[1] * (1.0 - y[0] * y[0]) * y[1];
        break;
    case ORACLE_ROBERTSON: {
        double d1 = 0.04 * (-w[0] * y[0] + w[1] * y[0]);
        double d2 = 3.0e7 * (-w[1] * y[1] * y[1] + w[2] * y[1] * y[1]);
        double d3 = 1.0e4 * (w[0] * y[1] * y[2] - w[1] * y[1] * y[2]);
        gp[0] += d1; gp[1] += d2; gp[2] += d3;
        break;
    }
    case ORACLE_MLP: {
        /* Back-propagation of w through the network. */
        double a1[HMAX], a2[HMAX], d2[HMAX], d1[HMAX], f[NMAX];
        mlp_forward(n, H, p, y, a1, a2, f);
        const double *W2 = p + H * n + H, *W3 = W2 + H * H + H;
        double *gW1 = gp, *gb1 = gW1 + H * n, *gW2 = gb1 + H, *gb2 = gW2 + H * H,
               *gW3 = gb2 + H, *gb3 = gW3 + n * H;
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < H; ++k) gW3[i * H + k] += w[i] * a2[k];
            gb3[i] += w[i];
        }
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += W3[i * H + k] * w[i];
            d2[k] = s * (1.0 - a2[k] * a2[k]);
        }
        for (int i = 0; i < H; ++i) {
            for (int k = 0; k < H; ++k) gW2[i * H + k] += d2[i] * a1[k];
            gb2[i] += d2[i];
        }
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += W2[i * H + k] * d2[i];
            d1[k] = s * (1.0 - a1[k] * a1[k]);
        }
        for (int i = 0; i < H; ++i) {
            for (int k = 0; k < n; ++k) gW1[i * n + k] += d1[i] * y[k];
            gb1[i] += d1[i];
        }
        break;
    }
    }
}

int oracle_rhs(int kind, int n, int hidden, const double *y, double t, const double *p,
               double *f, double *J)
{
    if (n < 1 || n > NMAX || oracle_param_count(kind, n, hidden) < 0) return -1;
    rhs(kind, n, hidden, y, t, p, f, J);
    return 0;
}

int oracle_vjp_p(int kind, int n, int hidden, const double *y, double t, const double *p,
                 const double *w, double *gp)
{
    if (n < 1 || n > NMAX || oracle_param_count(kind, n, hidden) < 0) return -1;
    vjp_p(kind, n, hidden, y, t, p, w, gp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Problem description shared by the forward and adjoint drivers.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind, n, H, P, params_shared;
    int explicit_scheme; /* 0: backward Euler, 1: forward Euler */
    int64_t B, N;
    const int64_t *offsets; /* point offsets [B+1] or NULL (uniform: N+1 points each) */
    const double *times, *y0, *params;
    double tol_a, tol_r;
    int max_newton;
    /* forward outputs */
    double *y;
    int32_t *status, *iters;
    /* adjoint inputs/outputs */
    const double *g;
    double *dLdp, *dLdy0;
    /* scheduling */
    const int64_t *order;
    int64_t next;
    pthread_mutex_t lock;
} problem_t;

static int64_t first_point(const problem_t *pb, int64_t b)
{
    return pb->offsets ? pb->offsets[b] : b * (pb->N + 1);
}
static int64_t n_steps(const problem_t *pb, int64_t b)
{
    return pb->offsets ? pb->offsets[b + 1] - pb->offsets[b] - 1 : pb->N;
}
static const double *series_times(const problem_t *pb, int64_t b)
{
    return pb->offsets ? pb->times + pb->offsets[b] : pb->times;
}
static const double *series_params(const problem_t *pb, int64_t b)
{
    return pb->params_shared ? pb->params : pb->params + b * pb->P;
}

/* Sequential backward Euler for one series (Section 2.2). */
static void forward_series(problem_t *pb, int64_t b)
{
    const int n = pb->n, H = pb->H, kind = pb->kind;
    const int64_t Nb = n_steps(pb, b);
    const double *t = series_times(pb, b), *p = series_params(pb, b);
    double *Y = pb->y + first_point(pb, b) * n;
    double yprev[NMAX], yk[NMAX], f[NMAX], r[NMAX], J[NMAX * NMAX];
    int32_t status = ORACLE_OK, total = 0;

    for (int i = 0; i < n; ++i) Y[i] = yprev[i] = pb->y0[b * n + i];
    for (int64_t k = 1; k <= Nb && status == ORACLE_OK; ++k) {
        const double dt = t[k] - t[k - 1];
        memcpy(yk, yprev, sizeof(double) * n);        /* start from y_{k-1} */
        double nu0 = 0.0;
        for (int it = 0;; ++it) {
            rhs(kind, n, H, yk, t[k], p, f, NULL);
            double nu = 0.0;
            for (int i = 0; i < n; ++i) {
                r[i] = yk[i] - yprev[i] - dt * f[i];
                nu += r[i] * r[i];
            }
            nu = sqrt(nu);
            if (!isfinite(nu)) { status = ORACLE_NONFINITE; break; }
            if (it == 0) nu0 = nu;
            if (nu <= pb->tol_a || nu <= pb->tol_r * nu0) break;
            if (it == pb->max_newton) { status = ORACLE_NOT_CONVERGED; break; }
            /* discrete Jacobian I - dt j and the Newton correction */
            rhs(kind, n, H, yk, t[k], p, f, J);
            for (int i = 0; i < n; ++i) {
                for (int c = 0; c < n; ++c) J[i * n + c] = (i == c ? 1.0 : 0.0) - dt * J[i * n + c];
                r[i] = -r[i];
            }
            if (lu_solve(n, J, r)) { status = ORACLE_SINGULAR; break; }
            for (int i = 0; i < n; ++i) yk[i] += r[i];
            ++total;
        }
        if (status != ORACLE_OK) {
            /* a failed series stops: this and every later state is NaN */
            for (int64_t q = k * n; q <= Nb * n + n - 1; ++q) Y[q] = NAN;
            break;
        }
        memcpy(yprev, yk, sizeof(double) * n);
        memcpy(Y + k * n, yk, sizeof(double) * n);
    }
    pb->status[b] = status;
    if (pb->iters) pb->iters[b] = total;
}

/* Discrete adjoint of the backward-Euler map for one series (Appendix A):
 *   (I - dt_k j_k)^T lam_k = lam_{k+1} + g_k,   k = N..1,  lam_{N+1} = 0,
 *   dL/dp += dt_k (dh/dp (y_k))^T lam_k,        dL/dy0 = g_0 + lam_1,
 * with j_k evaluated at the converged y_k. */
static void adjoint_series(problem_t *pb, int64_t b, double *gp)
{
    const int n = pb->n, H = pb->H, kind = pb->kind;
    const int64_t Nb = n_steps(pb, b), p0 = first_point(pb, b);
    const double *t = series_times(pb, b), *p = series_params(pb, b);
    const double *Y = pb->y + p0 * n, *G = pb->g + p0 * n;
    double lam[NMAX], f[NMAX], J[NMAX * NMAX], Dt[NMAX * NMAX], w[NMAX];
    int32_t status = ORACLE_OK;

    memset(lam, 0, sizeof(lam));
    for (int64_t k = Nb; k >= 1; --k) {
        const double dt = t[k] - t[k - 1];
        rhs(kind, n, H, Y + k * n, t[k], p, f, J);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < n; ++c) Dt[c * n + i] = (i == c ? 1.0 : 0.0) - dt * J[i * n + c];
        for (int i = 0; i < n; ++i) lam[i] += G[k * n + i];
        if (lu_solve(n, Dt, lam)) { status = ORACLE_SINGULAR; break; }
        for (int i = 0; i < n; ++i) w[i] = dt * lam[i];
        vjp_p(kind, n, H, Y + k * n, t[k], p, w, gp);
    }
    for (int i = 0; i < n; ++i) pb->dLdy0[b * n + i] = G[i] + lam[i];
    pb->status[b] = status;
}

/* Sequential forward Euler for one series (Section 2.2, Eq. forward-euler):
 *   y_k = y_{k-1} + dt_k h(y_{k-1}, t_{k-1}; p).
 * A non-finite state stops the series (NONFINITE; NaN from that step on). */
static void forward_euler_series(problem_t *pb, int64_t b)
{
    const int n = pb->n, H = pb->H, kind = pb->kind;
    const int64_t Nb = n_steps(pb, b);
    const double *t = series_times(pb, b), *p = series_params(pb, b);
    double *Y = pb->y + first_point(pb, b) * n;
    double f[NMAX];
    int32_t status = ORACLE_OK;

    for (int i = 0; i < n; ++i) Y[i] = pb->y0[b * n + i];
    for (int64_t k = 1; k <= Nb; ++k) {
        const double dt = t[k] - t[k - 1];
        const double *yp = Y + (k - 1) * n;
        rhs(kind, n, H, yp, t[k - 1], p, f, NULL);
        int finite = 1;
        for (int i = 0; i < n; ++i) {
            Y[k * n + i] = yp[i] + dt * f[i];
            finite &= isfinite(Y[k * n + i]) ? 1 : 0;
        }
        if (!finite) {
            status = ORACLE_NONFINITE;
            for (int64_t q = k * n; q <= Nb * n + n - 1; ++q) Y[q] = NAN;
            break;
        }
    }
    pb->status[b] = status;
    if (pb->iters) pb->iters[b] = 0;
}

/* Discrete adjoint of the forward-Euler map for one series.  With the
 * constraints c_k = y_k - y_{k-1} - dt_k h(y_{k-1}) = 0, stationarity of
 * L - sum_k lam_k^T c_k in y_k gives
 *   lam_k = g_k + (I + dt_{k+1} j(y_k))^T lam_{k+1},   k = N..1,  lam_{N+1} = 0,
 *   dL/dp = sum_k dt_k (dh/dp (y_{k-1}))^T lam_k,
 *   dL/dy0 = g_0 + (I + dt_1 j(y_0))^T lam_1. */
static void adjoint_forward_euler_series(problem_t *pb, int64_t b, double *gp)
{
    const int n = pb->n, H = pb->H, kind = pb->kind;
    const int64_t Nb = n_steps(pb, b), p0 = first_point(pb, b);
    const double *t = series_times(pb, b), *p = series_params(pb, b);
    const double *Y = pb->y + p0 * n, *G = pb->g + p0 * n;
    double lam[NMAX], nxt[NMAX], f[NMAX], J[NMAX * NMAX], w[NMAX];

    memset(lam, 0, sizeof(lam)); /* lam_{N+1} */
    for (int64_t k = Nb; k >= 0; --k) {
        /* nxt = (I + dt_{k+1} j(y_k))^T lam_{k+1}; zero at k = N */
        for (int i = 0; i < n; ++i) nxt[i] = 0.0;
        if (k < Nb) {
            const double dt1 = t[k + 1] - t[k];
            rhs(kind, n, H, Y + k * n, t[k], p, f, J);
            for (int i = 0; i < n; ++i) {
                double s = lam[i];
                for (int r = 0; r < n; ++r) s += dt1 * J[r * n + i] * lam[r];
                nxt[i] = s;
            }
        }
        for (int i = 0; i < n; ++i) lam[i] = G[k * n + i] + nxt[i];
        if (k == 0) break; /* lam now holds dL/dy0 */
        const double dt = t[k] - t[k - 1];
        for (int i = 0; i < n; ++i) w[i] = dt * lam[i];
        vjp_p(kind, n, H, Y + (k - 1) * n, t[k - 1], p, w, gp);
    }
    for (int i = 0; i < n; ++i) pb->dLdy0[b * n + i] = lam[i];
    pb->status[b] = ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Thread pool over series, longest series first.                           */
/* ------------------------------------------------------------------------ */
typedef struct { problem_t *pb; int adjoint; double *gp_series; } job_t;

static void *worker(void *arg)
{
    job_t *job = arg;
    problem_t *pb = job->pb;
    for (;;) {
        pthread_mutex_lock(&pb->lock);
        int64_t i = pb->next++;
        pthread_mutex_unlock(&pb->lock);
        if (i >= pb->B) break;
        int64_t b = pb->order[i];
        if (job->adjoint) {
            if (pb->explicit_scheme) adjoint_forward_euler_series(pb, b, job->gp_series + b * pb->P);
            else adjoint_series(pb, b, job->gp_series + b * pb->P);
        } else {
            if (pb->explicit_scheme) forward_euler_series(pb, b);
            else forward_series(pb, b);
        }
    }
    return NULL;
}

static const problem_t *sort_ctx;
static int cmp_len(const void *a, const void *b)
{
    int64_t la = n_steps(sort_ctx, *(const int64_t *)a), lb = n_steps(sort_ctx, *(const int64_t *)b);
    if (la != lb) return la > lb ? -1 : 1;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    return ia < ib ? -1 : (ia > ib);
}

static pthread_mutex_t sort_lock = PTHREAD_MUTEX_INITIALIZER;

static int run_pool(problem_t *pb, int threads, int adjoint, double *gp_series)
{
    int64_t *order = malloc(sizeof(int64_t) * (pb->B > 0 ? pb->B : 1));
    if (!order) return -3;
    for (int64_t b = 0; b < pb->B; ++b) order[b] = b;
    pthread_mutex_lock(&sort_lock);
    sort_ctx = pb;
    qsort(order, (size_t)pb->B, sizeof(int64_t), cmp_len);
    pthread_mutex_unlock(&sort_lock);
    pb->order = order;
    pb->next = 0;
    pthread_mutex_init(&pb->lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > pb->B) threads = pb->B > 0 ? (int)pb->B : 1;
    pthread_t *tid = malloc(sizeof(pthread_t) * threads);
    job_t job = { pb, adjoint, gp_series };
    for (int i = 1; i < threads; ++i) pthread_create(&tid[i], NULL, worker, &job);
    worker(&job);
    for (int i = 1; i < threads; ++i) pthread_join(tid[i], NULL);
    free(tid);
    pthread_mutex_destroy(&pb->lock);
    free(order);
    return 0;
}

static int validate(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets)
{
    if (n < 1 || n > NMAX || B < 0) return -1;
    if (oracle_param_count(kind, n, hidden) < 0) return -1;
    if (kind == ORACLE_VANDERPOL && n != 2) return -1;
    if (kind == ORACLE_ROBERTSON && n != 3) return -1;
    if (kind == ORACLE_CHABOCHE && n < 3) return -1;
    if (kind == ORACLE_NEURON && (n < 4 || n % 4)) return -1;
    if (kind == ORACLE_MLP && (hidden < 1 || hidden > HMAX)) return -1;
    if (!offsets && N < 0) return -1;
    if (offsets)
        for (int64_t b = 0; b < B; ++b)
            if (offsets[b + 1] - offsets[b] < 1) return -1;
    return 0;
}

static int forward_driver(int explicit_scheme, int kind, int n, int hidden, int64_t B, int64_t N,
                          const int64_t *offsets, const double *times, const double *y0, const double *params,
                          int params_shared, double tol_a, double tol_r, int max_newton, int threads,
                          double *y_out, int32_t *status, int32_t *iters)
{
    if (validate(kind, n, hidden, B, N, offsets)) return -1;
    problem_t pb;
    memset(&pb, 0, sizeof(pb));
    pb.explicit_scheme = explicit_scheme;
    pb.kind = kind; pb.n = n; pb.H = hidden; pb.P = oracle_param_count(kind, n, hidden);
    pb.params_shared = params_shared; pb.B = B; pb.N = N; pb.offsets = offsets;
    pb.times = times; pb.y0 = y0; pb.params = params;
    pb.tol_a = tol_a; pb.tol_r = tol_r; pb.max_newton = max_newton;
    pb.y = y_out; pb.status = status; pb.iters = iters;
    return run_pool(&pb, threads, 0, NULL);
}

static int adjoint_driver(int explicit_scheme, int kind, int n, int hidden, int64_t B, int64_t N,
                          const int64_t *offsets, const double *times, const double *y, const double *params,
                          int params_shared, const double *g, int threads, double *dLdp, double *dLdy0,
                          int32_t *status)
{
    if (validate(kind, n, hidden, B, N, offsets)) return -1;
    problem_t pb;
    memset(&pb, 0, sizeof(pb));
    pb.explicit_scheme = explicit_scheme;
    pb.kind = kind; pb.n = n; pb.H = hidden; pb.P = oracle_param_count(kind, n, hidden);
    pb.params_shared = params_shared; pb.B = B; pb.N = N; pb.offsets = offsets;
    pb.times = times; pb.params = params;
    pb.y = (double *)y; pb.g = g; pb.dLdy0 = dLdy0; pb.status = status;
    /* Per-series partial gradients; a shared parameter vector is their sum in
       series order, so the result does not depend on the thread count. */
    double *gp_series;
    if (params_shared) {
        gp_series = calloc((size_t)(B > 0 ? B : 1) * pb.P, sizeof(double));
        if (!gp_series) return -3;
    } else {
        gp_series = dLdp;
        memset(dLdp, 0, sizeof(double) * (size_t)B * pb.P);
    }
    int rc = run_pool(&pb, threads, 1, gp_series);
    if (params_shared) {
        memset(dLdp, 0, sizeof(double) * pb.P);
        for (int64_t b = 0; b < B; ++b)
            for (int i = 0; i < pb.P; ++i) dLdp[i] += gp_series[b * pb.P + i];
        free(gp_series);
    }
    return rc;
}

int oracle_forward(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                   const double *times, const double *y0, const double *params, int params_shared,
                   double tol_a, double tol_r, int max_newton, int threads,
                   double *y_out, int32_t *status, int32_t *iters)
{
    return forward_driver(0, kind, n, hidden, B, N, offsets, times, y0, params, params_shared, tol_a, tol_r,
                          max_newton, threads, y_out, status, iters);
}

int oracle_adjoint(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                   const double *times, const double *y, const double *params, int params_shared,
                   const double *g, int threads, double *dLdp, double *dLdy0, int32_t *status)
{
    return adjoint_driver(0, kind, n, hidden, B, N, offsets, times, y, params, params_shared, g, threads, dLdp,
                          dLdy0, status);
}

int oracle_forward_euler(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                         const double *times, const double *y0, const double *params, int params_shared,
                         int threads, double *y_out, int32_t *status)
{
    return forward_driver(1, kind, n, hidden, B, N, offsets, times, y0, params, params_shared, 0.0, 0.0, 0,
                          threads, y_out, status, NULL);
}

int oracle_forward_euler_adjoint(int kind, int n, int hidden, int64_t B, int64_t N, const int64_t *offsets,
                                 const double *times, const double *y, const double *params, int params_shared,
                                 const double *g, int threads, double *dLdp, double *dLdy0, int32_t *status)
{
    return adjoint_driver(1, kind, n, hidden, B, N, offsets, times, y, params, params_shared, g, threads, dLdp,
                          dLdy0, status);
}
