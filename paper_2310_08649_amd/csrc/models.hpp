// Right-hand sides h(y, t; p) with analytic state Jacobians j = dh/dy
// (Section 2.2: the analytic option) and parameter vector-Jacobian products
// (dh/dp)^T w for the adjoint gradient (Appendix A).  All device-side, in
// double, with per-series parameters held in registers.
#pragma once

#include "device.hpp"
#include "dual.hpp"

namespace tvi {

// h = A y, p = A (row-major n x n).
template <int NN>
struct Linear {
    static constexpr int N = NN;
    static constexpr int P = NN * NN;
    double A[NN][NN];

    template <class IO>
    __device__ __forceinline__ void load(const IO *p)
    {
#pragma unroll
        for (int i = 0; i < NN; ++i)
#pragma unroll
            for (int k = 0; k < NN; ++k) A[i][k] = ld(p + i * NN + k);
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[NN], double, V (&f)[NN]) const
    {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            V s = V(0.0);
#pragma unroll
            for (int k = 0; k < NN; ++k) s = fma_t(A[i][k], y[k], s);
            f[i] = s;
        }
    }
    __device__ __forceinline__ void rhs(const double (&y)[NN], double t, double (&f)[NN]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&)[NN], double, double (&J)[NN][NN]) const
    {
#pragma unroll
        for (int i = 0; i < NN; ++i)
#pragma unroll
            for (int k = 0; k < NN; ++k) J[i][k] = A[i][k];
    }
    // dL/dA_ik += w_i y_k
    __device__ __forceinline__ void vjp_p(const double (&y)[NN], double, const double (&w)[NN],
                                          double (&gp)[P]) const
    {
#pragma unroll
        for (int i = 0; i < NN; ++i)
#pragma unroll
            for (int k = 0; k < NN; ++k) gp[i * NN + k] = fma(w[i], y[k], gp[i * NN + k]);
    }
};

// Van der Pol: h = (y2, mu (1 - y1^2) y2 - y1), p = (mu).
struct VanDerPol {
    static constexpr int N = 2;
    static constexpr int P = 1;
    double mu;

    template <class IO>
    __device__ __forceinline__ void load(const IO *p) { mu = ld(p); }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[2], double, V (&f)[2]) const
    {
        f[0] = y[1];
        f[1] = mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
    }
    __device__ __forceinline__ void rhs(const double (&y)[2], double t, double (&f)[2]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&y)[2], double, double (&J)[2][2]) const
    {
        J[0][0] = 0.0;
        J[0][1] = 1.0;
        J[1][0] = -2.0 * mu * y[0] * y[1] - 1.0;
        J[1][1] = mu * (1.0 - y[0] * y[0]);
    }
    // dh/dmu = (0, (1 - y1^2) y2)
    __device__ __forceinline__ void vjp_p(const double (&y)[2], double, const double (&w)[2], double (&gp)[1]) const
    {
        gp[0] = fma(w[1], (1.0 - y[0] * y[0]) * y[1], gp[0]);
    }
};

// Robertson kinetics: k1 = 0.04 s1, k2 = 3e7 s2 (on y2^2), k3 = 1e4 s3 (on y2 y3).
struct Robertson {
    static constexpr int N = 3;
    static constexpr int P = 3;
    double k1, k2, k3;

    template <class IO>
    __device__ __forceinline__ void load(const IO *p)
    {
        k1 = 0.04 * ld(p);
        k2 = 3.0e7 * ld(p + 1);
        k3 = 1.0e4 * ld(p + 2);
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[3], double, V (&f)[3]) const
    {
        const V a = k1 * y[0], b = k3 * y[1] * y[2], c = k2 * y[1] * y[1];
        f[0] = -a + b;
        f[1] = a - b - c;
        f[2] = c;
    }
    __device__ __forceinline__ void rhs(const double (&y)[3], double t, double (&f)[3]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&y)[3], double, double (&J)[3][3]) const
    {
        J[0][0] = -k1;
        J[0][1] = k3 * y[2];
        J[0][2] = k3 * y[1];
        J[1][0] = k1;
        J[1][1] = -k3 * y[2] - 2.0 * k2 * y[1];
        J[1][2] = -k3 * y[1];
        J[2][0] = 0.0;
        J[2][1] = 2.0 * k2 * y[1];
        J[2][2] = 0.0;
    }
    // dh/ds1 = 0.04 (-y1, y1, 0); dh/ds2 = 3e7 (0, -y2^2, y2^2); dh/ds3 = 1e4 (y2 y3, -y2 y3, 0)
    __device__ __forceinline__ void vjp_p(const double (&y)[3], double, const double (&w)[3], double (&gp)[3]) const
    {
        gp[0] += 0.04 * y[0] * (w[1] - w[0]);
        gp[1] += 3.0e7 * y[1] * y[1] * (w[2] - w[1]);
        gp[2] += 1.0e4 * y[1] * y[2] * (w[0] - w[1]);
    }
};

// Chaboche viscoplasticity (Section 5.1.1) with NU backstresses: state
// (sigma, K, X_1..X_NU), p = (E, n, eta, sigma0, K_inf, tau, C_1..C_NU,
// gamma_1..gamma_NU, edot_a, T).  With s = sigma - sum X and
// a = (|s| - K - sigma0) / eta the plastic rate is ep = <a>^n sign(s):
//   dsigma/dt = E (edot(t) - ep),  dK/dt = tau (K_inf - K) |ep|,
//   dX_i/dt = 2/3 C_i ep - gamma_i X_i |ep|,  edot(t) = edot_a sin(2 pi t / T)
// (isotropic hardening driven by the plastic rate, the model's standard form).
template <int NU>
struct Chaboche {
    static constexpr int N = 2 + NU;
    static constexpr int P = 8 + 2 * NU;
    double E, ex, eta, s0, Kinf, tau, C[NU], gam[NU], eda, T;

    template <class IO>
    __device__ __forceinline__ void load(const IO *p)
    {
        E = ld(p);
        ex = ld(p + 1);
        eta = ld(p + 2);
        s0 = ld(p + 3);
        Kinf = ld(p + 4);
        tau = ld(p + 5);
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            C[i] = ld(p + 6 + i);
            gam[i] = ld(p + 6 + NU + i);
        }
        eda = ld(p + 6 + 2 * NU);
        T = ld(p + 7 + 2 * NU);
    }
    // sign of s, the overstress a, <a>^n, d<a>^n/d|s| and the imposed strain rate
    struct Flow {
        double sg, a, pa, dpa, edot;
    };
    __device__ __forceinline__ Flow flow(const double (&y)[N], double t) const
    {
        Flow c;
        double sx = 0.0;
#pragma unroll
        for (int i = 0; i < NU; ++i) sx += y[2 + i];
        const double s = y[0] - sx;
        c.sg = s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0);
        c.a = (fabs(s) - y[1] - s0) / eta;
        const double pm1 = c.a > 0.0 ? pow(c.a, ex - 1.0) : 0.0;
        c.pa = pm1 * c.a;
        c.dpa = ex * pm1 / eta;
        c.edot = eda * sin(2.0 * M_PI * t / T);
        return c;
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[N], double t, V (&f)[N]) const
    {
        V sx = V(0.0);
#pragma unroll
        for (int i = 0; i < NU; ++i) sx = sx + y[2 + i];
        const V s = y[0] - sx;
        const double sg = val(s) > 0.0 ? 1.0 : (val(s) < 0.0 ? -1.0 : 0.0);
        const V a = (abs_t(s) - y[1] - s0) / eta;
        const V pa = val(a) > 0.0 ? pow_pos(a, ex) : V(0.0);  // <a>^n as a^(n-1) a, as in flow()
        const V ep = pa * sg;
        const double edot = eda * sin(2.0 * M_PI * t / T);
        f[0] = E * (edot - ep);
        f[1] = tau * (Kinf - y[1]) * pa;
#pragma unroll
        for (int i = 0; i < NU; ++i) f[2 + i] = 2.0 / 3.0 * C[i] * ep - gam[i] * y[2 + i] * pa;
    }
    __device__ __forceinline__ void rhs(const double (&y)[N], double t, double (&f)[N]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&y)[N], double t, double (&J)[N][N]) const
    {
        const Flow c = flow(y, t);
        // derivatives of ep and of |ep| with respect to sigma, K and X_j
        double dep[N], dab[N];
        dep[0] = c.dpa * c.sg * c.sg;
        dab[0] = c.dpa * c.sg;
        dep[1] = -c.dpa * c.sg;
        dab[1] = -c.dpa;
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            dep[2 + j] = -c.dpa * c.sg * c.sg;
            dab[2 + j] = -c.dpa * c.sg;
        }
        const double hk = tau * (Kinf - y[1]);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            J[0][k] = -E * dep[k];
            J[1][k] = hk * dab[k] - ((k == 1) ? tau * c.pa : 0.0);
#pragma unroll
            for (int i = 0; i < NU; ++i)
                J[2 + i][k] = 2.0 / 3.0 * C[i] * dep[k] - gam[i] * y[2 + i] * dab[k] - ((k == 2 + i) ? gam[i] * c.pa : 0.0);
        }
    }
    __device__ __forceinline__ void vjp_p(const double (&y)[N], double t, const double (&w)[N], double (&gp)[P]) const
    {
        const Flow c = flow(y, t);
        const double ep = c.pa * c.sg;
        // the weights carried by ep and by |ep| = <a>^n
        double g_ep = -E * w[0], g_pa = w[1] * tau * (Kinf - y[1]);
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            g_ep += 2.0 / 3.0 * C[i] * w[2 + i];
            g_pa -= gam[i] * y[2 + i] * w[2 + i];
        }
        const double g_a = g_ep * c.sg + g_pa;
        if (c.a > 0.0) {
            gp[1] += g_a * c.pa * log(c.a);
            gp[2] += g_a * (-ex * c.pa / eta);
            gp[3] += g_a * (-c.dpa);
        }
        gp[0] += w[0] * (c.edot - ep);
        gp[4] += w[1] * tau * c.pa;
        gp[5] += w[1] * (Kinf - y[1]) * c.pa;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            gp[6 + i] += w[2 + i] * (2.0 / 3.0) * ep;
            gp[6 + NU + i] -= w[2 + i] * y[2 + i] * c.pa;
        }
        const double ph = 2.0 * M_PI * t / T;
        gp[6 + 2 * NU] += w[0] * E * sin(ph);
        gp[7 + 2 * NU] += w[0] * E * eda * cos(ph) * (-ph / T);
    }
};

// One neuron of the coupled-neuron model (Section 5.1.1): state (V, m, h, n),
// p = (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf, tau_m, h_inf, tau_h, n_inf,
// tau_n, g_C, T, I_a):
//   dV/dt = (-g_Na m^3 h (V - E_Na) - g_K n^4 (V - E_K) - g_L (V - E_L) + I(t)) / C,
//   dx/dt = (x_inf - x) / tau_x for x = m, h, n,  I(t) = I_a sin(2 pi t / T)
// (the coupling sum over the other neurons is empty for one neuron).
struct Neuron1 {
    static constexpr int N = 4;
    static constexpr int P = 16;
    double q[P];

    template <class IO>
    __device__ __forceinline__ void load(const IO *p)
    {
#pragma unroll
        for (int k = 0; k < P; ++k) q[k] = ld(p + k);
    }
    enum { C, GNA, ENA, GK, EK, GL, EL, MINF, TM, HINF, TH, NINF, TN, GC, TP, IA };
    template <class V>
    __device__ __forceinline__ V current(const V (&y)[4], double t) const
    {
        const V m3 = y[1] * y[1] * y[1], n4 = y[3] * y[3] * y[3] * y[3];
        return -q[GNA] * m3 * y[2] * (y[0] - q[ENA]) - q[GK] * n4 * (y[0] - q[EK]) - q[GL] * (y[0] - q[EL]) +
               q[IA] * sin(2.0 * M_PI * t / q[TP]);
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[4], double t, V (&f)[4]) const
    {
        f[0] = current(y, t) / q[C];
        f[1] = (q[MINF] - y[1]) / q[TM];
        f[2] = (q[HINF] - y[2]) / q[TH];
        f[3] = (q[NINF] - y[3]) / q[TN];
    }
    __device__ __forceinline__ void rhs(const double (&y)[4], double t, double (&f)[4]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&y)[4], double, double (&J)[4][4]) const
    {
        const double m = y[1], h = y[2], n = y[3], V = y[0];
        J[0][0] = (-q[GNA] * m * m * m * h - q[GK] * n * n * n * n - q[GL]) / q[C];
        J[0][1] = -3.0 * q[GNA] * m * m * h * (V - q[ENA]) / q[C];
        J[0][2] = -q[GNA] * m * m * m * (V - q[ENA]) / q[C];
        J[0][3] = -4.0 * q[GK] * n * n * n * (V - q[EK]) / q[C];
#pragma unroll
        for (int r = 1; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) J[r][c] = 0.0;
        J[1][1] = -1.0 / q[TM];
        J[2][2] = -1.0 / q[TH];
        J[3][3] = -1.0 / q[TN];
    }
    __device__ __forceinline__ void vjp_p(const double (&y)[4], double t, const double (&w)[4], double (&gp)[P]) const
    {
        const double m = y[1], h = y[2], n = y[3], V = y[0];
        const double m3 = m * m * m, n4 = n * n * n * n;
        const double ph = 2.0 * M_PI * t / q[TP];
        const double wv = w[0] / q[C];
        gp[C] -= wv * current(y, t) / q[C];
        gp[GNA] -= wv * m3 * h * (V - q[ENA]);
        gp[ENA] += wv * q[GNA] * m3 * h;
        gp[GK] -= wv * n4 * (V - q[EK]);
        gp[EK] += wv * q[GK] * n4;
        gp[GL] -= wv * (V - q[EL]);
        gp[EL] += wv * q[GL];
        gp[TP] += wv * q[IA] * cos(ph) * (-ph / q[TP]);
        gp[IA] += wv * sin(ph);
        gp[MINF] += w[1] / q[TM];
        gp[TM] -= w[1] * (q[MINF] - m) / (q[TM] * q[TM]);
        gp[HINF] += w[2] / q[TH];
        gp[TH] -= w[2] * (q[HINF] - h) / (q[TH] * q[TH]);
        gp[NINF] += w[3] / q[TN];
        gp[TN] -= w[3] * (q[NINF] - n) / (q[TN] * q[TN]);
    }
};

// NU coupled neurons (Section 5.1.1): state (V_i, m_i, h_i, n_i) per neuron,
// p = the 15 per-neuron values (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf, tau_m,
// h_inf, tau_h, n_inf, tau_n, g_C, T) of each neuron, then I_a:
//   dV_i/dt = (-g_Na m^3 h (V_i - E_Na) - g_K n^4 (V_i - E_K) - g_L (V_i - E_L)
//              + I_a sin(2 pi t / T_i) + g_C sum_j (V_i - V_j)) / C_i,
//   dx_i/dt = (x_inf - x_i) / tau_x for x = m, h, n.
template <int NU>
struct Neurons {
    static constexpr int N = 4 * NU;
    static constexpr int P = 15 * NU + 1;
    double q[P];
    enum { C, GNA, ENA, GK, EK, GL, EL, MINF, TM, HINF, TH, NINF, TN, GC, TP };

    template <class IO>
    __device__ __forceinline__ void load(const IO *p)
    {
#pragma unroll
        for (int k = 0; k < P; ++k) q[k] = ld(p + k);
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[N], double t, V (&f)[N]) const
    {
        V vs = V(0.0);
#pragma unroll
        for (int j = 0; j < NU; ++j) vs = vs + y[4 * j];
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            const double *u = q + 15 * i;
            const V &Vi = y[4 * i], &m = y[4 * i + 1], &h = y[4 * i + 2], &n = y[4 * i + 3];
            const V m3 = m * m * m, n4 = n * n * n * n;
            const V cpl = NU * Vi - vs;  // sum over j of (V_i - V_j)
            const V F = -u[GNA] * m3 * h * (Vi - u[ENA]) - u[GK] * n4 * (Vi - u[EK]) - u[GL] * (Vi - u[EL]) +
                        q[15 * NU] * sin(2.0 * M_PI * t / u[TP]) + u[GC] * cpl;
            f[4 * i] = F / u[C];
            f[4 * i + 1] = (u[MINF] - m) / u[TM];
            f[4 * i + 2] = (u[HINF] - h) / u[TH];
            f[4 * i + 3] = (u[NINF] - n) / u[TN];
        }
    }
    __device__ __forceinline__ void rhs(const double (&y)[N], double t, double (&f)[N]) const { rhs_t(y, t, f); }
    __device__ __forceinline__ void jac(const double (&y)[N], double, double (&J)[N][N]) const
    {
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) J[r][c] = 0.0;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            const double *u = q + 15 * i;
            const double V = y[4 * i], m = y[4 * i + 1], h = y[4 * i + 2], n = y[4 * i + 3];
#pragma unroll
            for (int j = 0; j < NU; ++j) J[4 * i][4 * j] = (j == i) ? 0.0 : -u[GC] / u[C];
            J[4 * i][4 * i] = (-u[GNA] * m * m * m * h - u[GK] * n * n * n * n - u[GL] + u[GC] * (NU - 1)) / u[C];
            J[4 * i][4 * i + 1] = -3.0 * u[GNA] * m * m * h * (V - u[ENA]) / u[C];
            J[4 * i][4 * i + 2] = -u[GNA] * m * m * m * (V - u[ENA]) / u[C];
            J[4 * i][4 * i + 3] = -4.0 * u[GK] * n * n * n * (V - u[EK]) / u[C];
            J[4 * i + 1][4 * i + 1] = -1.0 / u[TM];
            J[4 * i + 2][4 * i + 2] = -1.0 / u[TH];
            J[4 * i + 3][4 * i + 3] = -1.0 / u[TN];
        }
    }
    __device__ __forceinline__ void vjp_p(const double (&y)[N], double t, const double (&w)[N], double (&gp)[P]) const
    {
        double vs = 0.0;
#pragma unroll
        for (int j = 0; j < NU; ++j) vs += y[4 * j];
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            const double *u = q + 15 * i;
            double *g = gp + 15 * i;
            const double V = y[4 * i], m = y[4 * i + 1], h = y[4 * i + 2], n = y[4 * i + 3];
            const double m3 = m * m * m, n4 = n * n * n * n, cpl = NU * V - vs;
            const double ph = 2.0 * M_PI * t / u[TP], Ia = q[15 * NU];
            const double F = -u[GNA] * m3 * h * (V - u[ENA]) - u[GK] * n4 * (V - u[EK]) - u[GL] * (V - u[EL]) +
                             Ia * sin(ph) + u[GC] * cpl;
            const double wv = w[4 * i] / u[C];
            g[C] -= wv * F / u[C];
            g[GNA] -= wv * m3 * h * (V - u[ENA]);
            g[ENA] += wv * u[GNA] * m3 * h;
            g[GK] -= wv * n4 * (V - u[EK]);
            g[EK] += wv * u[GK] * n4;
            g[GL] -= wv * (V - u[EL]);
            g[EL] += wv * u[GL];
            g[GC] += wv * cpl;
            g[TP] += wv * Ia * cos(ph) * (-ph / u[TP]);
            gp[15 * NU] += wv * sin(ph);
            g[MINF] += w[4 * i + 1] / u[TM];
            g[TM] -= w[4 * i + 1] * (u[MINF] - m) / (u[TM] * u[TM]);
            g[HINF] += w[4 * i + 2] / u[TH];
            g[TH] -= w[4 * i + 2] * (u[HINF] - h) / (u[TH] * u[TH]);
            g[NINF] += w[4 * i + 3] / u[TN];
            g[TN] -= w[4 * i + 3] * (u[NINF] - n) / (u[TN] * u[TN]);
        }
    }
};

// A model whose state Jacobian comes from forward-mode automatic
// differentiation of its right-hand side (one evaluation on duals seeded with
// the unit vectors) instead of the hand-written one; the rate and the
// parameter products are the model's own.
template <class M>
struct ForwardAD : M {
    static constexpr int N = M::N;
    __device__ __forceinline__ void jac(const double (&y)[N], double t, double (&J)[N][N]) const
    {
        Dual<N> yd[N], fd[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            yd[k].v = y[k];
#pragma unroll
            for (int c = 0; c < N; ++c) yd[k].d[c] = (c == k) ? 1.0 : 0.0;
        }
        this->rhs_t(yd, t, fd);
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) J[r][c] = fd[r].d[c];
    }
};

} // namespace tvi
