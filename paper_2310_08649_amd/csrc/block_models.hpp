// Right-hand sides of the block solver (state sizes up to 40), written for
// one wavefront per state: lane i evaluates component i of h(y, t; p) and
// writes row i of the state Jacobian dh/dy (NP entries, zero beyond n) to its
// LDS row `jrow`, reading the whole state from LDS.  For the
// adjoint each model writes per-step factors F such that every entry of
// (dh/dp)^T w is the product of two of them (pair(q)), so that
// dL/dp_q = sum over steps of F[a_q] F[b_q].  The paper's example problems of
// Section 5.1.1, with per-series parameter vectors in global memory.
#pragma once

#include "block.hpp"

namespace tvi {
namespace blk {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Mass-damper-spring chain of nu = n / 2 units, state (d_1, v_1, ..., d_nu,
// v_nu), p = (K_1..K_nu, C_1..C_nu, M_1..M_nu, f_a, T).  Unit i is mass M_i
// joined to mass i + 1 (the wall for the last unit) by spring K_i and damper
// C_i; the force f_a sin(2 pi t / T) acts on the first mass:
//   dd_i/dt = v_i,  dv_i/dt = [K_i (d_{i+1} - d_i) + C_i (v_{i+1} - v_i)
//                    - K_{i-1} (d_i - d_{i-1}) - C_{i-1} (v_i - v_{i-1})] / M_i + f_i(t).
struct MdsBlock {
    int n, nu;
    const double *p;

    template <int NP>
    static constexpr int scratch() { return 0; }
    template <int NP>
    static constexpr int max_params() { return 3 * (NP / 2) + 2; }
    static int params(int n) { return 3 * (n / 2) + 2; }
    static int nf(int n) { return 5 * (n / 2) + 3; }

    __device__ void init(int n_, const double *p_) { n = n_; nu = n_ / 2; p = p_; }

    // spring and damper acceleration of mass u
    __device__ double accel(const double *y, int u) const
    {
        const double *K = p, *C = p + nu, *M = p + 2 * nu;
        const double d = y[2 * u], v = y[2 * u + 1];
        const double dn = (u + 1 < nu) ? y[2 * u + 2] : 0.0, vn = (u + 1 < nu) ? y[2 * u + 3] : 0.0;
        double a = K[u] * (dn - d) + C[u] * (vn - v);
        if (u > 0) a -= K[u - 1] * (d - y[2 * u - 2]) + C[u - 1] * (v - y[2 * u - 1]);
        return a / M[u];
    }

    __device__ double rate(const double *y, double t, double *, double *, int lane) const
    {
        if (lane >= n) return 0.0;
        if ((lane & 1) == 0) return y[lane + 1];
        const int u = lane >> 1;
        const double a = accel(y, u);
        return a + (u == 0 ? p[3 * nu] * sin(kTwoPi * t / p[3 * nu + 1]) : 0.0);
    }

    template <int NP>
    __device__ double rate_row(const double *y, double t, double *scr, double *blk, int lane, double *jrow) const
    {
        const double f = rate(y, t, scr, blk, lane);
        if (lane < NP) {
#pragma unroll
            for (int c = 0; c < NP; ++c) jrow[c] = 0.0;
        }
        if (lane < n) {
            if ((lane & 1) == 0) {
                jrow[lane + 1] = 1.0;
            } else {
                const int u = lane >> 1;
                const double *K = p, *C = p + nu, *M = p + 2 * nu;
                double vdd = -K[u] / M[u], vdv = -C[u] / M[u];
                if (u + 1 < nu) {
                    jrow[2 * u + 2] = K[u] / M[u];
                    jrow[2 * u + 3] = C[u] / M[u];
                }
                if (u > 0) {
                    vdd -= K[u - 1] / M[u];
                    vdv -= C[u - 1] / M[u];
                    jrow[2 * u - 2] = K[u - 1] / M[u];
                    jrow[2 * u - 1] = C[u - 1] / M[u];
                }
                jrow[2 * u] = vdd;
                jrow[2 * u + 1] = vdv;
            }
        }
        return f;
    }

    // F = (e_u = d_{u+1} - d_u, e'_u = v_{u+1} - v_u, U_u = w_{v_u}/M_u - w_{v_{u+1}}/M_{u+1},
    //      W_u = w_{v_u}/M_u, -a_u (each over u), w_{v_1}, sin(2 pi t/T), f_a cos(2 pi t/T)(-2 pi t/T^2))
    __device__ void factors(const double *y, double t, const double *w, double *, double *, int lane, double *F) const
    {
        const double *M = p + 2 * nu;
        if (lane < nu) {
            const int u = lane;
            const double d = y[2 * u], v = y[2 * u + 1];
            const double dn = (u + 1 < nu) ? y[2 * u + 2] : 0.0, vn = (u + 1 < nu) ? y[2 * u + 3] : 0.0;
            const double wu = w[2 * u + 1] / M[u];
            const double wn = (u + 1 < nu) ? w[2 * u + 3] / M[u + 1] : 0.0;
            F[u] = dn - d;
            F[nu + u] = vn - v;
            F[2 * nu + u] = wu - wn;
            F[3 * nu + u] = wu;
            F[4 * nu + u] = -accel(y, u);
        }
        if (lane == 0) {
            const double T = p[3 * nu + 1], ph = kTwoPi * t / T;
            F[5 * nu] = w[1];
            F[5 * nu + 1] = sin(ph);
            F[5 * nu + 2] = p[3 * nu] * cos(ph) * (-ph / T);
        }
    }

    __device__ void pair(int q, int &a, int &b) const
    {
        if (q < nu) { a = 2 * nu + q; b = q; }                       // K
        else if (q < 2 * nu) { a = 2 * nu + q - nu; b = q; }         // C: (U, e')
        else if (q < 3 * nu) { a = 3 * nu + q - 2 * nu; b = 4 * nu + q - 2 * nu; }  // M: (W, -a)
        else if (q == 3 * nu) { a = 5 * nu; b = 5 * nu + 1; }        // f_a
        else { a = 5 * nu; b = 5 * nu + 2; }                          // T
    }
};

// Coupled neurons, nu = n / 4, state (V_i, m_i, h_i, n_i); per neuron
// p = (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf, tau_m, h_inf, tau_h, n_inf,
// tau_n, g_C, T), then I_a:
//   dV_i/dt = (-g_Na m^3 h (V_i - E_Na) - g_K n^4 (V_i - E_K) - g_L (V_i - E_L)
//              + I_a sin(2 pi t / T_i) + g_C sum_j (V_i - V_j)) / C_i,
//   dx/dt = (x_inf - x) / tau_x  for x = m, h, n.
struct NeuronBlock {
    int n, nu;
    const double *p;
    enum { C_, GNA, ENA, GK, EK, GL, EL, MINF, TM, HINF, TH, NINF, TN, GC, TP, PER };
    static constexpr int kF = 19;  // factors per neuron

    template <int NP>
    static constexpr int scratch() { return 0; }
    template <int NP>
    static constexpr int max_params() { return PER * (NP / 4) + 1; }
    static int params(int n) { return PER * (n / 4) + 1; }
    static int nf(int n) { return kF * (n / 4) + 2; }

    __device__ void init(int n_, const double *p_) { n = n_; nu = n_ / 4; p = p_; }

    __device__ double coupling(const double *y, double V) const
    {
        double c = 0.0;
        for (int j = 0; j < nu; ++j) c += V - y[4 * j];
        return c;
    }

    __device__ double rate(const double *y, double t, double *, double *, int lane) const
    {
        if (lane >= n) return 0.0;
        const int u = lane >> 2, comp = lane & 3;
        const double *q = p + PER * u;
        const double x = y[lane];
        if (comp == 1) return (q[MINF] - x) / q[TM];
        if (comp == 2) return (q[HINF] - x) / q[TH];
        if (comp == 3) return (q[NINF] - x) / q[TN];
        const double V = x, m = y[lane + 1], hh = y[lane + 2], nn = y[lane + 3];
        const double I = p[PER * nu] * sin(kTwoPi * t / q[TP]);
        const double m3 = m * m * m, n4 = nn * nn * nn * nn;
        const double F = -q[GNA] * m3 * hh * (V - q[ENA]) - q[GK] * n4 * (V - q[EK]) - q[GL] * (V - q[EL]) + I +
                         q[GC] * coupling(y, V);
        return F / q[C_];
    }

    template <int NP>
    __device__ double rate_row(const double *y, double t, double *scr, double *blk, int lane, double *jrow) const
    {
        const double f = rate(y, t, scr, blk, lane);
        if (lane < NP) {
#pragma unroll
            for (int c = 0; c < NP; ++c) jrow[c] = 0.0;
        }
        if (lane < n) {
            const int u = lane >> 2, comp = lane & 3;
            const double *q = p + PER * u;
            if (comp == 0) {
                const double V = y[lane], m = y[lane + 1], hh = y[lane + 2], nn = y[lane + 3];
                const double m3 = m * m * m, n4 = nn * nn * nn * nn;
                const double off = -q[GC] / q[C_];
                for (int j = 0; j < nu; ++j) jrow[4 * j] = off;
                jrow[lane] = (-q[GNA] * m3 * hh - q[GK] * n4 - q[GL] + q[GC] * (nu - 1)) / q[C_];
                jrow[lane + 1] = -3.0 * q[GNA] * m * m * hh * (V - q[ENA]) / q[C_];
                jrow[lane + 2] = -q[GNA] * m3 * (V - q[ENA]) / q[C_];
                jrow[lane + 3] = -4.0 * q[GK] * nn * nn * nn * (V - q[EK]) / q[C_];
            } else {
                jrow[lane] = -1.0 / q[comp == 1 ? TM : comp == 2 ? TH : TN];
            }
        }
        return f;
    }

    // per neuron u at F[19 u + k]: the weights w_V / C, w_m, w_h, w_n and the
    // partial derivatives they multiply; then sum_u (w_V/C)_u sin(2 pi t/T_u) and 1
    __device__ void factors(const double *y, double t, const double *w, double *, double *, int lane, double *F) const
    {
        double sIa = 0.0;
        if (lane < nu) {
            const int u = lane;
            const double *q = p + PER * u;
            double *o = F + kF * u;
            const double V = y[4 * u], m = y[4 * u + 1], hh = y[4 * u + 2], nn = y[4 * u + 3];
            const double Ia = p[PER * nu], ph = kTwoPi * t / q[TP];
            const double m3 = m * m * m, n4 = nn * nn * nn * nn, cpl = coupling(y, V);
            const double Fv = -q[GNA] * m3 * hh * (V - q[ENA]) - q[GK] * n4 * (V - q[EK]) - q[GL] * (V - q[EL]) +
                              Ia * sin(ph) + q[GC] * cpl;
            const double wv = w[4 * u] / q[C_];
            o[0] = wv;
            o[1] = -Fv / q[C_];
            o[2] = -m3 * hh * (V - q[ENA]);
            o[3] = q[GNA] * m3 * hh;
            o[4] = -n4 * (V - q[EK]);
            o[5] = q[GK] * n4;
            o[6] = -(V - q[EL]);
            o[7] = q[GL];
            o[8] = cpl;
            o[9] = Ia * cos(ph) * (-ph / q[TP]);
            o[10] = w[4 * u + 1];
            o[11] = 1.0 / q[TM];
            o[12] = -(q[MINF] - m) / (q[TM] * q[TM]);
            o[13] = w[4 * u + 2];
            o[14] = 1.0 / q[TH];
            o[15] = -(q[HINF] - hh) / (q[TH] * q[TH]);
            o[16] = w[4 * u + 3];
            o[17] = 1.0 / q[TN];
            o[18] = -(q[NINF] - nn) / (q[TN] * q[TN]);
            sIa = wv * sin(ph);
        }
        sIa = seg_sum<kWave>(sIa);
        if (lane == 0) {
            F[kF * nu] = sIa;
            F[kF * nu + 1] = 1.0;
        }
    }

    __device__ void pair(int q, int &a, int &b) const
    {
        if (q >= PER * nu) { a = kF * nu; b = kF * nu + 1; return; }  // I_a
        const int u = q / PER, k = q - u * PER;
        int fa = 0, fb;
        switch (k) {
        case C_: fb = 1; break;
        case GNA: fb = 2; break;
        case ENA: fb = 3; break;
        case GK: fb = 4; break;
        case EK: fb = 5; break;
        case GL: fb = 6; break;
        case EL: fb = 7; break;
        case MINF: fa = 10; fb = 11; break;
        case TM: fa = 10; fb = 12; break;
        case HINF: fa = 13; fb = 14; break;
        case TH: fa = 13; fb = 15; break;
        case NINF: fa = 16; fb = 17; break;
        case TN: fa = 16; fb = 18; break;
        case GC: fb = 8; break;
        default: fb = 9; break;  // T
        }
        a = kF * u + fa;
        b = kF * u + fb;
    }
};

// Forced neural ODE of size n (Section 5.1.1): x = (y, f_a sin(2 pi t / T)),
// a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), h = tanh(W3 a2 + b3) with
// W1, W2 (n+1) x (n+1), W3 n x (n+1); p = (W1, b1, W2, b2, W3, b3, f_a, T),
// matrices row-major.  The wave computes one layer at a time, lane a holding
// unit a, the layer inputs shared through LDS.
struct FnodeBlock {
    int n, m;
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    double fa, T;

    // scratch: x, a1, a2, a3, d3, d2, d1 (NP + 1 each)
    template <int NP>
    static constexpr int scratch() { return 7 * (NP + 1); }
    template <int NP>
    static constexpr int max_params() { return 2 * (NP + 1) * (NP + 1) + 2 * (NP + 1) + NP * (NP + 1) + NP + 2; }
    static int params(int n) { return 2 * (n + 1) * (n + 1) + 2 * (n + 1) + n * (n + 1) + n + 2; }
    static int nf(int n) { return 5 * (n + 1) + n + 4; }

    __device__ void init(int n_, const double *p)
    {
        n = n_;
        m = n_ + 1;
        W1 = p;
        b1 = W1 + m * m;
        W2 = b1 + m;
        b2 = W2 + m * m;
        W3 = b2 + m;
        b3 = W3 + n * m;
        fa = b3[n];
        T = b3[n + 1];
    }

    // layers at state y (LDS), time t: x, a1, a2, a3 into scr
    __device__ void layers(const double *y, double t, double *scr, int lane) const
    {
        double *x = scr, *a1 = scr + m, *a2 = scr + 2 * m, *a3 = scr + 3 * m;
        if (lane < n) x[lane] = y[lane];
        if (lane == n) x[n] = fa * sin(kTwoPi * t / T);
        wave_sync();
        if (lane < m) {
            double s = b1[lane];
            for (int k = 0; k < m; ++k) s += W1[lane * m + k] * x[k];
            a1[lane] = tanh(s);
        }
        wave_sync();
        if (lane < m) {
            double s = b2[lane];
            for (int k = 0; k < m; ++k) s += W2[lane * m + k] * a1[k];
            a2[lane] = tanh(s);
        }
        wave_sync();
        if (lane < n) {
            double s = b3[lane];
            for (int k = 0; k < m; ++k) s += W3[lane * m + k] * a2[k];
            a3[lane] = tanh(s);
        }
        wave_sync();
    }

    __device__ double rate(const double *y, double t, double *scr, double *, int lane) const
    {
        layers(y, t, scr, lane);
        return lane < n ? scr[3 * m + lane] : 0.0;
    }

    // row i of diag(1 - h^2) W3 diag(1 - a2^2) G with G = W2 diag(1 - a1^2) W1[:, 0:n]
    // (G by lane a = row a into blk first)
    template <int NP>
    __device__ double rate_row(const double *y, double t, double *scr, double *blk, int lane, double *jrow) const
    {
        layers(y, t, scr, lane);
        const double *a1 = scr + m, *a2 = scr + 2 * m, *a3 = scr + 3 * m;
        if (lane < m) {
            double acc[NP];
#pragma unroll
            for (int c = 0; c < NP; ++c) acc[c] = 0.0;
            for (int b = 0; b < m; ++b) {
                const double coef = W2[lane * m + b] * (1.0 - a1[b] * a1[b]);
                const double *wr = W1 + b * m;
#pragma unroll
                for (int c = 0; c < NP; ++c)
                    if (c < n) acc[c] = fma(coef, wr[c], acc[c]);
            }
#pragma unroll
            for (int c = 0; c < NP; ++c) blk[lane * (NP + 1) + c] = acc[c];
        }
        wave_sync();
        double row[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) row[c] = 0.0;
        double f = 0.0;
        if (lane < n) {
            for (int a = 0; a < m; ++a) {
                const double u = W3[lane * m + a] * (1.0 - a2[a] * a2[a]);
                const double *gr = blk + a * (NP + 1);
#pragma unroll
                for (int c = 0; c < NP; ++c) row[c] = fma(u, gr[c], row[c]);
            }
            f = a3[lane];
            const double s3 = 1.0 - f * f;
#pragma unroll
            for (int c = 0; c < NP; ++c) row[c] *= s3;
        }
        wave_sync();  // every lane is done with G before the rows overwrite it
        if (lane < NP) {
#pragma unroll
            for (int c = 0; c < NP; ++c) jrow[c] = row[c];
        }
        return f;
    }

    // F = (x, a1, a2, d1, d2 (m each), d3 (n), 1, g_x, sin(2 pi t/T), f_a cos(2 pi t/T)(-2 pi t/T^2))
    // with d3 = w (1 - h^2), d2 = (W3^T d3)(1 - a2^2), d1 = (W2^T d2)(1 - a1^2), g_x = W1[:, n] . d1
    __device__ void factors(const double *y, double t, const double *w, double *scr, double *, int lane,
                            double *F) const
    {
        layers(y, t, scr, lane);
        const double *x = scr, *a1 = scr + m, *a2 = scr + 2 * m, *a3 = scr + 3 * m;
        double *d3 = scr + 4 * m, *d2 = scr + 5 * m, *d1 = scr + 6 * m;
        if (lane < n) d3[lane] = w[lane] * (1.0 - a3[lane] * a3[lane]);
        wave_sync();
        if (lane < m) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += W3[i * m + lane] * d3[i];
            d2[lane] = s * (1.0 - a2[lane] * a2[lane]);
        }
        wave_sync();
        double gx = 0.0;
        if (lane < m) {
            double s = 0.0;
            for (int c = 0; c < m; ++c) s += W2[c * m + lane] * d2[c];
            d1[lane] = s * (1.0 - a1[lane] * a1[lane]);
            gx = W1[lane * m + n] * d1[lane];
        }
        gx = seg_sum<kWave>(gx);
        if (lane < m) {
            F[lane] = x[lane];
            F[m + lane] = a1[lane];
            F[2 * m + lane] = a2[lane];
            F[3 * m + lane] = d1[lane];
            F[4 * m + lane] = d2[lane];
        }
        if (lane < n) F[5 * m + lane] = d3[lane];
        if (lane == 0) {
            const double ph = kTwoPi * t / T;
            F[5 * m + n] = 1.0;
            F[5 * m + n + 1] = gx;
            F[5 * m + n + 2] = sin(ph);
            F[5 * m + n + 3] = fa * cos(ph) * (-ph / T);
        }
        wave_sync();
    }

    __device__ void pair(int q, int &a, int &b) const
    {
        const int one = 5 * m + n, mm = m * m;
        if (q < mm) { a = 3 * m + q / m; b = q % m; return; }                 // W1: d1_a x_b
        q -= mm;
        if (q < m) { a = 3 * m + q; b = one; return; }                         // b1
        q -= m;
        if (q < mm) { a = 4 * m + q / m; b = m + q % m; return; }             // W2: d2_a a1_b
        q -= mm;
        if (q < m) { a = 4 * m + q; b = one; return; }                         // b2
        q -= m;
        if (q < n * m) { a = 5 * m + q / m; b = 2 * m + q % m; return; }     // W3: d3_i a2_a
        q -= n * m;
        if (q < n) { a = 5 * m + q; b = one; return; }                         // b3
        q -= n;
        a = one + 1;
        b = q == 0 ? one + 2 : one + 3;                                         // f_a, T
    }
};

}  // namespace blk
}  // namespace tvi
