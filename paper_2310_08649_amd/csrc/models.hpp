// Right-hand sides h(y, t; p) with analytic state Jacobians j = dh/dy
// (Section 2.2: the analytic option) and parameter vector-Jacobian products
// (dh/dp)^T w for the adjoint gradient (Appendix A).  All device-side, in
// double, with per-series parameters held in registers.
#pragma once

#include "device.hpp"

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
    __device__ __forceinline__ void rhs(const double (&y)[NN], double, double (&f)[NN]) const
    {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) s = fma(A[i][k], y[k], s);
            f[i] = s;
        }
    }
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
    __device__ __forceinline__ void rhs(const double (&y)[2], double, double (&f)[2]) const
    {
        f[0] = y[1];
        f[1] = mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
    }
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
    __device__ __forceinline__ void rhs(const double (&y)[3], double, double (&f)[3]) const
    {
        const double a = k1 * y[0], b = k3 * y[1] * y[2], c = k2 * y[1] * y[1];
        f[0] = -a + b;
        f[1] = a - b - c;
        f[2] = c;
    }
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

} // namespace tvi
