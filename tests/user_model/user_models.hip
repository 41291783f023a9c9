// Right-hand sides written as user models (tvi_user_model.hpp): only the rate,
// once for plain and dual arguments; the state Jacobian and the parameter
// products of the adjoint come from forward-mode automatic differentiation.
// The Van der Pol and Robertson rates of the test workloads, so that the
// results can be checked against the oracle's hand-written models.
#include "tvi_user_model.hpp"

struct UserVanDerPol {
    static constexpr int N = 2;
    static constexpr int P = 1;  // mu
    template <class R, class Q>
    __device__ static void rate(const R (&y)[2], double, const Q (&p)[1], R (&f)[2])
    {
        f[0] = y[1];
        f[1] = p[0] * (1.0 - y[0] * y[0]) * y[1] - y[0];
    }
};

struct UserRobertson {
    static constexpr int N = 3;
    static constexpr int P = 3;  // scale factors of 0.04, 3e7 (on y2^2), 1e4 (on y2 y3)
    template <class R, class Q>
    __device__ static void rate(const R (&y)[3], double, const Q (&p)[3], R (&f)[3])
    {
        const R a = 0.04 * p[0] * y[0], b = 1.0e4 * p[2] * y[1] * y[2], c = 3.0e7 * p[1] * y[1] * y[1];
        f[0] = b - a;
        f[1] = a - b - c;
        f[2] = c;
    }
};

TVI_USER_MODEL(UserVanDerPol, user_vanderpol)
TVI_USER_MODEL(UserRobertson, user_robertson)
