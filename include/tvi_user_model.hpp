/*
 * tvi_user_model.hpp -- your own right-hand side in the chunked backward-Euler
 * solver and its discrete adjoint, without hand-written derivatives.
 *
 * The method needs, besides the rate h(y, t; p), the state Jacobian dh/dy for
 * the Newton blocks D_j = I - dt_j dh/dy (Section 2.2, which lets it come from
 * automatic differentiation instead of by hand) and the parameter products
 * (dh/dp)^T w of the adjoint gradient (Appendix A).  Here both come from one
 * forward-mode evaluation of the rate on dual numbers: N directions seeded on
 * the state for the Jacobian, P directions seeded on the parameters for the
 * parameter products.
 *
 * A model is a struct with
 *     static constexpr int N;   // state size, 1 <= N <= 8
 *     static constexpr int P;   // parameters per series, 1 <= P <= 32
 *     template <class R, class Q>
 *     __device__ static void rate(const R (&y)[N], double t, const Q (&p)[P], R (&f)[N]);
 * written once for every argument type: R is double or tvi::Dual<K>, Q is
 * double or R.  Use +, -, *, / (also with double constants) and the functions
 * tvi::exp_t, log_t, sqrt_t, sin_t, cos_t, tanh_t, abs_t, pow_pos, fma_t,
 * which take plain and dual arguments alike.
 *
 * In one HIP source file, compiled for gfx950 with this directory and
 * paper_2310_08649_amd/csrc on the include path (and -Xclang -target-feature
 * -Xclang -packed-fp32-ops, as the library itself is built),
 *     TVI_USER_MODEL(MyModel, mymodel)
 * defines the C entry points
 *     tvi_status mymodel_solve_forward(const tvi_options *opt, int64_t B, int64_t N,
 *         const int64_t *offsets, const void *times, const void *y0, const void *params,
 *         void *y_out, void *ckpt, int32_t *status, int32_t *iters, void *stream);
 *     tvi_status mymodel_solve_adjoint(const tvi_options *opt, int64_t B, int64_t N,
 *         const int64_t *offsets, const void *times, const void *params, const void *y,
 *         const void *ckpt, const void *g, void *dLdp, void *dLdy0, int32_t *status,
 *         void *workspace, size_t workspace_bytes, void *stream);
 *     size_t mymodel_adjoint_workspace_bytes(const tvi_options *opt, int64_t B);
 * with the meaning, layouts, checks and errors of tvi_solve_forward and
 * tvi_solve_adjoint (tvi.h) for double storage and per-series parameters
 * [B][P]: backward Euler, zero or extrapolated start, any lane tiling of the
 * library's solver (one step per lane when N > 4).
 */
#ifndef TVI_USER_MODEL_HPP
#define TVI_USER_MODEL_HPP

#include "api_common.hpp"
#include "dispatch.hpp"
#include "tvi.h"

namespace tvi {
namespace user {

// The solver's model interface on top of a user rate.
template <class U>
struct UserAD {
    static constexpr int N = U::N;
    static constexpr int P = U::P;
    static_assert(N >= 1 && N <= 8, "user models: 1 <= N <= 8");
    static_assert(P >= 1 && P <= 32, "user models: 1 <= P <= 32");
    double p[P];

    template <class IO>
    __device__ __forceinline__ void load(const IO *q)
    {
#pragma unroll
        for (int k = 0; k < P; ++k) p[k] = ld(q + k);
    }
    template <class V>
    __device__ __forceinline__ void rhs_t(const V (&y)[N], double t, V (&f)[N]) const { U::rate(y, t, p, f); }
    __device__ __forceinline__ void rhs(const double (&y)[N], double t, double (&f)[N]) const { U::rate(y, t, p, f); }
    __device__ __forceinline__ void jac(const double (&y)[N], double t, double (&J)[N][N]) const
    {
        Dual<N> yd[N], fd[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            yd[k].v = y[k];
#pragma unroll
            for (int c = 0; c < N; ++c) yd[k].d[c] = (c == k) ? 1.0 : 0.0;
        }
        U::rate(yd, t, p, fd);
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) J[r][c] = fd[r].d[c];
    }
    // gp += (dh/dp)^T w
    __device__ __forceinline__ void vjp_p(const double (&y)[N], double t, const double (&w)[N], double (&gp)[P]) const
    {
        Dual<P> yd[N], pd[P], fd[N];
#pragma unroll
        for (int k = 0; k < N; ++k) yd[k] = Dual<P>(y[k]);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            pd[k].v = p[k];
#pragma unroll
            for (int c = 0; c < P; ++c) pd[k].d[c] = (c == k) ? 1.0 : 0.0;
        }
        U::rate(yd, t, pd, fd);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            double s = gp[c];
#pragma unroll
            for (int r = 0; r < N; ++r) s = fma(w[r], fd[r].d[c], s);
            gp[c] = s;
        }
    }
};

}  // namespace user

// user models get the plain backward-Euler instances only
template <class U>
struct Variants<user::UserAD<U>> {
    static constexpr bool value = false;
};
template <class U>
struct MaxStepsPerLane<user::UserAD<U>> {
    static constexpr int value = U::N <= 4 ? 8 : 1;
};

namespace user {

template <class M>
tvi_status solve_forward(const tvi_options *opt, int64_t B, int64_t N, const int64_t *offsets, const void *times,
                         const void *y0, const void *params, void *y_out, void *ckpt, int32_t *status,
                         int32_t *iters, void *stream)
{
    tvi_status e = api::check_user_options(opt);
    if (e != TVI_OK) return e;
    if (B < 0 || N < 0) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!times || !y0 || !params || !status || (!y_out && !ckpt)) return TVI_EINVAL;
    int S, T;
    if ((e = api::resolve_tiling(opt, S, T)) != TVI_OK) return e;
    SolveArgs<double> a = api::make_args<double>(opt, B, N, offsets, times, y0, params, 0);
    a.y = static_cast<double *>(y_out);
    a.ckpt = static_cast<double *>(ckpt);
    a.status = status;
    a.iters = iters;
    return launch_solver<M, double>(PASS_FORWARD, a, S, T, static_cast<hipStream_t>(stream));
}

inline size_t adjoint_workspace_bytes(int n, const tvi_options *opt, int64_t B)
{
    if (!opt || B < 0 || opt->chunk < 1) return 0;
    return (size_t)B * (size_t)opt->chunk * (size_t)n * sizeof(double);
}

template <class M>
tvi_status solve_adjoint(const tvi_options *opt, int64_t B, int64_t N, const int64_t *offsets, const void *times,
                         const void *params, const void *y, const void *ckpt, const void *g, void *dLdp, void *dLdy0,
                         int32_t *status, void *workspace, size_t workspace_bytes, void *stream)
{
    tvi_status e = api::check_user_options(opt);
    if (e != TVI_OK) return e;
    if (B < 0 || N < 0) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!times || !params || !g || !dLdp || !dLdy0 || !status) return TVI_EINVAL;
    const bool recompute = y == nullptr;
    if (recompute && (!ckpt || !workspace || workspace_bytes < adjoint_workspace_bytes(M::N, opt, B)))
        return TVI_EINVAL;
    int S, T;
    if ((e = api::resolve_tiling(opt, S, T)) != TVI_OK) return e;
    SolveArgs<double> a = api::make_args<double>(opt, B, N, offsets, times, nullptr, params, 0);
    a.y = const_cast<double *>(static_cast<const double *>(y));
    a.ckpt = const_cast<double *>(static_cast<const double *>(ckpt));
    a.g = static_cast<const double *>(g);
    a.dLdp = static_cast<double *>(dLdp);
    a.dLdy0 = static_cast<double *>(dLdy0);
    a.status = status;
    a.ws = static_cast<double *>(workspace);
    return launch_solver<M, double>(recompute ? PASS_ADJOINT_RECOMPUTE : PASS_ADJOINT, a, S, T,
                                    static_cast<hipStream_t>(stream));
}

}  // namespace user
}  // namespace tvi

#define TVI_USER_MODEL(Type, name)                                                                                   \
    extern "C" tvi_status name##_solve_forward(const tvi_options *opt, int64_t B, int64_t N, const int64_t *offsets, \
                                               const void *times, const void *y0, const void *params, void *y_out,  \
                                               void *ckpt, int32_t *status, int32_t *iters, void *stream)           \
    {                                                                                                                \
        return tvi::user::solve_forward<tvi::user::UserAD<Type>>(opt, B, N, offsets, times, y0, params, y_out, ckpt, \
                                                                 status, iters, stream);                             \
    }                                                                                                                \
    extern "C" tvi_status name##_solve_adjoint(const tvi_options *opt, int64_t B, int64_t N, const int64_t *offsets, \
                                               const void *times, const void *params, const void *y, const void *ckpt, \
                                               const void *g, void *dLdp, void *dLdy0, int32_t *status,             \
                                               void *workspace, size_t workspace_bytes, void *stream)               \
    {                                                                                                                \
        return tvi::user::solve_adjoint<tvi::user::UserAD<Type>>(opt, B, N, offsets, times, params, y, ckpt, g,      \
                                                                  dLdp, dLdy0, status, workspace, workspace_bytes,   \
                                                                  stream);                                           \
    }                                                                                                                \
    extern "C" size_t name##_adjoint_workspace_bytes(const tvi_options *opt, int64_t B)                             \
    {                                                                                                                \
        return tvi::user::adjoint_workspace_bytes(Type::N, opt, B);                                                  \
    }

#endif
