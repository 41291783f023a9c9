// Host-side argument checks and the kernel-argument record shared by the
// library's entry points and by user models compiled against the library
// (tvi_user_model.hpp).
#pragma once

#include <string.h>

#include "block.hpp"
#include "solver.hpp"
#include "tvi.h"

namespace tvi {
namespace api {

inline bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

inline int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Longest chunk of the register solver: one wave of 64 lanes x 8 steps, or a
// workgroup of up to 4 such waves (wide.hpp: some models, backward Euler).
constexpr int kMaxWaves = 4;
constexpr int kMaxRegisterChunk = kMaxWaves * kWave * 8;  // 2048

// Lanes per series S and steps per lane T for a chunk of C steps: the fewest
// steps per lane that fit the chunk in one wavefront, then the fewest lanes;
// beyond 512 steps, 8 steps per lane over 2 or 4 waves.
inline void choose_tiling(int C, int &S, int &T)
{
    if (C <= 1) { S = 1; T = 1; return; }
    T = 1;
    while (T < 8 && T * kWave < C) T <<= 1;
    S = next_pow2((C + T - 1) / T);
    if (S < 4) S = 4;
    if (S > kMaxWaves * kWave) S = kMaxWaves * kWave;
}

// Lane tiling of the standalone block-bidiagonal solve: at least the rows per
// lane that m needs in one wave, raised towards the count that runs fastest
// for the block size (a lane's own rows cost one composition each, a
// reduction level one per lane, so more rows per lane cut the compositions
// per row; for 2 x 2 blocks the loads, not the arithmetic, set the time, and
// one row per lane keeps them contiguous across the wave), while at least
// four lanes share a system.
inline void pcr_tiling(int n, bool f64, int m, int &S, int &T)
{
    choose_tiling(m, S, T);
    const int pref = n == 2 ? 1 : (n == 4 && !f64) ? 8 : 2;
    while (T < pref && (m + 2 * T - 1) / (2 * T) >= 4) T <<= 1;
    S = next_pow2((m + T - 1) / T);
    if (S < 4) S = 4;
}

inline tvi_status resolve_tiling(const tvi_options *o, int &S, int &T)
{
    if (o->lanes == 0 && o->steps_per_lane == 0) {
        choose_tiling(o->chunk, S, T);
    } else {
        S = o->lanes;
        T = o->steps_per_lane;
        const bool one_wave = (S == 1 || pow2_in(S, 4, kWave)) && pow2_in(T, 1, 8);
        const bool waves = pow2_in(S, 2 * kWave, kMaxWaves * kWave) && pow2_in(T, 2, 8);
        if (!one_wave && !waves) return TVI_EINVAL;
    }
    if (o->chunk > kMaxRegisterChunk || (int64_t)S * T < o->chunk) return TVI_EINVAL;
    return TVI_OK;
}

inline tvi_status check_options(const tvi_options *o)
{
    if (!o) return TVI_EINVAL;
    if (o->obs_idx && o->n_obs < 1) return TVI_EINVAL;
    if (o->chunk < 1 || o->chunk > kMaxRegisterChunk) return TVI_EINVAL;
    if (o->max_newton < 1 || o->max_newton_chunk < 0) return TVI_EINVAL;
    if (!(o->tol_a >= 0.0) || !(o->tol_r >= 0.0)) return TVI_EINVAL;
    if (o->init != TVI_INIT_ZERO && o->init != TVI_INIT_EXTRAP && o->init != TVI_INIT_PREDICTOR) return TVI_EINVAL;
    if (o->init == TVI_INIT_PREDICTOR &&
        (!o->predictor || o->predictor_hidden < 1 || o->predictor_hidden > 256 || o->predictor_steps < o->chunk ||
         (o->predictor_base != 0 && o->predictor_base != 1)))
        return TVI_EINVAL;
    if (o->scheme != TVI_BACKWARD_EULER && o->scheme != TVI_FORWARD_EULER) return TVI_EINVAL;
    if (o->scheme == TVI_FORWARD_EULER && o->init == TVI_INIT_PREDICTOR) return TVI_EUNSUPPORTED;
    if (o->jacobian != TVI_JACOBIAN_ANALYTIC && o->jacobian != TVI_JACOBIAN_FORWARD_AD) return TVI_EINVAL;
    if (o->reference_residual != 0 && o->reference_residual != 1) return TVI_EINVAL;
    if (o->jacobian == TVI_JACOBIAN_FORWARD_AD &&
        (o->scheme != TVI_BACKWARD_EULER || o->init == TVI_INIT_PREDICTOR))
        return TVI_EUNSUPPORTED;
    return TVI_OK;
}

template <class IO>
inline SolveArgs<IO> make_args(const tvi_options *opt, int64_t B, int64_t N, const int64_t *offsets, const void *times,
                        const void *y0, const void *params, int params_shared)
{
    SolveArgs<IO> a;
    memset(&a, 0, sizeof(a));
    a.B = B;
    a.N = N;
    a.K = (N + opt->chunk - 1) / opt->chunk + 1;
    a.offsets = offsets;
    a.times = static_cast<const IO *>(times);
    a.y0 = static_cast<const IO *>(y0);
    a.params = static_cast<const IO *>(params);
    a.params_shared = params_shared;
    a.chunk = opt->chunk;
    a.max_newton = opt->max_newton;
    a.max_newton_chunk = opt->max_newton_chunk;
    a.init = opt->init;
    a.halving = opt->halving;
    a.tol_a = opt->tol_a;
    a.tol_r = opt->tol_r;
    a.pred = static_cast<const float *>(opt->predictor);
    a.pred_hidden = opt->predictor_hidden;
    a.pred_steps = opt->predictor_steps;
    a.pred_base = opt->predictor_base;
    a.order = opt->order;
    a.scheme = opt->scheme;
    a.zero_ref = opt->reference_residual;
    return a;
}

// The options a user model takes: the plain backward-Euler solver with the
// zero or extrapolated start (its Jacobians come from automatic differentiation).
inline tvi_status check_user_options(const tvi_options *o)
{
    tvi_status e = check_options(o);
    if (e != TVI_OK) return e;
    if (o->init == TVI_INIT_PREDICTOR || o->scheme != TVI_BACKWARD_EULER || o->reference_residual != 0)
        return TVI_EUNSUPPORTED;
    if (o->g_divisor || o->obs_idx) return TVI_EUNSUPPORTED;  // register solver: plain g only
    if (o->series_sumsq) return TVI_EUNSUPPORTED;               // the wide forward only
    return TVI_OK;
}

}  // namespace api
}  // namespace tvi
