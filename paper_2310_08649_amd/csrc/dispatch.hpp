// Host-side selection of the kernel instance for a (model, storage type,
// lanes per series S, steps per lane T) combination.
#pragma once

#include <hip/hip_runtime.h>

#include "solver.hpp"
#include "tvi.h"

namespace tvi {

enum Pass : int { PASS_FORWARD = 0, PASS_ADJOINT = 1, PASS_ADJOINT_RECOMPUTE = 2 };

// Models with the learned-start and forward-Euler instances
// (the forward-AD Jacobian variants have the plain backward-Euler ones only).
template <class M>
struct Variants {
    static constexpr bool value = true;
};
template <class M>
struct Variants<ForwardAD<M>> {
    static constexpr bool value = false;
};
// Chaboche with 3-5 backstresses (n = 5..7): one step per lane and the plain
// backward-Euler instances only (the registers of larger blocks)
template <int NU>
struct Variants<Chaboche<NU>> {
    static constexpr bool value = NU <= 2;
};
// Two coupled neurons (n = 8): likewise
template <int NU>
struct Variants<Neurons<NU>> {
    static constexpr bool value = false;
};
template <class M>
struct MaxStepsPerLane {
    static constexpr int value = 8;
};
template <int NU>
struct MaxStepsPerLane<Neurons<NU>> {
    static constexpr int value = 1;
};
template <int NU>
struct MaxStepsPerLane<Chaboche<NU>> {
    static constexpr int value = NU <= 2 ? 8 : 1;
};

template <class Model, class IO, int S, int T>
static tvi_status launch_st(int pass, const SolveArgs<IO> &a, hipStream_t stream)
{
    const int64_t per_block = kWave / S;
    const int64_t blocks = (a.B + per_block - 1) / per_block;
    if (blocks == 0) return TVI_OK;
    if (blocks > 0x7fffffffLL) return TVI_EINVAL;
    dim3 grid((unsigned)blocks), block(kWave);
    const bool pred = a.init == INIT_PREDICTOR;
    // the learned start has its own instances (segments of >= 4 lanes, T n <= kPredictorMaxTN)
    constexpr bool kVar = Variants<Model>::value;
    constexpr bool kPred = kVar && S >= 4 && T * Model::N <= kPredictorMaxTN;
    if (pred && !kPred && pass != PASS_ADJOINT) return TVI_EUNSUPPORTED;
    // its hidden layers and outputs: [segments][2H + n S T] floats of LDS
    const size_t lds = pred ? (size_t)per_block * (2 * a.pred_hidden + Model::N * S * T) * sizeof(float) : 0;
    // the zero-increment reference of the relative test (matters only for a nonzero start)
    const bool zref = a.zero_ref != 0 && a.init != INIT_ZERO;
    // (instances for the plain backward-Euler solver only)
    if (zref && (!kVar || pred || a.scheme != 0)) return TVI_EUNSUPPORTED;
    if (a.scheme == 1) {  // forward Euler: its own instances, no learned start
        if (pred || !kVar) return TVI_EUNSUPPORTED;
        if constexpr (kVar) switch (pass) {
        case PASS_FORWARD:
            hipLaunchKernelGGL((forward_kernel<Model, IO, S, T, false, true>), grid, block, 0, stream, a);
            break;
        case PASS_ADJOINT:
            hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, false, false, true>), grid, block, 0, stream, a);
            break;
        case PASS_ADJOINT_RECOMPUTE:
            hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, true, false, true>), grid, block, 0, stream, a);
            break;
        default: return TVI_EINVAL;
        }
        return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
    }
    switch (pass) {
    case PASS_FORWARD:
        if constexpr (kPred) {
            if (pred) {
                hipLaunchKernelGGL((forward_kernel<Model, IO, S, T, true>), grid, block, lds, stream, a);
                break;
            }
        }
        if constexpr (kVar) {
            if (zref) {
                hipLaunchKernelGGL((forward_kernel<Model, IO, S, T, false, false, true>), grid, block, 0, stream, a);
                break;
            }
        }
        hipLaunchKernelGGL((forward_kernel<Model, IO, S, T, false>), grid, block, 0, stream, a);
        break;
    case PASS_ADJOINT:
        hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, false, false>), grid, block, 0, stream, a);
        break;
    case PASS_ADJOINT_RECOMPUTE:
        if constexpr (kPred) {
            if (pred) {
                hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, true, true>), grid, block, lds, stream, a);
                break;
            }
        }
        if constexpr (kVar) {
            if (zref) {
                hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, true, false, false, true>), grid, block, 0, stream,
                                   a);
                break;
            }
        }
        hipLaunchKernelGGL((adjoint_kernel<Model, IO, S, T, true, false>), grid, block, 0, stream, a);
        break;
    default: return TVI_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

template <class Model, class IO, int S>
static tvi_status launch_s(int pass, const SolveArgs<IO> &a, int T, hipStream_t stream)
{
    constexpr int kMaxT = MaxStepsPerLane<Model>::value;
    if (T > kMaxT) return TVI_EUNSUPPORTED;
    switch (T) {
    case 1: return launch_st<Model, IO, S, 1>(pass, a, stream);
    case 2:
        if constexpr (kMaxT >= 2) return launch_st<Model, IO, S, 2>(pass, a, stream);
        break;
    case 4:
        if constexpr (kMaxT >= 4) return launch_st<Model, IO, S, 4>(pass, a, stream);
        break;
    case 8:
        if constexpr (kMaxT >= 8) return launch_st<Model, IO, S, 8>(pass, a, stream);
        break;
    default: break;
    }
    return TVI_EUNSUPPORTED;
}

template <class Model, class IO>
tvi_status launch_solver(int pass, const SolveArgs<IO> &a, int S, int T, hipStream_t stream)
{
    switch (S) {
    case 1: return launch_s<Model, IO, 1>(pass, a, T, stream);
    case 4: return launch_s<Model, IO, 4>(pass, a, T, stream);
    case 8: return launch_s<Model, IO, 8>(pass, a, T, stream);
    case 16: return launch_s<Model, IO, 16>(pass, a, T, stream);
    case 32: return launch_s<Model, IO, 32>(pass, a, T, stream);
    case 64: return launch_s<Model, IO, 64>(pass, a, T, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

// One entry per model family, defined in its own translation unit.
tvi_status launch_vanderpol(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_robertson(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
// chunks over 2 or 4 waves (S = 128, 256; T = 2, 4, 8), csrc/model_{vanderpol,robertson}_wide.hip
struct WideExtras {
    const double *g_div = nullptr;  // stored-trajectory adjoint: device scalar dividing every entry of g
    double *sumsq = nullptr;        // forward: [B] per-series sums of squares of the stored states
};
tvi_status launch_vanderpol_wide(int pass, int dtype, const void *args, int S, int T, hipStream_t stream,
                                 const WideExtras &x = WideExtras{});
tvi_status launch_robertson_wide(int pass, int dtype, const void *args, int S, int T, hipStream_t stream,
                                 const WideExtras &x = WideExtras{});
tvi_status launch_linear2(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_linear3(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_linear4(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_chaboche3(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_chaboche4(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_chaboche5(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_chaboche6(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_chaboche7(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_neuron4(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_neuron8(int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
// the same models with forward-AD state Jacobians (double storage only)
tvi_status launch_ad(int kind, int n, int pass, int dtype, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_ad_vdp_rob(int kind, int pass, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_ad_linear(int n, int pass, const void *args, int S, int T, hipStream_t stream);
tvi_status launch_pcr(int dtype, int n, int64_t B, int m, const void *D, const void *r, void *x, int transpose,
                      int S, int T, hipStream_t stream);
struct GradInput;
// gi: how the adjoint reads dL/dy (null: the plain trajectory-shaped g)
tvi_status launch_mlp(int pass, int dtype, const void *args, hipStream_t stream, const GradInput *gi = nullptr);
size_t mlp_theta_workspace_bytes(int64_t B);
tvi_status launch_mlp_eval(int dtype, int64_t M, const void *states, const void *params, void *f, void *J,
                           hipStream_t stream);
tvi_status launch_eval(int kind, int n, int dtype, int64_t M, const void *states, const void *times,
                       const void *params, int shared, void *f, void *J, hipStream_t stream);
tvi_status launch_order(const int64_t *offsets, int64_t B, int32_t *order, hipStream_t stream);
tvi_status launch_loss_from_sums(const double *sums, int64_t B, double *loss, hipStream_t stream);
tvi_status launch_loss(int kind, int dtype, int64_t count, const void *y, const uint8_t *observed,
                       int64_t point_stride, double scale, void *g, double *loss, double *partial,
                       hipStream_t stream);
size_t loss_workspace_bytes();
int64_t predictor_param_count(int n_in, int H, int n_out);
size_t predictor_workspace_bytes(int n_in, int H, int n_out, int64_t M);
tvi_status predictor_forward(int n_in, int H, int n_out, int64_t M, const float *x, const float *params, float *out,
                             void *ws, hipStream_t st);
tvi_status predictor_pack(int n_in, int H, int n_out, const float *params, float *packed, hipStream_t st);
tvi_status predictor_train_step(int n_in, int H, int n_out, int64_t M, const float *x, const float *target,
                                float *params, float *grad, float *adam_m, float *adam_v, int64_t step, float lr,
                                float *loss, void *ws, hipStream_t st);

// Block solver (state sizes up to 40), csrc/block_*.hip: pass 0 forward,
// 1 adjoint (stored trajectory), 2 model evaluation.
namespace blk {
struct BlockArgs;
struct EvalArgs;
}
tvi_status launch_block_mds(int pass, int n, const blk::BlockArgs *ba, const blk::EvalArgs *ev, hipStream_t st);
tvi_status launch_block_neuron(int pass, int n, const blk::BlockArgs *ba, const blk::EvalArgs *ev, hipStream_t st);
tvi_status launch_block_fnode(int pass, int n, const blk::BlockArgs *ba, const blk::EvalArgs *ev, hipStream_t st);
int block_params_mds(int n);
int block_params_neuron(int n);
int block_params_fnode(int n);
int block_nf_mds(int n);
int block_nf_neuron(int n);
int block_nf_fnode(int n);

} // namespace tvi
