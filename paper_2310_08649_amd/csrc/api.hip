// C ABI entry points (declared in tvi.h): argument checks on the host, choice
// of the lane tiling, and the launch on the caller's stream.
#include <mutex>
#include <string.h>

#include "api_common.hpp"
#include "grad_input.hpp"
#include "dispatch.hpp"

using namespace tvi;
using namespace tvi::api;

namespace {

int model_params(const tvi_model *m)
{
    switch (m->kind) {
    case TVI_LINEAR: return m->n * m->n;
    case TVI_VANDERPOL: return 1;
    case TVI_ROBERTSON: return 3;
    case TVI_CHABOCHE: return 8 + 2 * (m->n - 2);
    case TVI_NEURON: return 15 * (m->n / 4) + 1;
    case TVI_MDS: return 3 * (m->n / 2) + 2;
    case TVI_FNODE: return 2 * (m->n + 1) * (m->n + 1) + 2 * (m->n + 1) + m->n * (m->n + 1) + m->n + 2;
    case TVI_MLP: {
        const int n = m->n, H = m->hidden;
        return H * n + H + H * H + H + n * H + n;
    }
    default: return -1;
    }
}

tvi_status check_model(const tvi_model *m)
{
    if (!m) return TVI_EINVAL;
    if (m->dtype != TVI_F32 && m->dtype != TVI_F64) return TVI_EINVAL;
    switch (m->kind) {
    case TVI_LINEAR: return (m->n >= 2 && m->n <= 4) ? TVI_OK : TVI_EUNSUPPORTED;
    case TVI_VANDERPOL: return m->n == 2 ? TVI_OK : TVI_EINVAL;
    case TVI_ROBERTSON: return m->n == 3 ? TVI_OK : TVI_EINVAL;
    case TVI_CHABOCHE:  // 1 to 5 backstresses in the register-resident solver
        if (m->n < 3) return TVI_EINVAL;
        return m->n <= 7 ? TVI_OK : TVI_EUNSUPPORTED;
    case TVI_NEURON:    // one or two neurons in registers, 3 to 10 by the block solver
        if (m->n < 4 || m->n % 4) return TVI_EINVAL;
        return m->n <= blk::kMaxN ? TVI_OK : TVI_EUNSUPPORTED;
    case TVI_MDS:
        if (m->n < 2 || m->n % 2) return TVI_EINVAL;
        return m->n <= blk::kMaxN ? TVI_OK : TVI_EUNSUPPORTED;
    case TVI_FNODE:
        if (m->n < 1) return TVI_EINVAL;
        return m->n <= blk::kMaxN ? TVI_OK : TVI_EUNSUPPORTED;
    case TVI_MLP:
        if (m->n != 8) return TVI_EINVAL;
        return m->hidden == 64 ? TVI_OK : TVI_EUNSUPPORTED;
    default: return TVI_EINVAL;
    }
}

// Models solved by the block solver: the paper's mass-damper-spring chain and
// forced neural ODE at every size, and more than two coupled neurons.
bool is_block(const tvi_model *m)
{
    return m->kind == TVI_MDS || m->kind == TVI_FNODE || (m->kind == TVI_NEURON && m->n > 8);
}

int block_nf(const tvi_model *m)
{
    switch (m->kind) {
    case TVI_MDS: return block_nf_mds(m->n);
    case TVI_FNODE: return block_nf_fnode(m->n);
    default: return block_nf_neuron(m->n);
    }
}

// Steps per segment of the block solver: 0 = the whole chunk (Thomas's algorithm).
int block_T(const tvi_options *o) { return o->steps_per_lane <= 0 || o->steps_per_lane > o->chunk ? o->chunk : o->steps_per_lane; }

tvi_status check_block(const tvi_model *m, const tvi_options *o)
{
    if (m->dtype != TVI_F64 || m->params_shared) return TVI_EUNSUPPORTED;
    if (o->chunk > blk::kMaxChunk || o->steps_per_lane < 0) return TVI_EINVAL;
    if (o->scheme != TVI_BACKWARD_EULER || o->jacobian != TVI_JACOBIAN_ANALYTIC || o->reference_residual != 0 ||
        o->init == TVI_INIT_PREDICTOR)
        return TVI_EUNSUPPORTED;
    return TVI_OK;
}

size_t block_ws_bytes(const tvi_model *m, const tvi_options *o, int64_t B, bool adjoint)
{
    const blk::WsLayout l = blk::ws_layout(blk::padded(m->n), o->chunk, block_T(o), adjoint ? block_nf(m) : 0);
    return (size_t)B * (size_t)l.total * sizeof(double);
}

tvi_status launch_block(int pass, const tvi_model *m, const blk::BlockArgs *ba, const blk::EvalArgs *ev,
                        hipStream_t st)
{
    switch (m->kind) {
    case TVI_MDS: return launch_block_mds(pass, m->n, ba, ev, st);
    case TVI_FNODE: return launch_block_fnode(pass, m->n, ba, ev, st);
    default: return launch_block_neuron(pass, m->n, ba, ev, st);
    }
}

tvi_status solve_block(int pass, const tvi_model *m, const tvi_options *o, const SolveArgs<double> &a, void *ws,
                       size_t ws_bytes, hipStream_t st, const GradInput *gi = nullptr)
{
    tvi_status e = check_block(m, o);
    if (e != TVI_OK) return e;
    const bool adj = pass != 0;
    if (!ws || ws_bytes < block_ws_bytes(m, o, a.B, adj)) return TVI_EINVAL;
    if (a.B > 0x7fffffffLL) return TVI_EINVAL;
    blk::BlockArgs ba;
    ba.a = a;
    ba.n = m->n;
    ba.P = model_params(m);
    ba.T = block_T(o);
    ba.NF = adj ? block_nf(m) : 0;
    ba.ws_stride = blk::ws_layout(blk::padded(m->n), o->chunk, ba.T, ba.NF).total;
    ba.ws = static_cast<double *>(ws);
    ba.gi = gi ? *gi : GradInput{nullptr, nullptr, 0};
    return launch_block(pass, m, &ba, nullptr, st);
}

tvi_status dispatch(int pass, const tvi_model *model, const void *args, int S, int T, hipStream_t stream,
                    int jacobian = TVI_JACOBIAN_ANALYTIC)
{
    if (jacobian == TVI_JACOBIAN_FORWARD_AD) return launch_ad(model->kind, model->n, pass, model->dtype, args, S, T, stream);
    switch (model->kind) {
    case TVI_VANDERPOL: return launch_vanderpol(pass, model->dtype, args, S, T, stream);
    case TVI_ROBERTSON: return launch_robertson(pass, model->dtype, args, S, T, stream);
    case TVI_CHABOCHE:
        switch (model->n) {
        case 3: return launch_chaboche3(pass, model->dtype, args, S, T, stream);
        case 4: return launch_chaboche4(pass, model->dtype, args, S, T, stream);
        case 5: return launch_chaboche5(pass, model->dtype, args, S, T, stream);
        case 6: return launch_chaboche6(pass, model->dtype, args, S, T, stream);
        case 7: return launch_chaboche7(pass, model->dtype, args, S, T, stream);
        default: return TVI_EUNSUPPORTED;
        }
    case TVI_NEURON:
        return model->n == 4 ? launch_neuron4(pass, model->dtype, args, S, T, stream)
                             : launch_neuron8(pass, model->dtype, args, S, T, stream);
    case TVI_MLP: return launch_mlp(pass, model->dtype, args, stream);
    case TVI_LINEAR:
        switch (model->n) {
        case 2: return launch_linear2(pass, model->dtype, args, S, T, stream);
        case 3: return launch_linear3(pass, model->dtype, args, S, T, stream);
        case 4: return launch_linear4(pass, model->dtype, args, S, T, stream);
        default: return TVI_EUNSUPPORTED;
        }
    default: return TVI_EUNSUPPORTED;
    }
}

// Static device scratch of tvi_solve_adjoint_noalloc.  Host code must not
// pass `scratch` itself to a kernel (in host code it names a host-side
// stand-in): the device address of each GPU's copy comes from
// hipGetSymbolAddress, looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[TVI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void *scratch_ptr[kMaxDevices] = {};

tvi_status device_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TVI_EHIP;
    if (dev >= kMaxDevices) return TVI_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TVI_EHIP;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return TVI_OK;
}

} // namespace

extern "C" {

void tvi_default_options(tvi_options *opt)
{
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->chunk = 64;
    opt->lanes = 0;
    opt->steps_per_lane = 0;
    opt->max_newton = 50;
    opt->tol_a = 1e-8;
    opt->tol_r = 1e-6;
    opt->init = TVI_INIT_ZERO;
    opt->halving = 1;
    opt->predictor = nullptr;
    opt->predictor_hidden = 0;
    opt->predictor_steps = 0;
    opt->predictor_base = 1;
    opt->order = nullptr;
    opt->scheme = TVI_BACKWARD_EULER;
    opt->jacobian = TVI_JACOBIAN_ANALYTIC;
    opt->reference_residual = 0;
    opt->workspace = nullptr;
    opt->workspace_bytes = 0;
    opt->g_divisor = nullptr;
    opt->obs_idx = nullptr;
    opt->n_obs = 0;
    opt->max_newton_chunk = 0;
    opt->series_sumsq = nullptr;
}

const char *tvi_status_str(int32_t s)
{
    switch (s) {
    case TVI_OK: return "ok";
    case TVI_NOT_CONVERGED: return "Newton iteration did not converge";
    case TVI_SINGULAR: return "singular diagonal block";
    case TVI_NONFINITE: return "non-finite residual";
    case TVI_EINVAL: return "invalid argument";
    case TVI_EHIP: return "HIP launch or runtime error";
    case TVI_ENOMEM: return "out of memory";
    case TVI_EUNSUPPORTED: return "unsupported model, size or tiling";
    case TVI_ESCRATCH: return "workspace needed exceeds the static scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

const char *tvi_version(void) { return "tvi 0.1 gfx950"; }

int32_t tvi_param_count(const tvi_model *model) { return model ? model_params(model) : -1; }

tvi_status tvi_model_eval(const tvi_model *model, int64_t M, const void *states, const void *times,
                          const void *params, void *f, void *J, void *stream)
{
    tvi_status e = check_model(model);
    if (e != TVI_OK) return e;
    if (M < 0) return TVI_EINVAL;
    if (M == 0) return TVI_OK;
    if (!states || !params || (!f && !J)) return TVI_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (model->kind == TVI_MLP) {
        if (!model->params_shared) return TVI_EUNSUPPORTED;
        return launch_mlp_eval(model->dtype, M, states, params, f, J, st);
    }
    if (is_block(model)) {
        if (model->dtype != TVI_F64) return TVI_EUNSUPPORTED;
        blk::EvalArgs ev{model->n, model_params(model), model->params_shared, M, static_cast<const double *>(states),
                         static_cast<const double *>(times), static_cast<const double *>(params),
                         static_cast<double *>(f), static_cast<double *>(J)};
        return launch_block(2, model, nullptr, &ev, st);
    }
    return launch_eval(model->kind, model->n, model->dtype, M, states, times, params, model->params_shared, f, J, st);
}

tvi_status tvi_pcr_solve(int32_t dtype, int32_t n, int64_t B, int64_t m, const void *D, const void *r, void *x,
                         int32_t transpose, void *stream)
{
    if (dtype != TVI_F32 && dtype != TVI_F64) return TVI_EINVAL;
    if ((n < 2 || n > 4) && !(n == 8 && dtype == TVI_F32)) return TVI_EUNSUPPORTED;
    if (n == 8 && m > 2 * kWave) return TVI_EUNSUPPORTED;  // two block rows per lane at most
    if (B < 0 || m < 1 || m > 8 * kWave) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!D || !r || !x) return TVI_EINVAL;
    int S, T;
    pcr_tiling(n, dtype == TVI_F64, (int)m, S, T);
    return launch_pcr(dtype, n, B, (int)m, D, r, x, transpose ? 1 : 0, S, T, static_cast<hipStream_t>(stream));
}

tvi_status tvi_solve_forward(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                             const int64_t *offsets, const void *times, const void *y0, const void *params,
                             void *y_out, void *ckpt, int32_t *status, int32_t *iters, void *stream)
{
    tvi_status e = check_model(model);
    if (e != TVI_OK) return e;
    if ((e = check_options(opt)) != TVI_OK) return e;
    if (B < 0 || N < 0) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!times || !y0 || !params || !status || (!y_out && !ckpt)) return TVI_EINVAL;
    int S = 0, T = 0;
    // per-series sums of squares: the forward pass over several waves only
    if (opt->series_sumsq && (is_block(model) || model->kind == TVI_MLP)) return TVI_EUNSUPPORTED;
    if (is_block(model)) {
        if ((e = check_block(model, opt)) != TVI_OK) return e;
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, y0, params, model->params_shared);
        a.y = static_cast<double *>(y_out);
        a.ckpt = static_cast<double *>(ckpt);
        a.status = status;
        a.iters = iters;
        return solve_block(0, model, opt, a, opt->workspace, opt->workspace_bytes, static_cast<hipStream_t>(stream));
    }
    if (model->kind == TVI_MLP) {
        if (opt->chunk > 128 || opt->jacobian != TVI_JACOBIAN_ANALYTIC)
            return TVI_EUNSUPPORTED;
    } else if ((e = resolve_tiling(opt, S, T)) != TVI_OK) {
        return e;
    } else if (opt->init == TVI_INIT_PREDICTOR && (S < 4 || T * model->n > kPredictorMaxTN)) {
        return TVI_EUNSUPPORTED;  // the network is shared by a segment's lanes; register budget
    }
    if (opt->series_sumsq) {
        const bool wide_kind = model->kind == TVI_ROBERTSON || model->kind == TVI_VANDERPOL;
        if (S <= kWave || !wide_kind || model->dtype != TVI_F64 || opt->jacobian != TVI_JACOBIAN_ANALYTIC)
            return TVI_EUNSUPPORTED;
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, y0, params, model->params_shared);
        a.y = static_cast<double *>(y_out);
        a.ckpt = static_cast<double *>(ckpt);
        a.status = status;
        a.iters = iters;
        WideExtras x;
        x.sumsq = opt->series_sumsq;
        const hipStream_t st = static_cast<hipStream_t>(stream);
        return model->kind == TVI_ROBERTSON ? launch_robertson_wide(PASS_FORWARD, TVI_F64, &a, S, T, st, x)
                                            : launch_vanderpol_wide(PASS_FORWARD, TVI_F64, &a, S, T, st, x);
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (model->dtype == TVI_F64) {
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, y0, params, model->params_shared);
        a.y = static_cast<double *>(y_out);
        a.ckpt = static_cast<double *>(ckpt);
        a.status = status;
        a.iters = iters;
        return dispatch(PASS_FORWARD, model, &a, S, T, st, opt->jacobian);
    }
    SolveArgs<float> a = make_args<float>(opt, B, N, offsets, times, y0, params, model->params_shared);
    a.y = static_cast<float *>(y_out);
    a.ckpt = static_cast<double *>(ckpt);
    a.status = status;
    a.iters = iters;
    return dispatch(PASS_FORWARD, model, &a, S, T, st, opt->jacobian);
}

size_t tvi_forward_workspace_bytes(const tvi_model *model, const tvi_options *opt, int64_t B)
{
    if (!model || !opt || B < 0 || opt->chunk < 1 || opt->chunk > kMaxRegisterChunk || check_model(model) != TVI_OK)
        return 0;
    if (!is_block(model) || opt->chunk > blk::kMaxChunk) return 0;
    return block_ws_bytes(model, opt, B, false);
}

size_t tvi_adjoint_workspace_bytes(const tvi_model *model, const tvi_options *opt, int64_t B)
{
    if (!model || !opt || B < 0 || model->n < 1 || opt->chunk < 1) return 0;
    if (model->kind == TVI_MLP) return mlp_theta_workspace_bytes(B);
    if (is_block(model)) {
        if (opt->chunk > blk::kMaxChunk || check_model(model) != TVI_OK) return 0;
        return block_ws_bytes(model, opt, B, true);
    }
    return (size_t)B * (size_t)opt->chunk * (size_t)model->n * sizeof(double);
}

tvi_status tvi_solve_adjoint(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                             const int64_t *offsets, const void *times, const void *params, const void *y,
                             const void *ckpt, const void *g, void *dLdp, void *dLdy0, int32_t *status,
                             void *workspace, size_t workspace_bytes, void *stream)
{
    tvi_status e = check_model(model);
    if (e != TVI_OK) return e;
    if ((e = check_options(opt)) != TVI_OK) return e;
    const bool mlp = model->kind == TVI_MLP;
    if (mlp != (model->params_shared != 0)) return TVI_EUNSUPPORTED;
    if (B < 0 || N < 0) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!times || !params || !g || !dLdp || !dLdy0 || !status) return TVI_EINVAL;
    if (opt->obs_idx && offsets) return TVI_EINVAL;  // observed steps: uniform grids
    const GradInput gi{opt->g_divisor, opt->obs_idx, opt->n_obs};
    const bool recompute = (y == nullptr);
    if (is_block(model)) {
        if (recompute) return TVI_EUNSUPPORTED;  // the block solver reads the stored trajectory
        if ((e = check_block(model, opt)) != TVI_OK) return e;
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
        a.y = const_cast<double *>(static_cast<const double *>(y));
        a.g = static_cast<const double *>(g);
        a.dLdp = static_cast<double *>(dLdp);
        a.dLdy0 = static_cast<double *>(dLdy0);
        a.status = status;
        return solve_block(1, model, opt, a, workspace, workspace_bytes, static_cast<hipStream_t>(stream), &gi);
    }
    if (recompute && !ckpt) return TVI_EINVAL;
    if ((recompute || mlp) &&
        (!workspace || workspace_bytes < tvi_adjoint_workspace_bytes(model, opt, B)))
        return TVI_EINVAL;
    if (mlp) {
        if (opt->chunk > 128 || opt->jacobian != TVI_JACOBIAN_ANALYTIC)
            return TVI_EUNSUPPORTED;
        const int pass = recompute ? PASS_ADJOINT_RECOMPUTE : PASS_ADJOINT;
        const hipStream_t st = static_cast<hipStream_t>(stream);
        if (model->dtype == TVI_F64) {
            SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
            a.y = const_cast<double *>(static_cast<const double *>(y));
            a.ckpt = const_cast<double *>(static_cast<const double *>(ckpt));
            a.g = static_cast<const double *>(g);
            a.dLdp = static_cast<double *>(dLdp);
            a.dLdy0 = static_cast<double *>(dLdy0);
            a.status = status;
            a.ws = static_cast<double *>(workspace);
            return launch_mlp(pass, TVI_F64, &a, st, &gi);
        }
        SolveArgs<float> a = make_args<float>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
        a.y = const_cast<float *>(static_cast<const float *>(y));
        a.ckpt = const_cast<double *>(static_cast<const double *>(ckpt));
        a.g = static_cast<const float *>(g);
        a.dLdp = static_cast<float *>(dLdp);
        a.dLdy0 = static_cast<float *>(dLdy0);
        a.status = status;
        a.ws = static_cast<double *>(workspace);
        return launch_mlp(pass, TVI_F32, &a, st, &gi);
    }
    // the register solver's adjoint reads the plain trajectory-shaped g; the
    // stored-trajectory adjoint over several waves also takes the divisor
    if (gi.obs) return TVI_EUNSUPPORTED;
    int S, T;
    if ((e = resolve_tiling(opt, S, T)) != TVI_OK) return e;
    if (gi.div) {
        const bool wide_kind = model->kind == TVI_ROBERTSON || model->kind == TVI_VANDERPOL;
        if (recompute || S <= kWave || !wide_kind || model->dtype != TVI_F64 ||
            opt->jacobian != TVI_JACOBIAN_ANALYTIC)
            return TVI_EUNSUPPORTED;
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
        a.y = const_cast<double *>(static_cast<const double *>(y));
        a.g = static_cast<const double *>(g);
        a.dLdp = static_cast<double *>(dLdp);
        a.dLdy0 = static_cast<double *>(dLdy0);
        a.status = status;
        const hipStream_t st = static_cast<hipStream_t>(stream);
        WideExtras x;
        x.g_div = gi.div;
        return model->kind == TVI_ROBERTSON ? launch_robertson_wide(PASS_ADJOINT, TVI_F64, &a, S, T, st, x)
                                            : launch_vanderpol_wide(PASS_ADJOINT, TVI_F64, &a, S, T, st, x);
    }
    if (recompute && opt->init == TVI_INIT_PREDICTOR && (S < 4 || T * model->n > kPredictorMaxTN))
        return TVI_EUNSUPPORTED;
    const int pass = recompute ? PASS_ADJOINT_RECOMPUTE : PASS_ADJOINT;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (model->dtype == TVI_F64) {
        SolveArgs<double> a = make_args<double>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
        a.y = const_cast<double *>(static_cast<const double *>(y));
        a.ckpt = const_cast<double *>(static_cast<const double *>(ckpt));
        a.g = static_cast<const double *>(g);
        a.dLdp = static_cast<double *>(dLdp);
        a.dLdy0 = static_cast<double *>(dLdy0);
        a.status = status;
        a.ws = static_cast<double *>(workspace);
        return dispatch(pass, model, &a, S, T, st, opt->jacobian);
    }
    SolveArgs<float> a = make_args<float>(opt, B, N, offsets, times, nullptr, params, model->params_shared);
    a.y = const_cast<float *>(static_cast<const float *>(y));
    a.ckpt = const_cast<double *>(static_cast<const double *>(ckpt));
    a.g = static_cast<const float *>(g);
    a.dLdp = static_cast<float *>(dLdp);
    a.dLdy0 = static_cast<float *>(dLdy0);
    a.status = status;
    a.ws = static_cast<double *>(workspace);
    return dispatch(pass, model, &a, S, T, st, opt->jacobian);
}

tvi_status tvi_solve_adjoint_noalloc(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                                     const int64_t *offsets, const void *times, const void *params, const void *y,
                                     const void *ckpt, const void *g, void *dLdp, void *dLdy0, int32_t *status,
                                     void *stream)
{
    tvi_status e = check_model(model);
    if (e != TVI_OK) return e;
    if ((e = check_options(opt)) != TVI_OK) return e;
    if (B < 0) return TVI_EINVAL;
    if (tvi_adjoint_workspace_bytes(model, opt, B) > TVI_NOALLOC_SCRATCH_BYTES) return TVI_ESCRATCH;
    void *ws = nullptr;
    if ((e = device_scratch(&ws)) != TVI_OK) return e;
    return tvi_solve_adjoint(model, opt, B, N, offsets, times, params, y, ckpt, g, dLdp, dLdy0, status, ws,
                             TVI_NOALLOC_SCRATCH_BYTES, stream);
}

size_t tvi_loss_workspace_bytes(void) { return loss_workspace_bytes(); }

tvi_status tvi_loss_grad(int32_t kind, int32_t dtype, int64_t points, int32_t n, const void *y,
                         const uint8_t *observed, int64_t n_observed, void *g, double *loss, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    if (kind != TVI_LOSS_FROBENIUS && kind != TVI_LOSS_MEAN_SQUARE) return TVI_EINVAL;
    if (dtype != TVI_F32 && dtype != TVI_F64) return TVI_EINVAL;
    if (points < 0 || n < 1) return TVI_EINVAL;
    if (!y || !loss || !workspace || workspace_bytes < loss_workspace_bytes()) return TVI_EINVAL;
    double scale = 1.0;
    if (kind == TVI_LOSS_MEAN_SQUARE) {
        if (!observed || n_observed < 1) return TVI_EINVAL;
        scale = 1.0 / ((double)n_observed * (double)n);
    }
    return launch_loss(kind, dtype, points * n, y, kind == TVI_LOSS_MEAN_SQUARE ? observed : nullptr, n, scale, g,
                       loss, static_cast<double *>(workspace), static_cast<hipStream_t>(stream));
}

tvi_status tvi_loss_from_sums(const double *sums, int64_t B, double *loss, void *stream)
{
    if (!sums || !loss || B < 1) return TVI_EINVAL;
    return launch_loss_from_sums(sums, B, loss, static_cast<hipStream_t>(stream));
}

static bool pred_ok(const tvi_predictor *p)
{
    return p && p->n_in >= 1 && p->hidden >= 1 && p->n_out >= 1 && p->n_in <= 64 && p->hidden <= 1024 &&
           p->n_out <= 4096;
}

int64_t tvi_predictor_param_count(const tvi_predictor *p)
{
    return pred_ok(p) ? predictor_param_count(p->n_in, p->hidden, p->n_out) : -1;
}

size_t tvi_predictor_workspace_bytes(const tvi_predictor *p, int64_t M)
{
    return (pred_ok(p) && M >= 0) ? predictor_workspace_bytes(p->n_in, p->hidden, p->n_out, M) : 0;
}

tvi_status tvi_predictor_forward(const tvi_predictor *p, int64_t M, const float *x, const float *params,
                                 float *out, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!pred_ok(p) || M < 0 || M > 0x7fffffff) return TVI_EINVAL;
    if (M == 0) return TVI_OK;
    if (!x || !params || !out || !workspace || workspace_bytes < tvi_predictor_workspace_bytes(p, M))
        return TVI_EINVAL;
    return predictor_forward(p->n_in, p->hidden, p->n_out, M, x, params, out, workspace,
                             static_cast<hipStream_t>(stream));
}

tvi_status tvi_order_longest_first(const int64_t *offsets, int64_t B, int32_t *order, void *stream)
{
    if (B < 0 || B > 0x7fffffffLL) return TVI_EINVAL;
    if (B == 0) return TVI_OK;
    if (!offsets || !order) return TVI_EINVAL;
    return launch_order(offsets, B, order, static_cast<hipStream_t>(stream));
}

tvi_status tvi_predictor_pack(const tvi_predictor *p, const float *params, float *packed, void *stream)
{
    if (!pred_ok(p) || !params || !packed || params == packed) return TVI_EINVAL;
    return predictor_pack(p->n_in, p->hidden, p->n_out, params, packed, static_cast<hipStream_t>(stream));
}

tvi_status tvi_predictor_train_step(const tvi_predictor *p, int64_t M, const float *x, const float *target,
                                    float *params, float *grad, float *adam_m, float *adam_v, int64_t step,
                                    float lr, float *loss, void *workspace, size_t workspace_bytes,
                                    void *stream)
{
    if (!pred_ok(p) || M < 1 || M > 0x7fffffff || step < 1 || !(lr >= 0.f)) return TVI_EINVAL;
    if (!x || !target || !params || !grad || !adam_m || !adam_v || !loss || !workspace ||
        workspace_bytes < tvi_predictor_workspace_bytes(p, M))
        return TVI_EINVAL;
    return predictor_train_step(p->n_in, p->hidden, p->n_out, M, x, target, params, grad, adam_m, adam_v, step, lr,
                                loss, workspace, static_cast<hipStream_t>(stream));
}

} // extern "C"
