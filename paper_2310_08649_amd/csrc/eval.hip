// Model rates and state Jacobians for a batch of independent states: the
// assembly step of the chunk system (h and j at every step) as an entry
// point of its own.
#include "dispatch.hpp"

namespace tvi {

template <class Model, class IO>
__global__ __launch_bounds__(256) void eval_kernel(int64_t M, const IO *states, const IO *times, const IO *params,
                                                   int32_t shared, IO *f, IO *J)
{
    constexpr int n = Model::N;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    Model model;
    model.load(shared ? params : params + q * Model::P);
    double y[n], fv[n], Jv[n][n];
#pragma unroll
    for (int k = 0; k < n; ++k) y[k] = ld(states + q * n + k);
    const double t = times ? ld(times + q) : 0.0;
    model.rhs(y, t, fv);
    model.jac(y, t, Jv);
    if (f) {
#pragma unroll
        for (int k = 0; k < n; ++k) st(f + q * n + k, fv[k]);
    }
    if (J) {
#pragma unroll
        for (int r = 0; r < n; ++r)
#pragma unroll
            for (int c = 0; c < n; ++c) st(J + (q * n + r) * n + c, Jv[r][c]);
    }
}

template <class Model, class IO>
static tvi_status eval_launch(int64_t M, const void *states, const void *times, const void *params, int shared,
                              void *f, void *J, hipStream_t stream)
{
    const int64_t blocks = (M + 255) / 256;
    if (blocks > 0x7fffffffLL) return TVI_EINVAL;
    hipLaunchKernelGGL((eval_kernel<Model, IO>), dim3((unsigned)blocks), dim3(256), 0, stream, M,
                       static_cast<const IO *>(states), static_cast<const IO *>(times),
                       static_cast<const IO *>(params), shared, static_cast<IO *>(f), static_cast<IO *>(J));
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

template <class Model>
static tvi_status eval_dtype(int dtype, int64_t M, const void *states, const void *times, const void *params,
                             int shared, void *f, void *J, hipStream_t stream)
{
    return dtype == TVI_F64 ? eval_launch<Model, double>(M, states, times, params, shared, f, J, stream)
                            : eval_launch<Model, float>(M, states, times, params, shared, f, J, stream);
}

tvi_status launch_eval(int kind, int n, int dtype, int64_t M, const void *states, const void *times,
                       const void *params, int shared, void *f, void *J, hipStream_t stream)
{
    if (M == 0) return TVI_OK;
    switch (kind) {
    case TVI_VANDERPOL: return eval_dtype<VanDerPol>(dtype, M, states, times, params, shared, f, J, stream);
    case TVI_ROBERTSON: return eval_dtype<Robertson>(dtype, M, states, times, params, shared, f, J, stream);
    case TVI_CHABOCHE:
        switch (n) {
        case 3: return eval_dtype<Chaboche<1>>(dtype, M, states, times, params, shared, f, J, stream);
        case 4: return eval_dtype<Chaboche<2>>(dtype, M, states, times, params, shared, f, J, stream);
        case 5: return eval_dtype<Chaboche<3>>(dtype, M, states, times, params, shared, f, J, stream);
        case 6: return eval_dtype<Chaboche<4>>(dtype, M, states, times, params, shared, f, J, stream);
        case 7: return eval_dtype<Chaboche<5>>(dtype, M, states, times, params, shared, f, J, stream);
        default: return TVI_EUNSUPPORTED;
        }
    case TVI_NEURON:
        if (n == 4) return eval_dtype<Neuron1>(dtype, M, states, times, params, shared, f, J, stream);
        if (n == 8) return eval_dtype<Neurons<2>>(dtype, M, states, times, params, shared, f, J, stream);
        return TVI_EUNSUPPORTED;
    case TVI_LINEAR:
        switch (n) {
        case 2: return eval_dtype<Linear<2>>(dtype, M, states, times, params, shared, f, J, stream);
        case 3: return eval_dtype<Linear<3>>(dtype, M, states, times, params, shared, f, J, stream);
        case 4: return eval_dtype<Linear<4>>(dtype, M, states, times, params, shared, f, J, stream);
        default: return TVI_EUNSUPPORTED;
        }
    default: return TVI_EUNSUPPORTED;
    }
}

} // namespace tvi
