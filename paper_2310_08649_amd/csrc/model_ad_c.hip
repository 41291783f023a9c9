// Forward-AD Jacobian instances: the Chaboche and neuron models (double
// storage), and the entry that picks the model.
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_ad(int kind, int n, int pass, int dtype, const void *args, int S, int T, hipStream_t stream)
{
    if (dtype != TVI_F64) return TVI_EUNSUPPORTED;
    const SolveArgs<double> &a = *static_cast<const SolveArgs<double> *>(args);
    switch (kind) {
    case TVI_VANDERPOL:
    case TVI_ROBERTSON: return launch_ad_vdp_rob(kind, pass, args, S, T, stream);
    case TVI_LINEAR: return launch_ad_linear(n, pass, args, S, T, stream);
    case TVI_CHABOCHE:
        if (n == 3) return launch_solver<ForwardAD<Chaboche<1>>, double>(pass, a, S, T, stream);
        if (n == 4) return launch_solver<ForwardAD<Chaboche<2>>, double>(pass, a, S, T, stream);
        return TVI_EUNSUPPORTED;
    case TVI_NEURON:
        if (n == 4) return launch_solver<ForwardAD<Neuron1>, double>(pass, a, S, T, stream);
        return TVI_EUNSUPPORTED;
    default: return TVI_EUNSUPPORTED;
    }
}

} // namespace tvi
