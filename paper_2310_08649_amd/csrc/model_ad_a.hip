// Forward-AD Jacobian instances: Van der Pol and Robertson (double storage).
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_ad_vdp_rob(int kind, int pass, const void *args, int S, int T, hipStream_t stream)
{
    const SolveArgs<double> &a = *static_cast<const SolveArgs<double> *>(args);
    if (kind == TVI_VANDERPOL) return launch_solver<ForwardAD<VanDerPol>, double>(pass, a, S, T, stream);
    return launch_solver<ForwardAD<Robertson>, double>(pass, a, S, T, stream);
}

} // namespace tvi
