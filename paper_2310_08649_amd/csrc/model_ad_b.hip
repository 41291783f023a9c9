// Forward-AD Jacobian instances: the linear model, n = 2, 3, 4 (double storage).
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_ad_linear(int n, int pass, const void *args, int S, int T, hipStream_t stream)
{
    const SolveArgs<double> &a = *static_cast<const SolveArgs<double> *>(args);
    switch (n) {
    case 2: return launch_solver<ForwardAD<Linear<2>>, double>(pass, a, S, T, stream);
    case 3: return launch_solver<ForwardAD<Linear<3>>, double>(pass, a, S, T, stream);
    case 4: return launch_solver<ForwardAD<Linear<4>>, double>(pass, a, S, T, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

} // namespace tvi
