// Kernel instances for the linear model h = A y with n = 2.
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_linear2(int pass, int dtype, const void *args, int S, int T, hipStream_t stream)
{
    if (dtype == TVI_F64)
        return launch_solver<Linear<2>, double>(pass, *static_cast<const SolveArgs<double> *>(args), S, T, stream);
    return launch_solver<Linear<2>, float>(pass, *static_cast<const SolveArgs<float> *>(args), S, T, stream);
}

} // namespace tvi
