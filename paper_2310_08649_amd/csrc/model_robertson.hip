// Kernel instances for the Robertson kinetics model.
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_robertson(int pass, int dtype, const void *args, int S, int T, hipStream_t stream)
{
    if (S > kWave) return launch_robertson_wide(pass, dtype, args, S, T, stream);  // chunks over 2 or 4 waves
    if (dtype == TVI_F64)
        return launch_solver<Robertson, double>(pass, *static_cast<const SolveArgs<double> *>(args), S, T, stream);
    return launch_solver<Robertson, float>(pass, *static_cast<const SolveArgs<float> *>(args), S, T, stream);
}

} // namespace tvi
