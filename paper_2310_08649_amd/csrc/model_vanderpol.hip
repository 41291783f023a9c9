// Kernel instances for the Van der Pol model.
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_vanderpol(int pass, int dtype, const void *args, int S, int T, hipStream_t stream)
{
    if (S > kWave) return launch_vanderpol_wide(pass, dtype, args, S, T, stream);  // chunks over 2 or 4 waves
    if (dtype == TVI_F64)
        return launch_solver<VanDerPol, double>(pass, *static_cast<const SolveArgs<double> *>(args), S, T, stream);
    return launch_solver<VanDerPol, float>(pass, *static_cast<const SolveArgs<float> *>(args), S, T, stream);
}

} // namespace tvi
