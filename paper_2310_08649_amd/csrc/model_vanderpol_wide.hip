// Kernel instances of the Van der Pol model for chunks over 2 or 4 waves (double storage).
#include "dispatch.hpp"
#include "wide.hpp"

namespace tvi {

tvi_status launch_vanderpol_wide(int pass, int dtype, const void *args, int S, int T, hipStream_t stream,
                                 const WideExtras &x)
{
    if (dtype != TVI_F64) return TVI_EUNSUPPORTED;
    return wide::launch<VanDerPol, double>(pass, *static_cast<const SolveArgs<double> *>(args), S, T, stream, x);
}

} // namespace tvi
