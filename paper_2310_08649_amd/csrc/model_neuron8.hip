// Kernel instances for the coupled-neuron model (two neurons; one step per lane).
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_neuron8(int pass, int dtype, const void *args, int S, int T, hipStream_t stream)
{
    // double storage only (the paper's example problems run in double)
    if (dtype != TVI_F64) return TVI_EUNSUPPORTED;
    return launch_solver<Neurons<2>, double>(pass, *static_cast<const SolveArgs<double> *>(args), S, T, stream);
}

} // namespace tvi
