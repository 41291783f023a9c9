// Block-solver instances (state sizes padded to 8, 16, 24, 32, 40) of one
// model; one file per model so that they compile in parallel.
#include "block_models.hpp"
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_block_neuron(int pass, int n, const blk::BlockArgs *ba, const blk::EvalArgs *ev, hipStream_t st)
{
    return blk::launch_model<blk::NeuronBlock>(pass, n, ba, ev, st);
}

int block_params_neuron(int n) { return blk::NeuronBlock::params(n); }
int block_nf_neuron(int n) { return blk::NeuronBlock::nf(n); }

}  // namespace tvi
