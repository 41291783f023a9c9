// Block-solver instances (state sizes padded to 8, 16, 24, 32, 40) of one
// model; one file per model so that they compile in parallel.
#include "block_models.hpp"
#include "dispatch.hpp"

namespace tvi {

tvi_status launch_block_fnode(int pass, int n, const blk::BlockArgs *ba, const blk::EvalArgs *ev, hipStream_t st)
{
    return blk::launch_model<blk::FnodeBlock>(pass, n, ba, ev, st);
}

int block_params_fnode(int n) { return blk::FnodeBlock::params(n); }
int block_nf_fnode(int n) { return blk::FnodeBlock::nf(n); }

}  // namespace tvi
