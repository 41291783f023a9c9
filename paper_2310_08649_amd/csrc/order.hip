// Launch order of ragged series: longest first.  With every series in its own
// workgroup (or lane segment) the hardware dispatcher hands out workgroups in
// launch order as slots free up, so launching the longest series first is the
// longest-processing-time-first schedule, and series of similar length share
// a wave.  The order is computed once per batch (its lengths are inputs).
#include "dispatch.hpp"

namespace tvi {

constexpr int kOrderThreads = 256;
constexpr int kOrderTile = 1024;

// rank(b) = #{c : N_c > N_b, or N_c == N_b and c < b}; order[rank(b)] = b.
// Lengths are staged through LDS one tile at a time; each thread ranks one series.
__global__ __launch_bounds__(kOrderThreads) void order_kernel(const int64_t *__restrict__ offsets, int64_t B,
                                                             int32_t *__restrict__ order)
{
    __shared__ int64_t len[kOrderTile];
    const int64_t b = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x;
    const int64_t nb = b < B ? offsets[b + 1] - offsets[b] : 0;
    int64_t rank = 0;
    for (int64_t c0 = 0; c0 < B; c0 += kOrderTile) {
        const int64_t cn = min((int64_t)kOrderTile, B - c0);
        __syncthreads();
        for (int64_t i = threadIdx.x; i < cn; i += kOrderThreads) len[i] = offsets[c0 + i + 1] - offsets[c0 + i];
        __syncthreads();
        for (int64_t i = 0; i < cn; ++i) {
            const int64_t c = c0 + i, nc = len[i];
            rank += (nc > nb || (nc == nb && c < b)) ? 1 : 0;
        }
    }
    if (b < B) order[rank] = (int32_t)b;
}

tvi_status launch_order(const int64_t *offsets, int64_t B, int32_t *order, hipStream_t stream)
{
    const int64_t blocks = (B + kOrderThreads - 1) / kOrderThreads;
    hipLaunchKernelGGL(order_kernel, dim3((unsigned)blocks), dim3(kOrderThreads), 0, stream, offsets, B, order);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

} // namespace tvi
