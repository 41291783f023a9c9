// Loss gradients g = dL/dy of the two losses the benchmarks integrate:
//   Frobenius:  L = sqrt(sum y^2) over every entry (the timing loss of Section 5.2),
//               g = y / L;
//   observed mean square: L = sum_{b, k in obs, i} y_{b,k,i}^2 / (B n_obs n) over the
//               observed steps of a uniform grid, g = 2 y / (B n_obs n) there, 0 elsewhere.
// The sum of squares is reduced deterministically: a fixed grid of partial sums,
// then one workgroup adds them in a fixed tree order.
#include "dispatch.hpp"

namespace tvi {

constexpr int kLossBlocks = 1024;
constexpr int kLossThreads = 256;

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// pass 1: partial sums of squares; an entry counts if it is observed (obs == null: all)
template <class IO>
__global__ __launch_bounds__(kLossThreads) void sumsq_kernel(int64_t count, const IO *y, const uint8_t *observed,
                                                             int64_t point_stride, double *partial)
{
    __shared__ double sh[kLossThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kLossThreads) {
        const double v = (double)y[i];
        const bool use = !observed || observed[(i / point_stride)];
        acc += use ? v * v : 0.0;
    }
    const double s = block_sum<kLossThreads>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// pass 2: the loss from the partials (one workgroup)
__global__ __launch_bounds__(kLossThreads) void loss_finish_kernel(const double *partial, int kind, double scale,
                                                                   double *loss)
{
    __shared__ double sh[kLossThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kLossBlocks; i += kLossThreads) acc += partial[i];
    const double s = block_sum<kLossThreads>(acc, sh);
    if (threadIdx.x == 0) loss[0] = kind == TVI_LOSS_FROBENIUS ? sqrt(s) : s * scale;
}

// pass 3: the gradient
template <class IO>
__global__ __launch_bounds__(kLossThreads) void loss_grad_kernel(int64_t count, const IO *y, const uint8_t *observed,
                                                                 int64_t point_stride, int kind, double scale,
                                                                 const double *loss, IO *g)
{
    const double L = loss[0];
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kLossThreads) {
        const double v = (double)y[i];
        double gi;
        if (kind == TVI_LOSS_FROBENIUS) gi = v / L;
        else gi = (!observed || observed[i / point_stride]) ? 2.0 * scale * v : 0.0;
        g[i] = (IO)gi;
    }
}

template <class IO>
static tvi_status loss_launch(int kind, int64_t count, const IO *y, const uint8_t *observed, int64_t point_stride,
                              double scale, IO *g, double *loss, double *partial, hipStream_t stream)
{
    hipLaunchKernelGGL(sumsq_kernel<IO>, dim3(kLossBlocks), dim3(kLossThreads), 0, stream, count, y, observed,
                       point_stride, partial);
    hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(kLossThreads), 0, stream, (const double *)partial, kind,
                       scale, loss);
    if (g)  // g null: the loss value only
        hipLaunchKernelGGL(loss_grad_kernel<IO>, dim3(kLossBlocks), dim3(kLossThreads), 0, stream, count, y, observed,
                           point_stride, kind, scale, (const double *)loss, g);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

// The Frobenius loss from per-series sums of squares (one workgroup, fixed order).
__global__ __launch_bounds__(kLossThreads) void sums_finish_kernel(const double *sums, int64_t B, double *loss)
{
    __shared__ double sh[kLossThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < B; i += kLossThreads) acc += sums[i];
    const double s = block_sum<kLossThreads>(acc, sh);
    if (threadIdx.x == 0) loss[0] = sqrt(s);
}

tvi_status launch_loss_from_sums(const double *sums, int64_t B, double *loss, hipStream_t stream)
{
    hipLaunchKernelGGL(sums_finish_kernel, dim3(1), dim3(kLossThreads), 0, stream, sums, B, loss);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

tvi_status launch_loss(int kind, int dtype, int64_t count, const void *y, const uint8_t *observed,
                       int64_t point_stride, double scale, void *g, double *loss, double *partial,
                       hipStream_t stream)
{
    if (dtype == TVI_F64)
        return loss_launch<double>(kind, count, static_cast<const double *>(y), observed, point_stride, scale,
                                   static_cast<double *>(g), loss, partial, stream);
    return loss_launch<float>(kind, count, static_cast<const float *>(y), observed, point_stride, scale,
                              static_cast<float *>(g), loss, partial, stream);
}

size_t loss_workspace_bytes() { return kLossBlocks * sizeof(double); }

} // namespace tvi
