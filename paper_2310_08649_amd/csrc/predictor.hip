// Learned chunk predictor: a fully connected network
//   x -> GELU(W1 x + b1) -> GELU(W2 . + b2) -> W3 . + b3
// trained by the library's own kernels (forward, backward of the mean
// squared error, Adam) and evaluated inside the neural-ODE solver to propose
// a chunk's initial Newton iterate.  Float32 on the vector ALUs: tiled
// products with every output element accumulated by one thread in a fixed
// order, so results are deterministic.
#include <algorithm>

#include "dispatch.hpp"

namespace tvi {

namespace pred {

constexpr int TM = 64, TN = 64, TK = 16;   // block tile
constexpr int kThreads = 256;              // 16 x 16 threads, 4 x 4 outputs each

enum Epilogue : int { EP_NONE = 0, EP_BIAS = 1, EP_BIAS_GELU = 2, EP_GELU_GRAD = 3 };

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x)
{
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C[M][N] = op(A) op(B) with op(A)[m][k] = TA ? A[k][m] : A[m][k] (leading
// dimension lda) and op(B)[k][n] = TB ? B[n][k] : B[k][n].  Epilogues:
//   EP_BIAS       C = acc + bias[n]
//   EP_BIAS_GELU  Z = acc + bias[n] (stored to Zout), C = gelu(Z)
//   EP_GELU_GRAD  C = acc * gelu'(Zin[m][n])
template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                        int ldc, int epilogue, const float *__restrict__ bias,
                                                        const float *__restrict__ Zin, float *__restrict__ Zout)
{
    __shared__ float As[TK][TM + 1];
    __shared__ float Bs[TK][TN + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int idx = threadIdx.x; idx < TM * TK; idx += kThreads) {
            const int mm = idx / TK, kk = idx % TK;
            const int m = m0 + mm, k = k0 + kk;
            As[kk][mm] = (m < M && k < K) ? (TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k]) : 0.f;
        }
        for (int idx = threadIdx.x; idx < TN * TK; idx += kThreads) {
            const int nn = idx / TK, kk = idx % TK;
            const int n = n0 + nn, k = k0 + kk;
            Bs[kk][nn] = (n < N && k < K) ? (TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = Bs[kk][tx + 16 * i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fmaf(a[i], b[jj], acc[i][jj]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty + 16 * i;
        if (m >= M) continue;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int n = n0 + tx + 16 * jj;
            if (n >= N) continue;
            float v = acc[i][jj];
            const int64_t o = (int64_t)m * ldc + n;
            if (epilogue == EP_BIAS) {
                v += bias[n];
            } else if (epilogue == EP_BIAS_GELU) {
                v += bias[n];
                Zout[o] = v;
                v = gelu(v);
            } else if (epilogue == EP_GELU_GRAD) {
                v *= gelu_grad(Zin[o]);
            }
            C[o] = v;
        }
    }
}

// column sums s[n] = sum_m X[m][n] (fixed order)
__global__ void colsum_kernel(int M, int N, const float *__restrict__ X, float *__restrict__ s)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float acc = 0.f;
    for (int m = 0; m < M; ++m) acc += X[(int64_t)m * N + n];
    s[n] = acc;
}

// d = 2 (out - target) / (M n_out) in place of out; per-block partial sums of the squared error
__global__ void mse_kernel(int64_t count, float *__restrict__ out, const float *__restrict__ target, float scale,
                           double *__restrict__ partial)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        const float d = out[i] - target[i];
        acc += (double)d * (double)d;
        out[i] = 2.f * scale * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void mse_finish_kernel(int nparts, const double *__restrict__ partial, double scale, float *__restrict__ loss)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nparts; ++i) s += partial[i];
        loss[0] = (float)(s * scale);
    }
}

// Adam (Kingma and Ba): bias-corrected moment estimates
__global__ void adam_kernel(int64_t P, float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float beta1, float beta2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

} // namespace pred
} // namespace tvi

namespace tvi {
namespace pred {

struct Layout {
    int n_in, H, n_out;
    int64_t P;  // network parameters
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, omu, osig;
    Layout(int a, int h, int c) : n_in(a), H(h), n_out(c)
    {
        oW1 = 0;
        ob1 = oW1 + (int64_t)H * n_in;
        oW2 = ob1 + H;
        ob2 = oW2 + (int64_t)H * H;
        oW3 = ob2 + H;
        ob3 = oW3 + (int64_t)n_out * H;
        P = ob3 + n_out;
        omu = P;
        osig = P + n_in;
    }
};

struct Work {
    float *xn, *z1, *a1, *z2, *a2, *out, *d2, *d1;
    double *partial;
};

constexpr int kMseBlocks = 64;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t work_bytes(const Layout &L, int64_t M)
{
    size_t b = 0;
    b += align256(sizeof(float) * M * L.n_in);
    b += 6 * align256(sizeof(float) * M * L.H);
    b += align256(sizeof(float) * M * L.n_out);
    b += align256(sizeof(double) * kMseBlocks);
    return b;
}

static Work carve(const Layout &L, int64_t M, void *ws)
{
    char *p = static_cast<char *>(ws);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    Work w;
    w.xn = (float *)take(sizeof(float) * M * L.n_in);
    w.z1 = (float *)take(sizeof(float) * M * L.H);
    w.a1 = (float *)take(sizeof(float) * M * L.H);
    w.z2 = (float *)take(sizeof(float) * M * L.H);
    w.a2 = (float *)take(sizeof(float) * M * L.H);
    w.d2 = (float *)take(sizeof(float) * M * L.H);
    w.d1 = (float *)take(sizeof(float) * M * L.H);
    w.out = (float *)take(sizeof(float) * M * L.n_out);
    w.partial = (double *)take(sizeof(double) * kMseBlocks);
    return w;
}

__global__ void standardise_kernel(int64_t M, int n_in, const float *__restrict__ x, const float *__restrict__ mu,
                                   const float *__restrict__ sig, float *__restrict__ xn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * n_in) return;
    const int c = (int)(i % n_in);
    xn[i] = (x[i] - mu[c]) / sig[c];
}

template <bool TA, bool TB>
static void gemm(hipStream_t st, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C,
                 int ldc, int ep, const float *bias, const float *Zin, float *Zout)
{
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(kThreads), 0, st, M, N, K, A, lda, B, ldb, C, ldc, ep, bias,
                       Zin, Zout);
}

static void forward(hipStream_t st, const Layout &L, int M, const float *x, const float *th, const Work &w,
                    float *out)
{
    const int64_t cnt = (int64_t)M * L.n_in;
    hipLaunchKernelGGL(standardise_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, (int64_t)M, L.n_in,
                       x, th + L.omu, th + L.osig, w.xn);
    gemm<false, true>(st, M, L.H, L.n_in, w.xn, L.n_in, th + L.oW1, L.n_in, w.a1, L.H, EP_BIAS_GELU, th + L.ob1,
                      nullptr, w.z1);
    gemm<false, true>(st, M, L.H, L.H, w.a1, L.H, th + L.oW2, L.H, w.a2, L.H, EP_BIAS_GELU, th + L.ob2, nullptr,
                      w.z2);
    gemm<false, true>(st, M, L.n_out, L.H, w.a2, L.H, th + L.oW3, L.H, out, L.n_out, EP_BIAS, th + L.ob3, nullptr,
                      nullptr);
}

} // namespace pred

int64_t predictor_param_count(int n_in, int H, int n_out) { return pred::Layout(n_in, H, n_out).P + 2 * n_in; }

namespace pred {
// Inference layout: the three weight matrices transposed (rows of length R
// become columns), everything else copied, offsets unchanged.
__global__ void pack_kernel(int n_in, int H, int n_out, int64_t count, const float *__restrict__ src,
                            float *__restrict__ dst)
{
    const int64_t w1 = 0, b1 = w1 + (int64_t)H * n_in, w2 = b1 + H, b2 = w2 + (int64_t)H * H, w3 = b2 + H,
                  b3 = w3 + (int64_t)n_out * H;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t from = i;
        if (i < b1) {                        // W1^T[k][u] = W1[u][k]
            const int64_t k = (i - w1) / H, u = (i - w1) % H;
            from = w1 + u * n_in + k;
        } else if (i >= w2 && i < b2) {      // W2^T[k][u] = W2[u][k]
            const int64_t k = (i - w2) / H, u = (i - w2) % H;
            from = w2 + u * H + k;
        } else if (i >= w3 && i < b3) {      // W3^T[k][o] = W3[o][k]
            const int64_t k = (i - w3) / n_out, o = (i - w3) % n_out;
            from = w3 + o * H + k;
        }
        dst[i] = src[from];
    }
}
} // namespace pred

tvi_status predictor_pack(int n_in, int H, int n_out, const float *params, float *packed, hipStream_t st)
{
    const int64_t count = predictor_param_count(n_in, H, n_out);
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(pred::pack_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_in, H, n_out, count, params,
                       packed);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

size_t predictor_workspace_bytes(int n_in, int H, int n_out, int64_t M)
{
    const pred::Layout L(n_in, H, n_out);
    return pred::work_bytes(L, M) + pred::align256(sizeof(float) * L.P);
}

tvi_status predictor_forward(int n_in, int H, int n_out, int64_t M, const float *x, const float *params, float *out,
                             void *ws, hipStream_t st)
{
    const pred::Layout L(n_in, H, n_out);
    const pred::Work w = pred::carve(L, M, ws);
    pred::forward(st, L, (int)M, x, params, w, out);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

tvi_status predictor_train_step(int n_in, int H, int n_out, int64_t M, const float *x, const float *target,
                                float *params, float *grad, float *adam_m, float *adam_v, int64_t step, float lr,
                                float *loss, void *ws, hipStream_t st)
{
    using namespace pred;
    const Layout L(n_in, H, n_out);
    const Work w = carve(L, M, ws);
    const int Mi = (int)M;
    forward(st, L, Mi, x, params, w, w.out);
    const int64_t cnt = M * L.n_out;
    const float scale = 1.f / (float)cnt;
    hipLaunchKernelGGL(mse_kernel, dim3(kMseBlocks), dim3(256), 0, st, cnt, w.out, target, scale, w.partial);
    hipLaunchKernelGGL(mse_finish_kernel, dim3(1), dim3(1), 0, st, kMseBlocks, (const double *)w.partial,
                       1.0 / (double)cnt, loss);
    float *g = grad;
    // w.out now holds d3 = dL/dout
    gemm<true, false>(st, L.n_out, L.H, Mi, w.out, L.n_out, w.a2, L.H, g + L.oW3, L.H, EP_NONE, nullptr, nullptr,
                      nullptr);                                                     // gW3 = d3^T a2
    hipLaunchKernelGGL(colsum_kernel, dim3((L.n_out + 255) / 256), dim3(256), 0, st, Mi, L.n_out, w.out, g + L.ob3);
    gemm<false, false>(st, Mi, L.H, L.n_out, w.out, L.n_out, params + L.oW3, L.H, w.d2, L.H, EP_GELU_GRAD, nullptr,
                       w.z2, nullptr);                                              // d2 = (d3 W3) gelu'(z2)
    gemm<true, false>(st, L.H, L.H, Mi, w.d2, L.H, w.a1, L.H, g + L.oW2, L.H, EP_NONE, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(colsum_kernel, dim3((L.H + 255) / 256), dim3(256), 0, st, Mi, L.H, w.d2, g + L.ob2);
    gemm<false, false>(st, Mi, L.H, L.H, w.d2, L.H, params + L.oW2, L.H, w.d1, L.H, EP_GELU_GRAD, nullptr, w.z1,
                       nullptr);                                                    // d1 = (d2 W2) gelu'(z1)
    gemm<true, false>(st, L.H, L.n_in, Mi, w.d1, L.H, w.xn, L.n_in, g + L.oW1, L.n_in, EP_NONE, nullptr, nullptr,
                      nullptr);
    hipLaunchKernelGGL(colsum_kernel, dim3((L.H + 255) / 256), dim3(256), 0, st, Mi, L.H, w.d1, g + L.ob1);
    if (lr != 0.f) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
        hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((L.P + 255) / 256)), dim3(256), 0, st, L.P, params,
                           (const float *)g, adam_m, adam_v, lr, b1, b2, 1e-8f, c1, c2);
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

} // namespace tvi
