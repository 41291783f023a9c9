// Chunked backward Euler for the neural-ODE model (n = 8, two tanh layers of
// 64, shared parameters): one workgroup of four waves per series.
//
// Per Newton iteration (Algorithm 1):
//   * each wave evaluates the network for its 32 steps of the chunk on MFMA
//     (hidden units along M, steps along N) and stores h(y_j) in LDS;
//   * the residual R_j = dy_j - dy_{j-1} - dt_j h(y_j) and its norm are formed
//     per step (one lane per step) and reduced over the workgroup;
//   * the state Jacobians of the 32 steps come from the same activations on
//     MFMA, every lane inverts its 8x8 block D_j = I - dt_j J_j (partial
//     pivoting, float) and the affine maps are composed by PCR across the
//     32 lanes of the wave and then across the four waves through LDS.
// The chunk start state is carried in double, the increments dy in float.
#include "dispatch.hpp"
#include "mlp.hpp"

namespace tvi {

using namespace mlp;

struct MlpShared {
    Weights W;
    float y[kMaxChunk][NS];     // network input of each step
    float f[kMaxChunk][NS];     // network output of each step
    float J[kMaxChunk][NS * NS];
    float dy[kMaxChunk][NS];
    float wmap[kWaves][NS * NS + NS];
    float red[kWaves];
    int flag[kWaves];
};

// Evaluate the network for the block's steps: every wave its 32 steps.
__device__ __forceinline__ void mlp_rates(MlpShared &S, Acts &A)
{
    const int w = threadIdx.x / kWave, r = lane_id() & 15;
    forward<true>(
        S.W, A,
        [&](int u, float (&y)[8]) {
#pragma unroll
            for (int e = 0; e < 8; ++e) y[e] = S.y[kSPW * w + 16 * u + r][e];
        },
        [&](int u, int row, float v) { S.f[kSPW * w + 16 * u + r][row] = v; });
}

template <class IO>
__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(SolveArgs<IO> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    const int tid = threadIdx.x, w = tid / kWave, l = lane_id();
    const int j = kSPW * w + (l & (kSPW - 1));   // step of the chunk owned by this lane (0-based)
    const bool writer = l < kSPW;                 // lanes 32..63 duplicate lanes 0..31
    const int64_t b = blockIdx.x;
    const SeriesView<IO> sv(a, b);
    const int C = a.chunk;

    load_weights(S.W, a.params);
    double ys[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) ys[k] = ld(a.y0 + b * NS + k);
    IO *yb = a.y ? a.y + sv.p0 * NS : nullptr;
    double *ck = a.ckpt ? a.ckpt + b * a.K * NS : nullptr;
    if (tid < NS) {
        if (yb) st(yb + tid, ys[tid]);
        if (ck) ck[tid] = ys[tid];
    }
    __syncthreads();

    int64_t s = 0;
    int mcur = C, m = 0, it = 0, total = 0, status = ST_OK;
    bool start = true, sing = false;
    float nrm0 = 0.f, dy[NS], tj = 0.f, hj = 0.f;
    Acts A;
    while (s < sv.Nb) {
        if (start) {
            const int64_t nom_end = min((s / C + 1) * (int64_t)C, sv.Nb);
            m = (int)min((int64_t)mcur, nom_end - s);
            const bool v = j < m;
            const double ts = ld(sv.t + s);
            const double t1 = ld(sv.t + (v ? s + j + 1 : s)), t0 = ld(sv.t + (v ? s + j : s));
            hj = (float)(t1 - t0);
            tj = (float)(t1 - ts);
#pragma unroll
            for (int k = 0; k < NS; ++k) dy[k] = 0.f;
            if (a.init == INIT_EXTRAP) {
                // the slope of the last step: h(y_s) for backward Euler
                if (writer) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) S.y[j][k] = (float)ys[k];
                }
                __syncthreads();
                mlp_rates(S, A);
                __syncthreads();
                if (v) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) dy[k] = tj * S.f[j][k];
                }
            }
            it = 0;
            sing = false;
            start = false;
        }
        const bool v = j < m;

        // ---- residual of the current iterate
        if (writer) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                S.y[j][k] = (float)(ys[k] + (double)dy[k]);
                S.dy[j][k] = dy[k];
            }
        }
        __syncthreads();
        mlp_rates(S, A);
        __syncthreads();
        float R[NS], acc = 0.f;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const float prev = j > 0 ? S.dy[j - 1][k] : 0.f;
            R[k] = v ? (dy[k] - prev) - hj * S.f[j][k] : 0.f;
            acc = fmaf(R[k], R[k], acc);
        }
        acc = seg_sum<kSPW>(acc);
        if (l == 0) S.red[w] = acc;
        __syncthreads();
        const float nrm = sqrtf(S.red[0] + S.red[1] + S.red[2] + S.red[3]);

        int act, code = ST_OK;
        if (it == 0) nrm0 = nrm;
        if (sing) { act = 2; code = ST_SINGULAR; }
        else if (!finite(nrm)) { act = 2; code = ST_NONFINITE; }
        else if ((double)nrm <= a.tol_a || (double)nrm <= a.tol_r * (double)nrm0) act = 1;
        else if (it >= a.max_newton) { act = 2; code = ST_NOT_CONVERGED; }
        else act = 3;

        if (act == 1) {
            if (writer && v && yb) {
#pragma unroll
                for (int k = 0; k < NS; ++k) st(yb + (s + j + 1) * NS + k, ys[k] + (double)dy[k]);
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) ys[k] += (double)S.dy[m - 1][k];
            s += m;
            if ((s % C == 0 || s >= sv.Nb) && ck && tid < NS) {
                const int64_t c = (s + C - 1) / C;
                if (c < a.K) ck[c * NS + tid] = ys[tid];
            }
            if (s % C == 0) mcur = C;
            start = true;
            __syncthreads();
            continue;
        }
        if (act == 2) {
            if (a.halving && m > 1) {
                mcur = (m + 1) / 2;
                start = true;
                __syncthreads();
                continue;
            }
            status = code;
            if (yb) {
                const double nan = __builtin_nan("");
                for (int64_t k = s + 1 + tid; k <= sv.Nb; k += kThreads)
#pragma unroll
                    for (int e = 0; e < NS; ++e) st(yb + k * NS + e, nan);
            }
            break;
        }

        // ---- Newton correction
        {
            const int r = l & 15;
            jacobian<false>(S.W, A, [&](int u, int row, int c, float val) {
                S.J[kSPW * w + 16 * u + r][row * NS + c] = val;
            });
        }
        __syncthreads();
        Affine<NS, float> map;
        affine_identity(map);
        int ok = 1;
        if (v) {
            float D[NS][NS];
#pragma unroll
            for (int r = 0; r < NS; ++r)
#pragma unroll
                for (int c = 0; c < NS; ++c) D[r][c] = ((r == c) ? 1.f : 0.f) - hj * S.J[j][r * NS + c];
            ok = invert(D, map.M) ? 1 : 0;
            float negR[NS], zero[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) { negR[k] = -R[k]; zero[k] = 0.f; }
            matvec_add(map.M, negR, zero, map.z);
        }
        seg_scan_up<NS, kSPW>(map);
        ok = seg_and<kWave>(ok);
        if (l == kSPW - 1) {
#pragma unroll
            for (int r = 0; r < NS; ++r) {
#pragma unroll
                for (int c = 0; c < NS; ++c) S.wmap[w][r * NS + c] = map.M[r][c];
                S.wmap[w][NS * NS + r] = map.z[r];
            }
        }
        if (l == 0) S.flag[w] = ok;
        __syncthreads();
        // the correction entering this wave: the maps of the earlier waves applied to 0
        float vin[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) vin[k] = 0.f;
        for (int q = 0; q < w; ++q) {
            float t[NS];
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                float acc2 = S.wmap[q][NS * NS + r];
#pragma unroll
                for (int c = 0; c < NS; ++c) acc2 = fmaf(S.wmap[q][r * NS + c], vin[c], acc2);
                t[r] = acc2;
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) vin[k] = t[k];
        }
        if (v) {
            float d[NS];
            matvec_add(map.M, vin, map.z, d);
#pragma unroll
            for (int k = 0; k < NS; ++k) dy[k] += d[k];
        }
        const int all_ok = S.flag[0] & S.flag[1] & S.flag[2] & S.flag[3];
        ++it;
        ++total;
        if (!all_ok) sing = true;
        __syncthreads();
    }
    if (tid == 0) {
        a.status[b] = status;
        if (a.iters) a.iters[b] = total;
    }
}

// h(y) and dh/dy for M independent states: 128 states per workgroup.
template <class IO>
__global__ __launch_bounds__(kThreads) void mlp_eval_kernel(int64_t M, const IO *states, const IO *params, IO *f,
                                                            IO *J)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    const int tid = threadIdx.x, w = tid / kWave, l = lane_id(), r = l & 15;
    const int64_t base = (int64_t)blockIdx.x * kMaxChunk;
    load_weights(S.W, params);
    for (int idx = tid; idx < kMaxChunk * NS; idx += kThreads) {
        const int64_t q = base + idx / NS;
        S.y[idx / NS][idx % NS] = q < M ? (float)states[q * NS + idx % NS] : 0.f;
    }
    __syncthreads();
    Acts A;
    mlp_rates(S, A);
    jacobian<true>(S.W, A, [&](int u, int row, int c, float val) {
        S.J[kSPW * w + 16 * u + r][row * NS + c] = val;
    });
    __syncthreads();
    for (int idx = tid; idx < kMaxChunk * NS; idx += kThreads) {
        const int64_t q = base + idx / NS;
        if (q < M && f) f[q * NS + idx % NS] = (IO)S.f[idx / NS][idx % NS];
    }
    for (int idx = tid; idx < kMaxChunk * NS * NS; idx += kThreads) {
        const int64_t q = base + idx / (NS * NS);
        if (q < M && J) J[q * NS * NS + idx % (NS * NS)] = (IO)S.J[idx / (NS * NS)][idx % (NS * NS)];
    }
}

size_t mlp_shared_bytes() { return sizeof(MlpShared); }

template <class IO>
static tvi_status mlp_launch(int pass, const SolveArgs<IO> &a, hipStream_t stream)
{
    if (a.B == 0) return TVI_OK;
    const size_t shm = sizeof(MlpShared);
    if (pass == PASS_FORWARD) {
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void *)mlp_forward_kernel<IO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm) != hipSuccess)
                return TVI_EHIP;
            attr = true;
        }
        hipLaunchKernelGGL(mlp_forward_kernel<IO>, dim3((unsigned)a.B), dim3(kThreads), shm, stream, a);
        return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
    }
    return TVI_EUNSUPPORTED;
}

tvi_status launch_mlp(int pass, int dtype, const void *args, hipStream_t stream)
{
    if (dtype == TVI_F64) return mlp_launch<double>(pass, *static_cast<const SolveArgs<double> *>(args), stream);
    return mlp_launch<float>(pass, *static_cast<const SolveArgs<float> *>(args), stream);
}

tvi_status launch_mlp_eval(int dtype, int64_t M, const void *states, const void *params, void *f, void *J,
                           hipStream_t stream)
{
    if (M == 0) return TVI_OK;
    const size_t shm = sizeof(MlpShared);
    const int64_t blocks = (M + kMaxChunk - 1) / kMaxChunk;
    if (blocks > 0x7fffffffLL) return TVI_EINVAL;
    if (dtype == TVI_F64) {
        hipFuncSetAttribute((const void *)mlp_eval_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
        hipLaunchKernelGGL(mlp_eval_kernel<double>, dim3((unsigned)blocks), dim3(kThreads), shm, stream, M,
                           static_cast<const double *>(states), static_cast<const double *>(params),
                           static_cast<double *>(f), static_cast<double *>(J));
    } else {
        hipFuncSetAttribute((const void *)mlp_eval_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
        hipLaunchKernelGGL(mlp_eval_kernel<float>, dim3((unsigned)blocks), dim3(kThreads), shm, stream, M,
                           static_cast<const float *>(states), static_cast<const float *>(params),
                           static_cast<float *>(f), static_cast<float *>(J));
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

} // namespace tvi
