// Standalone batched block-bidiagonal solve (Section 3): the linear kernel of
// the chunked Newton update with its blocks materialised in HBM.
//
// System b (of B), m block rows, diagonal blocks D[b][j] (n x n), sub-diagonal
// blocks -I:
//   forward:    D_j x_j - x_{j-1} = r_j          (x_0 = 0)
//   transposed: D_j^T x_j - x_{j+1} = r_j        (x_{m+1} = 0)
// One segment of S lanes per system; lane q owns rows q*T .. q*T+T-1.  Each
// lane inverts its blocks, composes its rows into one affine map, the segment
// runs log2(S) reduction levels (Section 3.2 with B = -I), and each lane
// replays its rows from the value entering it.  Every byte of D and r is read
// once and every byte of x written once.
#include "dispatch.hpp"

namespace tvi {

// Arithmetic precision: double for double storage, float for float storage
// (an HBM-bound solve; the float path is the one the neural ODE's 8 x 8
// blocks take).
template <class IO>
struct Compute {
    using type = double;
};
template <>
struct Compute<float> {
    using type = float;
};

template <int N, class IO, int T>
struct Rows {
    using R = typename Compute<IO>::type;
    R D[T][N][N], r[T][N];
};

// Non-temporal ("streamed") accesses only for 2x2 blocks.  A lane's block row is
// read element by element, so one load instruction touches one element of
// each of 64 rows; with n = 3 or 4 the rows span several cache lines and
// streamed lines are evicted before the lane's later loads reach them
// (measured: 44% more HBM reads and 1.8x the time at n = 4 in FP64).
template <int N>
constexpr bool kStream = N == 2;

template <int N, class T>
__device__ __forceinline__ T load_elem(const T *p)
{
    if constexpr (kStream<N>) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int N, class T>
__device__ __forceinline__ void store_elem(T *p, T v)
{
    if constexpr (kStream<N>) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Loads of a lane's T rows: the data is used once.
template <int N, class IO, int S, int T, bool TR>
__device__ __forceinline__ void load_rows(Rows<N, IO, T> &v, const IO *__restrict__ D, const IO *__restrict__ r,
                                          int64_t b, int m, int q)
{
    const IO *Db = D + b * (int64_t)m * N * N;
    const IO *rb = r + b * (int64_t)m * N;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const int j = q * T + i;
        const bool ok = j < m;
        const int jj = ok ? j : 0;
#pragma unroll
        for (int e = 0; e < N; ++e) {
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const auto val = (typename Compute<IO>::type)load_elem<N>(Db + ((int64_t)jj * N + e) * N + c);
                if (TR) v.D[i][c][e] = val;
                else v.D[i][e][c] = val;
            }
            v.r[i][e] = (typename Compute<IO>::type)load_elem<N>(rb + (int64_t)jj * N + e);
        }
    }
}

// Grid-stride over systems; the rows of the next system are loaded before the
// current one is reduced, so every wave keeps loads in flight.
template <int N, class IO, int S, int T, bool TR>
__global__ __launch_bounds__(kWave) void pcr_kernel(int64_t B, int m, const IO *__restrict__ D,
                                                   const IO *__restrict__ r, IO *__restrict__ x)
{
    using R = typename Compute<IO>::type;
    const int lane = lane_id();
    const int q = lane & (S - 1);
    const int64_t per_block = kWave / S;
    const int64_t stride = (int64_t)gridDim.x * per_block;
    int64_t b = (int64_t)blockIdx.x * per_block + lane / S;

    // prefetching doubles the row registers: only where they are few
    constexpr bool kPrefetch = T * (N * N + N) <= 24;
    Rows<N, IO, T> next;
    if (kPrefetch && b < B) load_rows<N, IO, S, T, TR>(next, D, r, b, m, q);
    for (int64_t b0 = (int64_t)blockIdx.x * per_block; b0 < B; b0 += stride, b += stride) {
        const bool valid = b < B;
        Rows<N, IO, T> cur;
        if (kPrefetch) {
            cur = next;
            if (b + stride < B) load_rows<N, IO, S, T, TR>(next, D, r, b + stride, m, q);
        } else if (valid) {
            load_rows<N, IO, S, T, TR>(cur, D, r, b, m, q);
        }

        R Fi[T][N][N], zi[T][N];  // I + Fi = D^{-1} (of the transposed block when TR)
        AffineI<N, R> map;
        affine_identity(map);
        int ok = 1;
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const int i = TR ? T - 1 - u : u;  // composition order: along the recurrence
            const int j = q * T + i;
            if (valid && j < m) {
                ok &= invert_plus(cur.D[i], Fi[i]) ? 1 : 0;
                const R zero[N] = {};
                apply_ip(Fi[i], cur.r[i], zero, zi[i]);
                AffineI<N, R> stp;
#pragma unroll
                for (int e = 0; e < N; ++e) {
#pragma unroll
                    for (int c = 0; c < N; ++c) stp.F[e][c] = Fi[i][e][c];
                    stp.z[e] = zi[i][e];
                }
                affine_after(stp, map);
                map = stp;
            }
        }
        if (!TR) seg_scan_up<N, S>(map);
        else seg_scan_down<N, S>(map);
        if constexpr (T == 1) {
            // the composed map's offset is the solution at the lane's row
#pragma unroll
            for (int e = 0; e < N; ++e) zi[0][e] = map.z[e];
        } else {
            R din[N];
            if (!TR) vec_prev(map.z, din);
            else vec_next(map.z, din);
            if (q == (TR ? S - 1 : 0)) {
#pragma unroll
                for (int e = 0; e < N; ++e) din[e] = R(0);
            }
#pragma unroll
            for (int u = 0; u < T; ++u) {
                const int i = TR ? T - 1 - u : u;
                const int j = q * T + i;
                if (valid && j < m) {
                    apply_ip(Fi[i], din, zi[i], din);
#pragma unroll
                    for (int e = 0; e < N; ++e) zi[i][e] = din[e];
                }
            }
        }
        ok = seg_and<S>(ok);
        const R nan = R(__builtin_nan(""));
        IO *xb = x + (valid ? b : 0) * (int64_t)m * N;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = q * T + i;
            if (valid && j < m) {
#pragma unroll
                for (int e = 0; e < N; ++e)
                    store_elem<N>(xb + (int64_t)j * N + e, (IO)(ok ? zi[i][e] : nan));
            }
        }
    }
}

template <int N, class IO, int S, int T>
static tvi_status pcr_launch_st(int64_t B, int m, const void *D, const void *r, void *x, int transpose,
                                hipStream_t stream)
{
    const int64_t per_block = kWave / S;
    int64_t blocks = (B + per_block - 1) / per_block;
    if (blocks == 0) return TVI_OK;
    // enough waves to fill every SIMD several times; each then walks the batch
    const int64_t resident = 256 * 4 * 8;
    if (blocks > resident) blocks = resident;
    const IO *Dp = static_cast<const IO *>(D);
    const IO *rp = static_cast<const IO *>(r);
    IO *xp = static_cast<IO *>(x);
    if (transpose)
        hipLaunchKernelGGL((pcr_kernel<N, IO, S, T, true>), dim3((unsigned)blocks), dim3(kWave), 0, stream, B, m,
                           Dp, rp, xp);
    else
        hipLaunchKernelGGL((pcr_kernel<N, IO, S, T, false>), dim3((unsigned)blocks), dim3(kWave), 0, stream, B, m,
                           Dp, rp, xp);
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

template <int N, class IO, int S>
static tvi_status pcr_launch_s(int64_t B, int m, const void *D, const void *r, void *x, int transpose, int T,
                               hipStream_t stream)
{
    switch (T) {
    case 1: return pcr_launch_st<N, IO, S, 1>(B, m, D, r, x, transpose, stream);
    case 2: return pcr_launch_st<N, IO, S, 2>(B, m, D, r, x, transpose, stream);
    case 4: return pcr_launch_st<N, IO, S, 4>(B, m, D, r, x, transpose, stream);
    case 8: return pcr_launch_st<N, IO, S, 8>(B, m, D, r, x, transpose, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

template <int N, class IO>
static tvi_status pcr_launch(int64_t B, int m, const void *D, const void *r, void *x, int transpose, int S, int T,
                             hipStream_t stream)
{
    switch (S) {
    case 1: return pcr_launch_s<N, IO, 1>(B, m, D, r, x, transpose, T, stream);
    case 4: return pcr_launch_s<N, IO, 4>(B, m, D, r, x, transpose, T, stream);
    case 8: return pcr_launch_s<N, IO, 8>(B, m, D, r, x, transpose, T, stream);
    case 16: return pcr_launch_s<N, IO, 16>(B, m, D, r, x, transpose, T, stream);
    case 32: return pcr_launch_s<N, IO, 32>(B, m, D, r, x, transpose, T, stream);
    case 64: return pcr_launch_s<N, IO, 64>(B, m, D, r, x, transpose, T, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

// 8 x 8 blocks (float): one or two rows per lane (the registers of larger T)
static tvi_status pcr_launch8(int64_t B, int m, const void *D, const void *r, void *x, int transpose, int S, int T,
                              hipStream_t stream)
{
    if (T > 2) return TVI_EUNSUPPORTED;
    switch (S) {
    case 4: return T == 1 ? pcr_launch_st<8, float, 4, 1>(B, m, D, r, x, transpose, stream)
                          : pcr_launch_st<8, float, 4, 2>(B, m, D, r, x, transpose, stream);
    case 8: return T == 1 ? pcr_launch_st<8, float, 8, 1>(B, m, D, r, x, transpose, stream)
                          : pcr_launch_st<8, float, 8, 2>(B, m, D, r, x, transpose, stream);
    case 16: return T == 1 ? pcr_launch_st<8, float, 16, 1>(B, m, D, r, x, transpose, stream)
                           : pcr_launch_st<8, float, 16, 2>(B, m, D, r, x, transpose, stream);
    case 32: return T == 1 ? pcr_launch_st<8, float, 32, 1>(B, m, D, r, x, transpose, stream)
                           : pcr_launch_st<8, float, 32, 2>(B, m, D, r, x, transpose, stream);
    case 64: return T == 1 ? pcr_launch_st<8, float, 64, 1>(B, m, D, r, x, transpose, stream)
                           : pcr_launch_st<8, float, 64, 2>(B, m, D, r, x, transpose, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

tvi_status launch_pcr(int dtype, int n, int64_t B, int m, const void *D, const void *r, void *x, int transpose,
                      int S, int T, hipStream_t stream)
{
    const bool f64 = dtype == TVI_F64;
    switch (n) {
    case 2: return f64 ? pcr_launch<2, double>(B, m, D, r, x, transpose, S, T, stream)
                       : pcr_launch<2, float>(B, m, D, r, x, transpose, S, T, stream);
    case 3: return f64 ? pcr_launch<3, double>(B, m, D, r, x, transpose, S, T, stream)
                       : pcr_launch<3, float>(B, m, D, r, x, transpose, S, T, stream);
    case 4: return f64 ? pcr_launch<4, double>(B, m, D, r, x, transpose, S, T, stream)
                       : pcr_launch<4, float>(B, m, D, r, x, transpose, S, T, stream);
    case 8: return f64 ? TVI_EUNSUPPORTED : pcr_launch8(B, m, D, r, x, transpose, S, T, stream);
    default: return TVI_EUNSUPPORTED;
    }
}

} // namespace tvi
