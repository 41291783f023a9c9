// Chunked backward Euler and its adjoint for the neural-ODE model (n = 8, two
// tanh layers of 64, shared parameters): one workgroup of four waves per series.
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
//
// Adjoint (Appendix A): nominal chunks in reverse; the chunk's states are
// re-solved from its checkpoint by the same code (or read from the
// trajectory), the transposed blocks D_j^T are inverted and reduced from the
// last step down, and lam_j is back-propagated through the network on MFMA to
// accumulate dL/dtheta = sum_j dt_j (dh/dtheta)^T lam_j.  Every workgroup
// writes its series' partial gradient; a second kernel sums the partials over
// the series in a fixed order.
//
// FE instances integrate the explicit scheme (Eq. forward-euler): the network
// is evaluated at the previous step's state (step j reads position j, which
// holds y_{j-1}), the blocks are I + dt_j J(y_{j-1}) with no inverse, and the
// adjoint evaluates position j at y_{s+j}: the map (I + dt_{s+j+1} J(y_{s+j}))^T
// and the parameter term of step s+j+1 share that position's activations.
#include "dispatch.hpp"
#include "grad_input.hpp"
#include "mlp.hpp"

namespace tvi {

using namespace mlp;

constexpr int kRow = H + 1;  // padded row of the sample-major scratch (no bank conflicts)

struct MlpShared {
    Weights W;
    float y[kMaxChunk][NS];     // network input of each step
    float f[kMaxChunk][NS];     // network output of each step (adjoint: dt * lam)
    float dy[kMaxChunk][NS];
    float yc[kMaxChunk][NS];    // converged states of the chunk (adjoint)
    union {
        float J[kMaxChunk][NS * NS];
        struct {
            float a[kWaves][kSPW][kRow];   // activations, sample-major
            float d[kWaves][kSPW][kRow];   // back-propagated deltas, sample-major
        } v;
        float theta[P];
    } u;
    float wmap[kWaves][NS * NS + NS];
    float red[kWaves];
    float lam[NS];
    int flag[kWaves];
};

// Evaluate the network for the block's steps (every wave its 32 steps) from S.y.
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

__device__ __forceinline__ void mlp_jacobians(MlpShared &S, const Acts &A, bool exact)
{
    const int w = threadIdx.x / kWave, r = lane_id() & 15;
    auto put = [&](int u, int row, int c, float val) { S.u.J[kSPW * w + 16 * u + r][row * NS + c] = val; };
    if (exact) jacobian<true>(S.W, A, put);
    else jacobian<false>(S.W, A, put);
}

// Where the converged states of a chunk go.
template <class IO>
struct MlpTrajectorySink {
    IO *y;       // series' first point or null
    double *ck;  // series' checkpoints or null
    int64_t K, Nb;
    int C;
    __device__ void put(int64_t k, const double (&ys)[NS], const float (&dy)[NS]) const
    {
        if (y) {
#pragma unroll
            for (int e = 0; e < NS; ++e) st(y + k * NS + e, ys[e] + (double)dy[e]);
        }
    }
    // c: index of the checkpoint (the chunk boundary just reached, or the end)
    __device__ void boundary(int64_t c, const double (&ys)[NS], int tid) const
    {
        if (ck && tid < NS && c < K) ck[c * NS + tid] = ys[tid];
    }
    __device__ void fail(int64_t s, int tid) const
    {
        if (!y) return;
        const double nan = __builtin_nan("");
        for (int64_t k = s + 1 + tid; k <= Nb; k += kThreads)
#pragma unroll
            for (int e = 0; e < NS; ++e) st(y + k * NS + e, nan);
    }
};

struct MlpChunkSink {
    float (*yc)[NS];
    int64_t c0;
    __device__ void put(int64_t k, const double (&ys)[NS], const float (&dy)[NS]) const
    {
        // the value the trajectory stores (float), as the network sees it
#pragma unroll
        for (int e = 0; e < NS; ++e) yc[k - c0 - 1][e] = (float)(ys[e] + (double)dy[e]);
    }
    __device__ void boundary(int64_t, const double (&)[NS], int) const {}
    __device__ void fail(int64_t, int) const {}
};

// Residual of the chunk iterate dy (Eq. batched-backward-euler; FE: Eq.
// forward-euler) for the lane's step, and its norm over the chunk (block-wide;
// every thread calls it).
template <bool FE = false>
__device__ __forceinline__ float chunk_residual(MlpShared &S, Acts &A, const double (&ys)[NS], const float (&dy)[NS],
                                                float hj, bool v, float (&R)[NS])
{
    const int w = threadIdx.x / kWave, l = lane_id();
    const int j = kSPW * w + (l & (kSPW - 1));
    if (l < kSPW) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if constexpr (FE) {
                // the network input of step j + 1 is this step's state; step 0 reads the chunk start
                if (j + 1 < kMaxChunk) S.y[j + 1][k] = (float)(ys[k] + (double)dy[k]);
                if (j == 0) S.y[0][k] = (float)ys[k];
            } else {
                S.y[j][k] = (float)(ys[k] + (double)dy[k]);
            }
            S.dy[j][k] = dy[k];
        }
    }
    __syncthreads();
    mlp_rates(S, A);
    __syncthreads();
    float acc = 0.f;
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
    __syncthreads();
    return nrm;
}

// The norm alone, with activations of its own (the caller's are not live here).
template <bool FE = false>
__device__ __noinline__ float chunk_residual_norm(MlpShared &S, const double (&ys)[NS], const float (&dy)[NS],
                                                  float hj, bool v)
{
    Acts A;
    float R[NS];
    return chunk_residual<FE>(S, A, ys, dy, hj, v, R);
}

// The learned predictor's corrections for the chunk starting at (ys, ts) with
// first step dts: out[o], o < m * NS, in LDS (block-wide; every thread calls it).
// params in the inference layout: W1^T[NS+2][Hp], b1, W2^T[Hp][Hp], b2,
// W3^T[Hp][NS*steps], b3, mean[NS+2], std[NS+2]; neighbouring threads compute
// neighbouring units and read neighbouring weights.
__device__ void predictor_corrections(float *a1, float *a2, float *out, const float *pp, int Hp, int steps,
                                      const double (&ys)[NS], double ts, double dts, int m)
{
    const int tid = threadIdx.x, nin = NS + 2, nout = NS * steps;
    const float *W1 = pp, *b1 = W1 + nin * Hp, *W2 = b1 + Hp, *b2 = W2 + (int64_t)Hp * Hp, *W3 = b2 + Hp,
                *b3 = W3 + (int64_t)Hp * nout, *mu = b3 + nout, *sd = mu + nin;
    float x[NS + 2];
#pragma unroll
    for (int k = 0; k < NS; ++k) x[k] = (float)ys[k];
    x[NS] = (float)ts;
    x[NS + 1] = (float)log(dts);
#pragma unroll
    for (int k = 0; k < NS + 2; ++k) x[k] = (x[k] - mu[k]) / sd[k];
    for (int o = tid; o < Hp; o += kThreads) {
        float z = b1[o];
#pragma unroll
        for (int k = 0; k < NS + 2; ++k) z = fmaf(W1[k * Hp + o], x[k], z);
        a1[o] = gelu_f(z);
    }
    __syncthreads();
    dense_t<2>(W2, Hp, b2, a1, Hp, tid, kThreads, Hp, a2, true);
    __syncthreads();
    dense_t<2>(W3, nout, b3, a2, Hp, tid, kThreads, m * NS, out, false);
    __syncthreads();
}

// I + F = (I - dt J)^{-1} with F = (I - dt J)^{-1} (dt J), J a row-major block in
// LDS.  F^T if TRANSPOSE.
template <bool TRANSPOSE>
__device__ __forceinline__ bool block_inverse_plus(const float *J, float dt, float (&F)[NS][NS])
{
    // F = (I - dt J)^{-1} (dt J): one Gauss-Jordan solve with right-hand side dt J
    float D[NS][NS], X[NS][NS];
#pragma unroll
    for (int r = 0; r < NS; ++r)
#pragma unroll
        for (int c = 0; c < NS; ++c) {
            const float e = dt * J[r * NS + c];
            D[r][c] = ((r == c) ? 1.f : 0.f) - e;
            X[r][c] = e;
        }
    const bool ok = gj_solve(D, X);
#pragma unroll
    for (int r = 0; r < NS; ++r)
#pragma unroll
        for (int c = 0; c < NS; ++c) {
            if (TRANSPOSE) F[c][r] = X[r][c];
            else F[r][c] = X[r][c];
        }
    return ok;
}

// ||dt J||_inf of a block (J row-major in LDS), and its largest value over the
// wave (every lane calls it: the choice below is wave-uniform; non-finite
// entries count as infinite, so such a block reaches the pivoting inverse and
// its check).
__device__ __forceinline__ float wave_block_norm(const float *J, float dt, bool v)
{
    float en = 0.f;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        float rs = 0.f;
#pragma unroll
        for (int c = 0; c < NS; ++c) rs += fabsf(J[r * NS + c]);
        en = fmaxf(en, rs == rs ? rs : __builtin_inff());  // a NaN block takes the pivoting path
    }
    en = v ? fabsf(dt) * en : 0.f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) en = fmaxf(en, __shfl_xor(en, o));
    return en;
}

// ---------------------------------------------------------------------------
// Row halves of the chunk's affine maps.  Lanes l and l + 32 hold the same step
// of the chunk; each keeps rows 4h..4h+3 (h = l / 32) of the step's map, with
// the columns in the lane's order, its own block first: column p is natural
// column p ^ 4h.  The other half's rows then index the same columns as p ^ 4,
// so every register index stays static, and a composition costs each lane half
// the products of a whole one.  Row i of a half is natural row i ^ 4h too, so
// entry (i, p) of a lane's half is natural entry (i ^ 4h, p ^ 4h).
// ---------------------------------------------------------------------------
struct HalfMap {
    float F[4][NS];
    float z[4];
};

__device__ __forceinline__ bool upper_half() { return (lane_id() & 32) != 0; }
__device__ __forceinline__ float other_half(float x) { return __shfl_xor(x, 32); }

__device__ __forceinline__ void half_identity(HalfMap &a)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) a.F[i][p] = 0.f;
        a.z[i] = 0.f;
    }
}

// A natural-order vector in the lane's order.
__device__ __forceinline__ void lane_order(const float (&x)[NS], float (&y)[NS], bool up)
{
#pragma unroll
    for (int p = 0; p < NS; ++p) y[p] = up ? x[p ^ 4] : x[p];
}

// The natural-order vector whose rows 4h..4h+3 are `own` (the other half
// holding the rest).  Every lane calls it.
__device__ __forceinline__ void join_halves(const float (&own)[4], float (&x)[NS], bool up)
{
    float oth[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) oth[i] = other_half(own[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = up ? oth[i] : own[i];
        x[4 + i] = up ? own[i] : oth[i];
    }
}

// a <- a o b, b the map of another step: b its rows of this half, bo its rows
// of the other half as that half keeps them.
//   F = Fa + Fb + Fa Fb,  z = za + zb + Fa zb
__device__ __forceinline__ void half_after(HalfMap &a, const HalfMap &b, const HalfMap &bo)
{
    float Fn[4][NS], zn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float t = a.z[i] + b.z[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) t = fmaf(a.F[i][k], b.z[k], t);
#pragma unroll
        for (int k = 0; k < 4; ++k) t = fmaf(a.F[i][4 + k], bo.z[k], t);
        zn[i] = t;
#pragma unroll
        for (int p = 0; p < NS; ++p) {
            float u = a.F[i][p] + b.F[i][p];
#pragma unroll
            for (int k = 0; k < 4; ++k) u = fmaf(a.F[i][k], b.F[k][p], u);
#pragma unroll
            for (int k = 0; k < 4; ++k) u = fmaf(a.F[i][4 + k], bo.F[k][p ^ 4], u);
            Fn[i][p] = u;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) a.F[i][p] = Fn[i][p];
        a.z[i] = zn[i];
    }
}

// b <- a moved by a DPP control (zero fill: the identity), bo <- the other
// half's b.  Every lane calls it.
template <int CTRL, int ROWS>
__device__ __forceinline__ void half_move(const HalfMap &a, HalfMap &b, HalfMap &bo)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) b.F[i][p] = dpp_zero<CTRL, ROWS>(a.F[i][p]);
        b.z[i] = dpp_zero<CTRL, ROWS>(a.z[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) bo.F[i][p] = other_half(b.F[i][p]);
        bo.z[i] = other_half(b.z[i]);
    }
}

// Inclusive prefix composition over each 32-lane half, lowest lane first
// (lane q ends with A_q o ... o A_0): row shifts inside 16-lane rows, then
// rows 1 and 3 take the totals of rows 0 and 2 (lanes 15, 47).
__device__ __forceinline__ void half_scan_up(HalfMap &a)
{
    HalfMap b, bo;
    half_move<dpp::ROW_SHR + 1, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHR + 2, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHR + 4, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHR + 8, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_BCAST15, 0xA>(a, b, bo);
    half_after(a, b, bo);
}

// Inclusive suffix composition, highest lane first (lane q ends with
// A_q o ... o A_31): row shifts, then rows 0 and 2 take the totals of rows 1
// and 3 (lanes 16, 48; read by lane broadcast).
__device__ __forceinline__ void half_scan_down(HalfMap &a)
{
    HalfMap b, bo;
    half_move<dpp::ROW_SHL + 1, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHL + 2, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHL + 4, 0xF>(a, b, bo);
    half_after(a, b, bo);
    half_move<dpp::ROW_SHL + 8, 0xF>(a, b, bo);
    half_after(a, b, bo);
    const bool up = upper_half(), take = (lane_id() & 16) == 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) {
            const float lo = lane_bcast(a.F[i][p], 16), hi = lane_bcast(a.F[i][p], 48);
            b.F[i][p] = take ? (up ? hi : lo) : 0.f;
            bo.F[i][p] = take ? (up ? lo : hi) : 0.f;
        }
        const float lo = lane_bcast(a.z[i], 16), hi = lane_bcast(a.z[i], 48);
        b.z[i] = take ? (up ? hi : lo) : 0.f;
        bo.z[i] = take ? (up ? lo : hi) : 0.f;
    }
    half_after(a, b, bo);
}

// This half's rows of F, I + F = (I - E)^{-1} with E = dt J (its transpose if
// TRANSPOSE), in the lane's order.  With eps = ||E||_inf (the wave's largest,
// so the choice is wave-uniform), F = E + E^2 + ... : the terms after E^K sum
// to at most eps^(K+1) / (1 - eps), and ||F|| >= ||E|| / (1 + eps), so cutting
// the series after K terms errs by at most eps^K (1 + eps) / (1 - eps)
// relative to F.  K = 2 (one product) where eps <= 2^-12 and K = 3 (two) where
// eps <= 2^-8 keep that at float rounding (2^-24); a neural ODE over short
// steps is there (dt ||J|| ~ 1e-4).  Beyond, Gauss-Jordan with partial pivoting.
template <bool TRANSPOSE>
__device__ __forceinline__ bool half_inverse_plus(const float *J, float dt, float eps, bool up, float (&Fo)[4][NS])
{
    const int m = up ? 4 : 0;
    if (!(eps <= 0x1p-8f)) {
        float F[NS][NS];
        const bool ok = block_inverse_plus<TRANSPOSE>(J, dt, F);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int p = 0; p < NS; ++p) Fo[i][p] = up ? F[i ^ 4][p ^ 4] : F[i][p];
        return ok;
    }
    // E (or E^T) = dt J in the lane's order: entry (a, b) is natural (a ^ m, b ^ m)
    float E[NS][NS];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b < NS; ++b)
            E[a][b] = dt * (TRANSPOSE ? J[(b ^ m) * NS + (a ^ m)] : J[(a ^ m) * NS + (b ^ m)]);
    // Q = this half's rows of E E; F = E + Q (two terms) or E + Q + Q E (three)
    float Q[4][NS];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int p = 0; p < NS; ++p) {
            float t = 0.f;
#pragma unroll
            for (int k = 0; k < NS; ++k) t = fmaf(E[i][k], E[k][p], t);
            Q[i][p] = t;
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int p = 0; p < NS; ++p) {
            float t = E[i][p] + Q[i][p];
            if (eps > 0x1p-12f) {
#pragma unroll
                for (int k = 0; k < NS; ++k) t = fmaf(Q[i][k], E[k][p], t);
            }
            Fo[i][p] = t;
        }
    return true;
}

// y = (I + F) x + c for this half's rows (x in the lane's order, c own rows).
__device__ __forceinline__ void half_apply(const float (&Fo)[4][NS], const float (&xl)[NS], const float (&c)[4],
                                           float (&y)[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float t = c[i] + xl[i];
#pragma unroll
        for (int p = 0; p < NS; ++p) t = fmaf(Fo[i][p], xl[p], t);
        y[i] = t;
    }
}

// Writes a half map's rows into a natural-order (F row-major, then z) buffer.
__device__ __forceinline__ void half_store(const HalfMap &a, float *dst, bool up)
{
    const int m = up ? 4 : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int p = 0; p < NS; ++p) dst[(i ^ m) * NS + (p ^ m)] = a.F[i][p];
        dst[NS * NS + (i ^ m)] = a.z[i];
    }
}

// Backward Euler from step s0 (state ys) to s_end in attempts that never cross
// a multiple of C.  Every thread of the block calls it; returns the status.
template <bool FE, class IO, class Sink>
__device__ int mlp_solve(MlpShared &S, const SolveArgs<IO> &a, const IO *t, double (&ys)[NS], int64_t s0,
                         int64_t s_end, int &total, const Sink &sink)
{
    const int tid = threadIdx.x, w = tid / kWave, l = lane_id();
    const int j = kSPW * w + (l & (kSPW - 1));   // step of the chunk owned by this lane (0-based)
    const bool writer = l < kSPW;                 // lanes 32..63 duplicate lanes 0..31
    const int C = a.chunk;
    int64_t s = s0;
    int mcur = C, m = 0, it = 0, status = ST_OK, accepted = 0;
    bool start = true, sing = false;
    int64_t ck_next = s / C + 1, ck_at = ck_next * C;  // next nominal boundary: no division in the loop
    float nrm0 = 0.f, nrm_zero = 0.f, dy[NS], hj = 0.f;
    // the reference of the relative test: the first iterate's residual, or Alg. 1's n0 = ||R(dy = 0)||
    const bool ref_zero = a.zero_ref != 0 && a.init != INIT_ZERO;
    Acts A;
    while (s < s_end) {
        if (start) {
            const int64_t nom_end = min(ck_at, s_end);
            m = (int)min((int64_t)mcur, nom_end - s);
            const bool v = j < m;
            const double ts = ld(t + s);
            const double t1 = ld(t + (v ? s + j + 1 : s)), t0 = ld(t + (v ? s + j : s));
            hj = (float)(t1 - t0);
            const float tj = (float)(t1 - ts);
#pragma unroll
            for (int k = 0; k < NS; ++k) dy[k] = 0.f;
            if (a.init == INIT_EXTRAP || (a.init == INIT_PREDICTOR && a.pred_base == 1)) {
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
            if (!FE && a.init == INIT_PREDICTOR) {  // not offered with the explicit scheme
                // the learned start: its base (zero or extrapolated increments) plus the
                // predicted corrections, kept only if its residual is below the base's
                float *scratch = &S.u.v.a[0][0][0];
                predictor_corrections(scratch, scratch + 256, scratch + 512, a.pred, a.pred_hidden, a.pred_steps, ys, ts,
                                 ld(t + s + 1) - ts, m);
                float dyp[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) dyp[k] = v ? dy[k] + scratch[512 + j * NS + k] : 0.f;
                const float n_base = chunk_residual_norm(S, ys, dy, hj, v);
                const float n_pred = chunk_residual_norm(S, ys, dyp, hj, v);
                if (n_pred < n_base) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) dy[k] = dyp[k];
                    ++accepted;
                }
            }
            if (ref_zero) {  // block-uniform
                float z0[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) z0[k] = 0.f;
                nrm_zero = chunk_residual_norm<FE>(S, ys, z0, hj, v);
            }
            it = 0;
            sing = false;
            start = false;
        }
        const bool v = j < m;

        // ---- residual of the current iterate
        float R[NS];
        const float nrm = chunk_residual<FE>(S, A, ys, dy, hj, v, R);

        int act, code = ST_OK;
        if (it == 0) nrm0 = ref_zero ? nrm_zero : nrm;
        if (sing) { act = 2; code = ST_SINGULAR; }
        else if (!finite(nrm)) { act = 2; code = ST_NONFINITE; }
        else if ((double)nrm <= a.tol_a || (double)nrm <= a.tol_r * (double)nrm0) act = 1;
        else if (it >= a.max_newton) { act = 2; code = ST_NOT_CONVERGED; }
        else act = 3;

        if (act == 1) {
            if (writer && v) sink.put(s + j + 1, ys, dy);
#pragma unroll
            for (int k = 0; k < NS; ++k) ys[k] += (double)S.dy[m - 1][k];
            s += m;
            const bool at_ck = s == ck_at;
            if (at_ck || s >= s_end) sink.boundary(ck_next, ys, tid);
            if (at_ck) {
                mcur = C;
                ++ck_next;
                ck_at += C;
            }
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
            sink.fail(s, tid);
            break;
        }

        // ---- Newton correction
        mlp_jacobians(S, A, false);
        __syncthreads();
        const float eps = FE ? 0.f : wave_block_norm(S.u.J[j], hj, v);
        const bool up = upper_half();
        HalfMap map;
        half_identity(map);
        int ok = 1;
        float negR[NS];
        {
            float Rl[NS];
            lane_order(R, Rl, up);
#pragma unroll
            for (int k = 0; k < NS; ++k) negR[k] = -Rl[k];
        }
        if (v) {
            if constexpr (FE) {
                // the correction map x -> (I + dt J(y_{j-1})) x - R
                const int m = up ? 4 : 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
#pragma unroll
                    for (int p = 0; p < NS; ++p) map.F[i][p] = hj * S.u.J[j][(i ^ m) * NS + (p ^ m)];
                    map.z[i] = negR[i];
                }
            } else {
                // (I - dt J)^{-1} = I + F; the correction map x -> (I + F)(x - R)
                ok = half_inverse_plus<false>(S.u.J[j], hj, eps, up, map.F) ? 1 : 0;
                const float zero[4] = {0.f, 0.f, 0.f, 0.f};
                half_apply(map.F, negR, zero, map.z);
            }
        }
        half_scan_up(map);
        ok = seg_and<kWave>(ok);
        if ((l & (kSPW - 1)) == kSPW - 1) half_store(map, S.wmap[w], up);
        if (l == 0) S.flag[w] = ok;
        __syncthreads();
        // the correction entering this wave: the maps of the earlier waves applied to 0
        float vin[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) vin[k] = 0.f;
        for (int q = 0; q < w; ++q) {
            float tv[NS];
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                float acc2 = S.wmap[q][NS * NS + r];
#pragma unroll
                for (int c = 0; c < NS; ++c) acc2 = fmaf(S.wmap[q][r * NS + c], vin[c], acc2);
                tv[r] = acc2 + vin[r];
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) vin[k] = tv[k];
        }
        {
            float vl[NS], dh[4], d[NS];
            lane_order(vin, vl, up);
            half_apply(map.F, vl, map.z, dh);
            join_halves(dh, d, up);
            if (v) {
#pragma unroll
                for (int k = 0; k < NS; ++k) dy[k] += d[k];
            }
        }
        const int all_ok = S.flag[0] & S.flag[1] & S.flag[2] & S.flag[3];
        ++it;
        ++total;
        if (!all_ok) sing = true;
        __syncthreads();
    }
    __syncthreads();
    (void)accepted;
    return status;
}

template <class IO, bool FE>
__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(SolveArgs<IO> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    const int tid = threadIdx.x;
    const SeriesView<IO> sv(a, blockIdx.x);
    if (!sv.valid) return;  // a launch order entry outside [0, B): the whole block idles
    const int64_t b = sv.b;

    load_weights(S.W, a.params);
    double ys[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) ys[k] = ld(a.y0 + b * NS + k);
    MlpTrajectorySink<IO> sink{a.y ? a.y + sv.p0 * NS : nullptr, a.ckpt ? a.ckpt + b * a.K * NS : nullptr, a.K,
                               sv.Nb, a.chunk};
    if (tid < NS && sink.y) st(sink.y + tid, ys[tid]);
    sink.boundary(0, ys, tid);
    __syncthreads();
    int total = 0;
    const int status = mlp_solve<FE>(S, a, sv.t, ys, 0, sv.Nb, total, sink);
    if (tid == 0) {
        a.status[b] = status;
        if (a.iters) a.iters[b] = total;
    }
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

// Gradient accumulators of one wave, in accumulator layout.
struct GradAcc {
    f32x4 w3[5];      // dW3 (rows 0..7 of tiles 0..3) and db3 (column 0 of tile 4)
    f32x4 w2[4][5];   // dW2 (tiles 0..3) and db2 (column 0 of tile 4)
    f32x4 w1[4];      // dW1 (columns 0..7) and db1 (column 8)
};

template <class IO, bool RECOMPUTE, bool FE>
__global__ __launch_bounds__(kThreads) void mlp_adjoint_kernel(SolveArgs<IO> a, float *theta_partial, GradInput gi)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    const int tid = threadIdx.x, w = tid / kWave, l = lane_id(), g = l >> 4, r = l & 15;
    const int j = kSPW * w + (l & (kSPW - 1));
    const bool writer = l < kSPW;
    const SeriesView<IO> sv(a, blockIdx.x);
    if (!sv.valid) return;  // a launch order entry outside [0, B): the whole block idles
    const int64_t b = sv.b;
    const int C = a.chunk;
    // dL/dy at step k (zero at steps that are not observed)
    auto gat = [&](int64_t k, int e) -> float {
        const IO *gp = grad_at(a.g, gi, b, sv.p0, k, NS);
        return gp ? (float)ld(gp + e) : 0.f;
    };
    const float gsc = (float)grad_scale(gi);  // g = (given g) / (*gi.div)

    load_weights(S.W, a.params);
    if (tid < NS) S.lam[tid] = 0.f;
    GradAcc G;
#pragma unroll
    for (int i = 0; i < 5; ++i) G.w3[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        G.w1[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 5; ++i) G.w2[mt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();
    int status = ST_OK;
    const int64_t nck = (sv.Nb + C - 1) / C;
    for (int64_t c = nck - 1; c >= 0; --c) {
        const int64_t c0 = c * C;
        const int m = (int)min((int64_t)C, sv.Nb - c0);
        const bool v = j < m;
        // ---- the chunk's converged states
        if (RECOMPUTE) {
            double ys[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) ys[k] = c < a.K ? a.ckpt[(b * a.K + c) * NS + k] : __builtin_nan("");
            int total = 0;
            const int st2 = mlp_solve<FE>(S, a, sv.t, ys, c0, c0 + m, total, MlpChunkSink{S.yc, c0});
            if (st2 != ST_OK && status == ST_OK) status = st2;
        } else if (writer) {
#pragma unroll
            for (int k = 0; k < NS; ++k) S.yc[j][k] = v ? (float)ld(a.y + (sv.p0 + c0 + j + 1) * NS + k) : 0.f;
        }
        __syncthreads();
        if (writer) {
            if constexpr (FE) {
                // position j holds y_{c0+j}: the chunk start, then the converged states
                float y0c[NS];
                if (j == 0) {
#pragma unroll
                    for (int k = 0; k < NS; ++k)
                        y0c[k] = RECOMPUTE ? (c < a.K ? (float)a.ckpt[(b * a.K + c) * NS + k] : 0.f)
                                           : (float)ld(a.y + (sv.p0 + c0) * NS + k);
                }
#pragma unroll
                for (int k = 0; k < NS; ++k) S.y[j][k] = !v ? 0.f : (j == 0 ? y0c[k] : S.yc[j - 1][k]);
            } else {
#pragma unroll
                for (int k = 0; k < NS; ++k) S.y[j][k] = v ? S.yc[j][k] : 0.f;
            }
        }
        __syncthreads();
        Acts A;
        mlp_rates(S, A);
        mlp_jacobians(S, A, true);
        __syncthreads();

        // ---- transposed blocks and the reduction from the last step down
        const double t1 = ld(sv.t + (v ? c0 + j + 1 : c0)), t0 = ld(sv.t + (v ? c0 + j : c0));
        const float hj = (float)(t1 - t0);
        const float eps = FE ? 0.f : wave_block_norm(S.u.J[j], hj, v);
        const bool up = upper_half();
        HalfMap map;
        half_identity(map);
        int ok = 1;
        if (v) {
            const int mo = up ? 4 : 0;
            if constexpr (FE) {
                // u_j = (I + dt_{c0+j+1} J(y_{c0+j}))^T u_{j+1} + g_{c0+j}: u_j = lam_{c0+j} for
                // j >= 1; u_0 (no g: it belongs to the earlier chunk) is carried
#pragma unroll
                for (int i = 0; i < 4; ++i) {
#pragma unroll
                    for (int p = 0; p < NS; ++p) map.F[i][p] = hj * S.u.J[j][(p ^ mo) * NS + (i ^ mo)];
                    map.z[i] = j == 0 ? 0.f : gsc * gat(c0 + j, i ^ mo);
                }
            } else {
                // (I - dt J)^{-T} = I + F^T
                float gk[NS], gl[NS];
                ok = half_inverse_plus<true>(S.u.J[j], hj, eps, up, map.F) ? 1 : 0;
#pragma unroll
                for (int k = 0; k < NS; ++k) gk[k] = gsc * gat(c0 + j + 1, k);
                lane_order(gk, gl, up);
                const float zero[4] = {0.f, 0.f, 0.f, 0.f};
                half_apply(map.F, gl, zero, map.z);
            }
        }
        half_scan_down(map);
        ok = seg_and<kWave>(ok);
        if ((l & (kSPW - 1)) == 0) half_store(map, S.wmap[w], up);
        if (l == 0) S.flag[w] = ok;
        __syncthreads();
        float lin[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            // FE: the chunk's last step, lam_{c0+m} = g_{c0+m} + the carried value
            lin[k] = S.lam[k];
            if constexpr (FE) lin[k] += gsc * gat(c0 + m, k);
        }
        for (int q = kWaves - 1; q > w; --q) {
            float tv[NS];
#pragma unroll
            for (int rr = 0; rr < NS; ++rr) {
                float acc2 = S.wmap[q][NS * NS + rr];
#pragma unroll
                for (int cc = 0; cc < NS; ++cc) acc2 = fmaf(S.wmap[q][rr * NS + cc], lin[cc], acc2);
                tv[rr] = acc2 + lin[rr];
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) lin[k] = tv[k];
        }
        float lam_j[NS];
        {
            float ll[NS], lh[4];
            lane_order(lin, ll, up);
            half_apply(map.F, ll, map.z, lh);
            join_halves(lh, lam_j, up);
        }
        // FE: the parameter term of step c0+j+1 takes lam_{c0+j+1}, the next position's value
        float lam_w[NS];
        if constexpr (FE) {
            vec_next(lam_j, lam_w);
            if ((l & (kSPW - 1)) == kSPW - 1) {
#pragma unroll
                for (int k = 0; k < NS; ++k) lam_w[k] = lin[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NS; ++k) lam_w[k] = lam_j[k];
        }
        if (!(S.flag[0] & S.flag[1] & S.flag[2] & S.flag[3]) && status == ST_OK) status = ST_SINGULAR;
        __syncthreads();
        // v_j = dt_j lam_j (zero beyond the chunk) into S.f; lam of the chunk's first step carried
        if (writer) {
#pragma unroll
            for (int k = 0; k < NS; ++k) S.f[j][k] = v ? hj * lam_w[k] : 0.f;
        }
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) S.lam[k] = lam_j[k];
        }

        // ---- back-propagation of v through the network (per wave, its 32 samples)
        // activations a2, sample-major
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) S.u.v.a[w][16 * u + r][16 * mt + 4 * g + i] = A.a2[mt][u][i];
        __syncthreads();
        // dW3 += v a2^T (M = state rows, K = samples, N = hidden), db3 from a ones column
        {
            float av[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = r < NS ? S.f[kSPW * w + 8 * g + e][r & (NS - 1)] : 0.f;
            const Split as = split8(av);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                float bv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = S.u.v.a[w][8 * g + e][16 * nt + r];
                G.w3[nt] = mma_acc<true>(as, split8(bv), G.w3[nt]);
            }
            float ones[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) ones[e] = r == 0 ? 1.f : 0.f;
            G.w3[4] = mma_acc<true>(as, split8(ones), G.w3[4]);
        }
        // delta2 = (W3^T v) * (1 - a2^2): M = hidden, K = state rows (k = 8 g + e < 8), N = samples
        f32x4 d2[4][2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = g == 0 ? S.f[kSPW * w + 16 * u + r][e] : 0.f;
            const Split bs = split8(bv);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 z = mma_acc<true>(split_lds(S.W.w3t[mt][l]), bs, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int i = 0; i < 4; ++i) d2[mt][u][i] = z[i] * (1.f - A.a2[mt][u][i] * A.a2[mt][u][i]);
            }
        }
        __syncthreads();
        // a1 and delta2, sample-major
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    S.u.v.a[w][16 * u + r][16 * mt + 4 * g + i] = A.a1[mt][u][i];
                    S.u.v.d[w][16 * u + r][16 * mt + 4 * g + i] = d2[mt][u][i];
                }
        __syncthreads();
        // dW2 += delta2 a1^T, db2 from a ones column
        {
            float ones[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) ones[e] = r == 0 ? 1.f : 0.f;
            const Split os = split8(ones);
            Split bsn[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                float bv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = S.u.v.a[w][8 * g + e][16 * nt + r];
                bsn[nt] = split8(bv);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                float av[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = S.u.v.d[w][8 * g + e][16 * mt + r];
                const Split as = split8(av);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) G.w2[mt][nt] = mma_acc<true>(as, bsn[nt], G.w2[mt][nt]);
                G.w2[mt][4] = mma_acc<true>(as, os, G.w2[mt][4]);
            }
        }
        // delta1 = (W2^T delta2) * (1 - a1^2), with delta2 chained from its accumulators
        f32x4 d1[4][2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            Split bk[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                float bv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = d2[2 * ks + (e >> 2)][u][e & 3];
                bk[ks] = split8(bv);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 z = mma_acc<true>(split_lds(S.W.w2t[mt][0][l]), bk[0], f32x4{0.f, 0.f, 0.f, 0.f});
                z = mma_acc<true>(split_lds(S.W.w2t[mt][1][l]), bk[1], z);
#pragma unroll
                for (int i = 0; i < 4; ++i) d1[mt][u][i] = z[i] * (1.f - A.a1[mt][u][i] * A.a1[mt][u][i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) S.u.v.d[w][16 * u + r][16 * mt + 4 * g + i] = d1[mt][u][i];
        __syncthreads();
        // dW1 += delta1 y^T (columns 0..7), db1 from column 8 (ones)
        {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int smp = kSPW * w + 8 * g + e;
                bv[e] = r < NS ? S.y[smp][r & (NS - 1)] : (r == NS ? 1.f : 0.f);
            }
            const Split bs = split8(bv);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                float av[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = S.u.v.d[w][8 * g + e][16 * mt + r];
                G.w1[mt] = mma_acc<true>(split8(av), bs, G.w1[mt]);
            }
        }
        __syncthreads();
    }

    // ---- dL/dy0 = g_0 + lam_1 (FE: g_0 + the carried (I + dt_1 J(y_0))^T lam_1), and the
    // series' parameter gradient (waves summed in order)
    if (tid < NS) st(a.dLdy0 + b * NS + tid, status == ST_OK ? (double)gsc * (double)gat(0, tid) + (double)S.lam[tid] : __builtin_nan(""));
    for (int idx = tid; idx < P; idx += kThreads) S.u.theta[idx] = 0.f;
    __syncthreads();
    for (int q = 0; q < kWaves; ++q) {
        if (w == q) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 4 * g + i;
                if (row < NS) {
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) S.u.theta[oW3 + row * H + 16 * nt + r] += G.w3[nt][i];
                    if (r == 0) S.u.theta[ob3 + row] += G.w3[4][i];
                }
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int mrow = 16 * mt + 4 * g + i;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) S.u.theta[oW2 + mrow * H + 16 * nt + r] += G.w2[mt][nt][i];
                    if (r == 0) S.u.theta[ob2 + mrow] += G.w2[mt][4][i];
                    if (r < NS) S.u.theta[oW1 + mrow * NS + r] += G.w1[mt][i];
                    if (r == NS) S.u.theta[ob1 + mrow] += G.w1[mt][i];
                }
        }
        __syncthreads();
    }
    const float nanf_ = __builtin_nanf("");
    for (int idx = tid; idx < P; idx += kThreads)
        theta_partial[b * P + idx] = status == ST_OK ? S.u.theta[idx] : nanf_;
    if (tid == 0) a.status[b] = status;
}

// dL/dtheta = sum over series of the partials, in series order.
template <class IO>
__global__ void mlp_theta_reduce_kernel(int64_t B, const float *partial, IO *out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int64_t b = 0; b < B; ++b) s += (double)partial[b * P + p];
    st(out + p, s);
}

// h(y) and dh/dy for M independent states: 128 states per workgroup.
template <class IO>
__global__ __launch_bounds__(kThreads) void mlp_eval_kernel(int64_t M, const IO *states, const IO *params, IO *f,
                                                            IO *J)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpShared &S = *reinterpret_cast<MlpShared *>(smem);
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kMaxChunk;
    load_weights(S.W, params);
    for (int idx = tid; idx < kMaxChunk * NS; idx += kThreads) {
        const int64_t q = base + idx / NS;
        S.y[idx / NS][idx % NS] = q < M ? (float)states[q * NS + idx % NS] : 0.f;
    }
    __syncthreads();
    Acts A;
    mlp_rates(S, A);
    mlp_jacobians(S, A, true);
    __syncthreads();
    for (int idx = tid; idx < kMaxChunk * NS; idx += kThreads) {
        const int64_t q = base + idx / NS;
        if (q < M && f) f[q * NS + idx % NS] = (IO)S.f[idx / NS][idx % NS];
    }
    for (int idx = tid; idx < kMaxChunk * NS * NS; idx += kThreads) {
        const int64_t q = base + idx / (NS * NS);
        if (q < M && J) J[q * NS * NS + idx % (NS * NS)] = (IO)S.u.J[idx / (NS * NS)][idx % (NS * NS)];
    }
}

template <class K>
static bool allow_lds(K kernel)
{
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(MlpShared)) == hipSuccess;
}

size_t mlp_theta_workspace_bytes(int64_t B) { return (size_t)B * P * sizeof(float); }

template <class IO, bool FE>
static tvi_status mlp_launch(int pass, const SolveArgs<IO> &a, hipStream_t stream, const GradInput &gi)
{
    if (a.B == 0) return TVI_OK;
    if (a.B > 0x7fffffffLL) return TVI_EINVAL;
    const size_t shm = sizeof(MlpShared);
    const dim3 grid((unsigned)a.B), block(kThreads);
    switch (pass) {
    case PASS_FORWARD:
        if (!allow_lds(mlp_forward_kernel<IO, FE>)) return TVI_EHIP;
        hipLaunchKernelGGL((mlp_forward_kernel<IO, FE>), grid, block, shm, stream, a);
        break;
    case PASS_ADJOINT:
    case PASS_ADJOINT_RECOMPUTE: {
        float *partial = reinterpret_cast<float *>(a.ws);
        if (pass == PASS_ADJOINT) {
            if (!allow_lds(mlp_adjoint_kernel<IO, false, FE>)) return TVI_EHIP;
            hipLaunchKernelGGL((mlp_adjoint_kernel<IO, false, FE>), grid, block, shm, stream, a, partial, gi);
        } else {
            if (!allow_lds(mlp_adjoint_kernel<IO, true, FE>)) return TVI_EHIP;
            hipLaunchKernelGGL((mlp_adjoint_kernel<IO, true, FE>), grid, block, shm, stream, a, partial, gi);
        }
        if (hipGetLastError() != hipSuccess) return TVI_EHIP;
        hipLaunchKernelGGL(mlp_theta_reduce_kernel<IO>, dim3((P + 255) / 256), dim3(256), 0, stream, a.B,
                           (const float *)partial, a.dLdp);
        break;
    }
    default: return TVI_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

template <class IO>
static tvi_status mlp_launch_scheme(int pass, const SolveArgs<IO> &a, hipStream_t stream, const GradInput &gi)
{
    return a.scheme == 1 ? mlp_launch<IO, true>(pass, a, stream, gi) : mlp_launch<IO, false>(pass, a, stream, gi);
}

tvi_status launch_mlp(int pass, int dtype, const void *args, hipStream_t stream, const GradInput *gi)
{
    const GradInput g = gi ? *gi : GradInput{nullptr, nullptr, 0};
    if (dtype == TVI_F64)
        return mlp_launch_scheme<double>(pass, *static_cast<const SolveArgs<double> *>(args), stream, g);
    return mlp_launch_scheme<float>(pass, *static_cast<const SolveArgs<float> *>(args), stream, g);
}

tvi_status launch_mlp_eval(int dtype, int64_t M, const void *states, const void *params, void *f, void *J,
                           hipStream_t stream)
{
    if (M == 0) return TVI_OK;
    const size_t shm = sizeof(MlpShared);
    const int64_t blocks = (M + kMaxChunk - 1) / kMaxChunk;
    if (blocks > 0x7fffffffLL) return TVI_EINVAL;
    if (dtype == TVI_F64) {
        if (!allow_lds(mlp_eval_kernel<double>)) return TVI_EHIP;
        hipLaunchKernelGGL(mlp_eval_kernel<double>, dim3((unsigned)blocks), dim3(kThreads), shm, stream, M,
                           static_cast<const double *>(states), static_cast<const double *>(params),
                           static_cast<double *>(f), static_cast<double *>(J));
    } else {
        if (!allow_lds(mlp_eval_kernel<float>)) return TVI_EHIP;
        hipLaunchKernelGGL(mlp_eval_kernel<float>, dim3((unsigned)blocks), dim3(kThreads), shm, stream, M,
                           static_cast<const float *>(states), static_cast<const float *>(params),
                           static_cast<float *>(f), static_cast<float *>(J));
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

} // namespace tvi
