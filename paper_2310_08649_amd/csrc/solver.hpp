// Chunked backward-Euler Newton solver and its discrete adjoint, one
// wavefront segment of S lanes per series.
//
// Tiling.  A chunk of m <= S*T steps is spread over the S lanes of a segment,
// lane q owning the T consecutive steps q*T+1 .. q*T+T.  Every Newton
// iteration (Algorithm 1, Eq. batched-update):
//   1. each lane evaluates the residual of its steps (Eq. batched-backward-
//      euler), R_j = dy_j - dy_{j-1} - dt_j h(y_s + dy_j, t_{s+j});
//      ||R||^2 is summed over the segment by DPP exchanges;
//   2. each lane forms its diagonal blocks D_j = I - dt_j j_j, inverts them
//      (kept as I + F) and composes its T rows serially into one affine map
//      (the in-lane part is Thomas's algorithm, Alg. thomas);
//   3. log2(S) parallel-cyclic-reduction levels (Section 3.2) compose the
//      lane maps across the segment by DPP lane moves;
//   4. each lane takes the correction of its rows (T = 1: the composed map's
//      offset; T > 1: a replay from the value entering the lane).
// S = 1 is the one-series-per-lane sequential solver (chunk = 1) or
// per-lane Thomas; T = 1 is pure PCR.
//
// FE instances integrate the explicit scheme (Eq. forward-euler) the same
// way: the chunk residual is R_j = dy_j - dy_{j-1} - dt_j h(y_s + dy_{j-1},
// t_{s+j-1}), the chunk Jacobian has identity diagonal blocks and
// sub-diagonal blocks -(I + dt_j j(y_{j-1})), so the correction is the affine
// recurrence delta_j = (I + dt_j j_{j-1}) delta_{j-1} - R_j: the same maps and
// scans, with no block inverse.  Newton on this lower-triangular system makes
// the chunk exact after at most m corrections (one for a linear h).
//
// Control flow is flattened into one wave-uniform loop so that series of a
// wave that converge, fail, halve their chunk or finish at different times
// never leave a cross-lane read divergent.
#pragma once

#include "device.hpp"
#include "models.hpp"

namespace tvi {

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_SINGULAR = 2, ST_NONFINITE = 3 };
enum : int { INIT_ZERO = 0, INIT_EXTRAP = 1, INIT_PREDICTOR = 2 };

template <class IO>
struct SolveArgs {
    int64_t B, N, K;           // series, steps (uniform) / max steps, checkpoints per series
    const int64_t *offsets;    // point offsets [B+1] or null
    const IO *times, *y0, *params;
    int32_t params_shared;
    IO *y;                     // trajectory (forward output / adjoint input) or null
    double *ckpt;              // [B][K][n] or null
    int32_t *status, *iters;
    int32_t chunk, max_newton, init, halving;
    int32_t max_newton_chunk;  // corrections per attempt of more than one step (0: max_newton)
    double tol_a, tol_r;
    const IO *g;               // adjoint: dL/dy
    IO *dLdp, *dLdy0;
    double *ws;                // adjoint recompute workspace [B][chunk][n]
    const float *pred;         // learned chunk predictor, inference layout (INIT_PREDICTOR)
    int32_t pred_hidden, pred_steps, pred_base;
    const int32_t *order;      // launch slot -> series (longest first), or null
    int32_t scheme;            // 0 backward Euler, 1 forward Euler (selects the instance)
    int32_t zero_ref;          // 1: the relative test measures against ||R(dy = 0)|| (Alg. 1's n0)
};

template <class IO>
struct SeriesView {
    int64_t b, p0, Nb;
    const IO *t;
    bool valid;
    // slot: the launch position; with an order the series is order[slot]
    // (entries outside [0, B) leave the slot idle)
    __device__ __forceinline__ SeriesView(const SolveArgs<IO> &a, int64_t slot) : b(slot)
    {
        if (a.order && slot < a.B) b = a.order[slot];
        valid = b >= 0 && b < a.B && slot < a.B;
        if (!valid) { b = 0; p0 = 0; Nb = 0; t = a.times; return; }
        if (a.offsets) {
            p0 = a.offsets[b];
            Nb = a.offsets[b + 1] - p0 - 1;
            t = a.times + p0;
        } else {
            p0 = b * (a.N + 1);
            Nb = a.N;
            t = a.times;
        }
    }
};

// Where converged states go: the trajectory and checkpoints (forward) or the
// per-series recompute workspace (adjoint).
template <class IO, int N>
struct TrajectorySink {
    IO *y;       // series' first point, or null
    double *ck;  // series' checkpoints, or null
    int64_t Nb;
    int64_t K;   // checkpoints per series
    int32_t C;
    __device__ __forceinline__ void put(int64_t k, const double (&v)[N]) const
    {
        if (y) {
#pragma unroll
            for (int i = 0; i < N; ++i) st(y + k * N + i, v[i]);
        }
    }
    // c: index of the checkpoint (the chunk boundary just reached, or the end)
    __device__ __forceinline__ void boundary(int64_t c, const double (&v)[N], int q) const
    {
        if (ck && q == 0 && c < K) {
#pragma unroll
            for (int i = 0; i < N; ++i) ck[c * N + i] = v[i];
        }
    }
    template <int S>
    __device__ __forceinline__ void fail(int64_t s, int q) const
    {
        if (!y) return;
        const double nan = __builtin_nan("");
        for (int64_t k = s + 1 + q; k <= Nb; k += S)
#pragma unroll
            for (int i = 0; i < N; ++i) st(y + k * N + i, nan);
    }
};

template <int N>
struct WorkspaceSink {
    double *w;   // series' workspace [chunk][N]
    int64_t c0;  // first step of the nominal chunk being recomputed
    __device__ __forceinline__ void put(int64_t k, const double (&v)[N]) const
    {
#pragma unroll
        for (int i = 0; i < N; ++i) w[(k - c0 - 1) * N + i] = v[i];
    }
    __device__ __forceinline__ void boundary(int64_t, const double (&)[N], int) const {}
    template <int S>
    __device__ __forceinline__ void fail(int64_t, int) const {}
};

// The learned chunk predictor as the solver sees it: network parameters in
// the inference layout (W1^T[n+2][H], b1[H], W2^T[H][H], b2[H],
// W3^T[H][n*steps], b3[n*steps], mean[n+2], std[n+2], float32), the start it
// corrects (0 zero, 1 extrapolation) and the wave's LDS scratch,
// [64/S][2H + n S T] floats.
constexpr int kPredictorMaxTN = 12;  // owned values per lane for which the learned start is compiled

struct PredictorRef {
    const float *p;
    int H, steps, base;
    float *lds;
};

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }

// out[o] = act(b[o] + sum_k Wt[k ld + o] in[k]) for o = o0, o0 + stride, ... < no:
// a layer of the predictor from transposed weights (Wt[K][ld]) and an input
// vector in LDS.  G outputs per pass share every read of `in` and keep G
// independent accumulators (and G loads in flight per k); lanes of a pass
// read neighbouring weights.
template <int G>
__device__ __forceinline__ void dense_t(const float *__restrict__ Wt, int ld, const float *__restrict__ b,
                                        const float *in, int K, int o0, int stride, int no, float *out, bool gelu)
{
    for (int ob = o0; ob < no; ob += G * stride) {
        float acc[G];
        int oi[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            oi[g] = min(ob + g * stride, no - 1);  // clamped: a surplus accumulator is discarded
            acc[g] = b[oi[g]];
        }
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            const float a = in[k];
            const float *w = Wt + (int64_t)k * ld;
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = fmaf(w[oi[g]], a, acc[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (ob + g * stride < no) out[ob + g * stride] = gelu ? gelu_f(acc[g]) : acc[g];
    }
}

// Per-lane state of the chunked Newton solve of one series (FE: the
// forward-Euler chunk system instead of the backward-Euler one).
template <class Model, int S, int T, bool FE = false>
struct ChunkNewton {
    static constexpr int n = Model::N;
    static constexpr bool kPredictorT = T * n <= kPredictorMaxTN;  // register budget of the learned start

    double ys[n];      // state at the chunk start
    int64_t s;         // chunk start step
    int64_t s_end;     // the solve ends when s reaches s_end
    int64_t ck_next;   // index of the next nominal chunk boundary ...
    int64_t ck_at;     // ... and its step (ck_next * C): no division inside the loop
    int m, mcur;       // attempt length and the current limit (halved on failure)
    int it, total;     // corrections in this attempt / in total
    double nrm0;       // squared residual norm at the attempt's first iterate (or at dy = 0)
    double nrm_zero;   // squared residual norm of the attempt at dy = 0
    bool active, start, sing;
    int status;
    double dy[T][n];   // Newton iterate Delta y of the owned steps
    double tt[T], hh[T];
    double t_s, h_s;   // time and first step of the current attempt (predictor features)

    __device__ __forceinline__ bool owned(int q, int i) const { return active && (q * T + i + 1 <= m); }

    // Backward-Euler residual of the chunk at iterate d (owned steps; zero
    // elsewhere), stored in R if KEEP, and its squared Euclidean norm over the
    // segment (the tests compare squares: no square root in the loop).
    // FE: the forward-Euler residual, the rate taken at the previous step.
    // Wave-uniform.
    template <bool KEEP>
    __device__ __forceinline__ double residual(const Model &model, const double (&d)[T][n], int q,
                                               double (&R)[T][n]) const
    {
        double prev[n];
        vec_prev(d[T - 1], prev);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            double yv[n], f[n];
            if constexpr (FE) {
#pragma unroll
                for (int k = 0; k < n; ++k) yv[k] = ys[k] + ((i == 0) ? (q > 0 ? prev[k] : 0.0) : d[i - 1][k]);
                model.rhs(yv, tt[i] - hh[i], f);
            } else {
#pragma unroll
                for (int k = 0; k < n; ++k) yv[k] = ys[k] + d[i][k];
                model.rhs(yv, tt[i], f);
            }
            const bool v = owned(q, i);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                const double dp = (i == 0) ? (q > 0 ? prev[k] : 0.0) : d[i - 1][k];
                const double r = v ? (d[i][k] - dp) - hh[i] * f[k] : 0.0;
                if (KEEP) R[i][k] = r;
                acc = fma(r, r, acc);
            }
        }
        return seg_sum<S>(acc);
    }

    // The extrapolated start: dy_j = (t_{s+j} - t_s) h(y_s) on the owned steps.
    __device__ __forceinline__ void extrapolate(const Model &model, int q, bool zero)
    {
        double slope[n];
        if (zero) {
#pragma unroll
            for (int k = 0; k < n; ++k) slope[k] = 0.0;
        } else {
            model.rhs(ys, t_s, slope);
        }
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const bool v = q * T + i + 1 <= m;
#pragma unroll
            for (int k = 0; k < n; ++k) dy[i][k] = v ? (tt[i] - t_s) * slope[k] : 0.0;
        }
    }

    // The predictor's corrections for the lane's owned steps of the current
    // attempt (chunk start ys, t_s, first step h_s) where `want` (segment-uniform).
    // The S lanes of a segment
    // share the hidden layers and the outputs through LDS; neighbouring lanes
    // compute neighbouring units and read neighbouring (transposed) weights.
    // Every lane of the wave calls it.
    __device__ void predict(const PredictorRef &pr, int q, int seg, bool want, double (&pc)[T][n]) const
    {
        const int H = pr.H, nin = n + 2, nout = n * pr.steps;
        const float *W1 = pr.p, *b1 = W1 + nin * H, *W2 = b1 + H, *b2 = W2 + (int64_t)H * H, *W3 = b2 + H,
                    *b3 = W3 + (int64_t)H * nout, *mu = b3 + nout, *sd = mu + nin;
        float x[n + 2];
#pragma unroll
        for (int k = 0; k < n; ++k) x[k] = (float)ys[k];
        x[n] = (float)t_s;
        x[n + 1] = (float)log(h_s);
#pragma unroll
        for (int k = 0; k < n + 2; ++k) x[k] = (x[k] - mu[k]) / sd[k];
        float *a1 = pr.lds + seg * (2 * H + n * S * T), *a2 = a1 + H, *out = a2 + H;
        for (int u = q; u < H; u += S) {
            float z = b1[u];
#pragma unroll
            for (int k = 0; k < n + 2; ++k) z = fmaf(W1[k * H + u], x[k], z);
            a1[u] = gelu_f(z);
        }
        __syncthreads();
        // fewer accumulators where the solver's own state already fills the registers
        constexpr int G = T == 1 ? 4 : 1;
        dense_t<G>(W2, H, b2, a1, H, q, S, H, a2, true);
        __syncthreads();
        dense_t<G>(W3, nout, b3, a2, H, q, S, want ? m * n : 0, out, false);  // this attempt's outputs (m <= S T)
        __syncthreads();
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = q * T + i;  // 0-based step of the chunk
#pragma unroll
            for (int k = 0; k < n; ++k) pc[i][k] = (want && j < m) ? (double)out[j * n + k] : 0.0;
        }
        __syncthreads();
    }

    // Solve steps s..s_end from ys (already set).  C is the nominal chunk
    // length: attempts never cross a multiple of C, so a checkpoint at every
    // multiple of C restarts the identical sequence of attempts.
    // PRED: this instance carries the learned start (kept out of the others:
    // its registers and code would slow every solve).
    // ZREF: the relative test measures against ||R(dy = 0)|| (instances of their own: the extra
    // residual evaluation would otherwise sit in every solver's loop)
    template <bool PRED, bool ZREF, class IO, class Sink>
    __device__ void run(const Model &model, const IO *t, int C, int max_newton, int max_newton_chunk, double tol_a,
                        double tol_r,
                        int init, bool halving, const Sink &sink, const PredictorRef &pr)
    {
        // the reference of the relative test differs from the first iterate's only for a nonzero start
        const bool ref_zero = ZREF && init != INIT_ZERO;
        nrm_zero = 0.0;
        const int lane = lane_id();
        const int q = lane & (S - 1);
        const int base = lane - q;
        start = true;
        sing = false;
        it = 0;
        nrm0 = 0.0;
        m = 0;
        mcur = C;
        ck_next = s / C + 1;
        ck_at = ck_next * C;
        const double tol_a2 = tol_a * tol_a, tol_r2 = tol_r * tol_r;
        bool fresh = false;  // an attempt whose initial iterate the predictor may still replace

        while (wave_any(active)) {
            // ---- attempt set-up: owned times and the initial iterate (lane-local)
            if (active && start) {
                const int64_t nom_end = min(ck_at, s_end);
                m = (int)min((int64_t)mcur, nom_end - s);
                t_s = ld(t + s);
                h_s = ld(t + s + 1) - t_s;
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const int j = q * T + i + 1;
                    const bool v = j <= m;
                    const int64_t kk = v ? s + j : s;
                    tt[i] = ld(t + kk);
                    const double tp = (i == 0) ? ld(t + (v ? kk - 1 : s)) : tt[i - 1];
                    hh[i] = v ? tt[i] - tp : 0.0;
                }
                extrapolate(model, q, init == INIT_ZERO || (init == INIT_PREDICTOR && pr.base == 0));
                it = 0;
                sing = false;
                start = false;
                fresh = true;
            }

            // ---- learned start: its base (zero or extrapolation) plus the predicted
            // corrections, kept where its residual is below the base's
            // (compiled only into PRED instances with T n <= kPredictorMaxTN)
            if constexpr (PRED && kPredictorT) {
              if (init == INIT_PREDICTOR && wave_any(fresh)) {
                double pc[T][n];
                predict(pr, q, lane / S, fresh, pc);
                double Rt[T][n];  // not kept (KEEP = false)
                const double n_base = residual<false>(model, dy, q, Rt);
#pragma unroll
                for (int i = 0; i < T; ++i)
#pragma unroll
                    for (int k = 0; k < n; ++k) dy[i][k] += (fresh && owned(q, i)) ? pc[i][k] : 0.0;
                const double n_pred = residual<false>(model, dy, q, Rt);
                if (fresh && !(n_pred < n_base)) extrapolate(model, q, pr.base == 0);
              }
            }
            const bool new_attempt = fresh;
            fresh = false;

            // ---- reference residual of a new attempt at dy = 0 (wave-uniform call)
            if constexpr (ZREF) {
              if (ref_zero && wave_any(new_attempt)) {
                double z0[T][n], Rt[T][n];
#pragma unroll
                for (int i = 0; i < T; ++i)
#pragma unroll
                    for (int k = 0; k < n; ++k) z0[i][k] = 0.0;
                const double nz = residual<false>(model, z0, q, Rt);
                if (new_attempt) nrm_zero = nz;
              }
            }

            // ---- residual of the owned steps and its segment norm
            double R[T][n];  // live within this trip only
            const double nrm2 = residual<true>(model, dy, q, R);

            // ---- per-series decision (uniform within the segment)
            int act = 0; // 1 converged, 2 failed, 3 correct
            int code = ST_OK;
            if (active) {
                if (it == 0) nrm0 = ref_zero ? nrm_zero : nrm2;
                if (sing) { act = 2; code = ST_SINGULAR; }
                else if (!finite(nrm2)) { act = 2; code = ST_NONFINITE; }
                else if (nrm2 <= tol_a2 || nrm2 <= tol_r2 * nrm0) act = 1;
                else if (it >= ((m > 1 && max_newton_chunk > 0) ? max_newton_chunk : max_newton)) {
                    act = 2;  // a longer attempt is halved sooner; a single step gets max_newton
                    code = ST_NOT_CONVERGED;
                }
                else act = 3;
            }

            // ---- commit converged chunks
            if (wave_any(act == 1)) {
                const int mm = (act == 1) ? m : 1;
                const int im = (mm - 1) % T, qm = (mm - 1) / T;
                double cand[n];
#pragma unroll
                for (int k = 0; k < n; ++k) cand[k] = dy[0][k];
#pragma unroll
                for (int i = 1; i < T; ++i)
#pragma unroll
                    for (int k = 0; k < n; ++k) cand[k] = (i == im) ? dy[i][k] : cand[k];
                double last[n];
                vec_read(cand, (act == 1) ? base + qm : lane, last);
                if (act == 1) {
#pragma unroll
                    for (int i = 0; i < T; ++i) {
                        if (owned(q, i)) {
                            double v[n];
#pragma unroll
                            for (int k = 0; k < n; ++k) v[k] = ys[k] + dy[i][k];
                            sink.put(s + q * T + i + 1, v);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < n; ++k) ys[k] += last[k];
                    s += m;
                    const bool at_ck = s == ck_at;
                    if (at_ck || s >= s_end) sink.boundary(ck_next, ys, q);
                    if (at_ck) {
                        mcur = C;
                        ++ck_next;
                        ck_at += C;
                    }
                    if (s >= s_end) active = false;
                    start = true;
                }
            }
            if (act == 2) {
                if (halving && m > 1) {
                    mcur = (m + 1) / 2;
                    start = true;
                } else {
                    status = code;
                    active = false;
                    sink.template fail<S>(s, q);
                }
            }

            // ---- Newton correction: blocks, in-lane composition, PCR, replay
            if (wave_any(act == 3)) {
                const bool corr = act == 3;
                double Fi[T][n][n], zi[T][n];
                AffineI<n, double> map;
                affine_identity(map);
                int ok = 1;
                double prev[n];  // FE: the increment at the step before the lane's first
                if constexpr (FE) vec_prev(dy[T - 1], prev);
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    if (corr && owned(q, i)) {
                        if constexpr (FE) {
                            // delta_j = (I + dt_j j(y_{j-1})) delta_{j-1} - R_j
                            double yv[n], J[n][n];
#pragma unroll
                            for (int k = 0; k < n; ++k)
                                yv[k] = ys[k] + ((i == 0) ? (q > 0 ? prev[k] : 0.0) : dy[i - 1][k]);
                            model.jac(yv, tt[i] - hh[i], J);
#pragma unroll
                            for (int r = 0; r < n; ++r) {
#pragma unroll
                                for (int c = 0; c < n; ++c) Fi[i][r][c] = hh[i] * J[r][c];
                                zi[i][r] = -R[i][r];
                            }
                        } else {
                            double yv[n], J[n][n], D[n][n];
#pragma unroll
                            for (int k = 0; k < n; ++k) yv[k] = ys[k] + dy[i][k];
                            model.jac(yv, tt[i], J);
#pragma unroll
                            for (int r = 0; r < n; ++r)
#pragma unroll
                                for (int c = 0; c < n; ++c) D[r][c] = ((r == c) ? 1.0 : 0.0) - hh[i] * J[r][c];
                            ok &= invert_plus(D, Fi[i]) ? 1 : 0;
                            const double zero[n] = {};
                            double negR[n];
#pragma unroll
                            for (int k = 0; k < n; ++k) negR[k] = -R[i][k];
                            apply_ip(Fi[i], negR, zero, zi[i]);
                        }
                        AffineI<n, double> step;
#pragma unroll
                        for (int r = 0; r < n; ++r) {
#pragma unroll
                            for (int c = 0; c < n; ++c) step.F[r][c] = Fi[i][r][c];
                            step.z[r] = zi[i][r];
                        }
                        if (i > 0) affine_after(step, map);
                        map = step;
                    }
                }
                seg_scan_up<n, S>(map);
                if constexpr (T == 1) {
                    // the composed map's offset is the solution at the lane's step
                    if (corr && owned(q, 0)) {
#pragma unroll
                        for (int k = 0; k < n; ++k) dy[0][k] += map.z[k];
                    }
                } else {
                    double din[n];
                    vec_prev(map.z, din);
                    if (q == 0) {
#pragma unroll
                        for (int k = 0; k < n; ++k) din[k] = 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < T; ++i) {
                        if (corr && owned(q, i)) {
                            apply_ip(Fi[i], din, zi[i], din);
#pragma unroll
                            for (int k = 0; k < n; ++k) dy[i][k] += din[k];
                        }
                    }
                }
                ok = seg_and<S>(ok);
                if (corr) {
                    ++it;
                    ++total;
                    if (!ok) sing = true;
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Forward kernel: one segment of S lanes per series, 64 / S series per wave.
// ---------------------------------------------------------------------------
template <class Model, class IO, int S, int T, bool PRED, bool FE = false, bool ZREF = false>
__global__ __launch_bounds__(kWave) void forward_kernel(SolveArgs<IO> a)
{
    constexpr int n = Model::N;
    const int lane = lane_id();
    const int q = lane & (S - 1);
    const SeriesView<IO> sv(a, (int64_t)blockIdx.x * (kWave / S) + lane / S);

    Model model;
    if (sv.valid) model.load(a.params_shared ? a.params : a.params + sv.b * Model::P);

    ChunkNewton<Model, S, T, FE> cn;
    if (sv.valid) {
#pragma unroll
        for (int k = 0; k < n; ++k) cn.ys[k] = ld(a.y0 + sv.b * n + k);
    } else {
#pragma unroll
        for (int k = 0; k < n; ++k) cn.ys[k] = 0.0;
    }
    TrajectorySink<IO, n> sink{a.y ? a.y + sv.p0 * n : nullptr, a.ckpt ? a.ckpt + sv.b * a.K * n : nullptr,
                               sv.Nb, a.K, a.chunk};
    if (sv.valid && q == 0) {
        sink.put(0, cn.ys);
        sink.boundary(0, cn.ys, 0);
    }
    cn.s = 0;
    cn.s_end = sv.Nb;
    cn.total = 0;
    cn.status = ST_OK;
    cn.active = sv.valid && sv.Nb > 0;
    extern __shared__ float pred_lds[];
    cn.template run<PRED, ZREF>(model, sv.t, a.chunk, a.max_newton, a.max_newton_chunk, a.tol_a, a.tol_r, a.init,
                                a.halving != 0, sink,
           PredictorRef{a.pred, a.pred_hidden, a.pred_steps, a.pred_base, pred_lds});
    if (sv.valid && q == 0) {
        a.status[sv.b] = cn.status;
        if (a.iters) a.iters[sv.b] = cn.total;
    }
}

// ---------------------------------------------------------------------------
// Adjoint kernel (Appendix A): nominal chunks in reverse order; the chunk's
// transposed block upper-bidiagonal system (D_j^T lam_j - lam_{j+1} = g_j) is
// the affine recurrence lam_j = D_j^{-T} lam_{j+1} + D_j^{-T} g_j, reduced by
// the same segment scan run from the highest lane down.  With RECOMPUTE the
// chunk's states are re-solved from its checkpoint by the forward code.
// FE: the discrete adjoint of the forward-Euler map,
//   lam_k = (I + dt_{k+1} j(y_k))^T lam_{k+1} + g_k,  lam_{N+1} = 0,
//   dL/dp = sum_k dt_k (dh/dp(y_{k-1}))^T lam_k,  dL/dy0 = g_0 + (I + dt_1 j(y_0))^T lam_1.
// ---------------------------------------------------------------------------
template <class Model, class IO, int S, int T, bool RECOMPUTE, bool PRED, bool FE = false, bool ZREF = false>
__global__ __launch_bounds__(kWave) void adjoint_kernel(SolveArgs<IO> a)
{
    constexpr int n = Model::N;
    constexpr int P = Model::P;
    const int lane = lane_id();
    const int q = lane & (S - 1);
    const int base = lane - q;
    const SeriesView<IO> sv(a, (int64_t)blockIdx.x * (kWave / S) + lane / S);
    const int C = a.chunk;

    Model model;
    if (sv.valid) model.load(a.params + sv.b * P);

    double lam[n], gp[P];
#pragma unroll
    for (int k = 0; k < n; ++k) lam[k] = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) gp[k] = 0.0;

    const IO *gb = a.g + sv.p0 * n;
    const IO *yb = a.y ? a.y + sv.p0 * n : nullptr;
    double *wsb = RECOMPUTE ? a.ws + sv.b * (int64_t)C * n : nullptr;
    int64_t c = sv.valid ? (sv.Nb + C - 1) / C - 1 : -1;
    bool active = c >= 0;
    int status = ST_OK;

    while (wave_any(active)) {
        const int64_t s = active ? c * C : 0;
        const int m = active ? (int)min((int64_t)C, sv.Nb - s) : 0;

        if (RECOMPUTE) {
            ChunkNewton<Model, S, T, FE> cn;
            const bool have_ckpt = active && c < a.K;
            if (active && !have_ckpt) status = ST_NONFINITE;
            cn.active = have_ckpt;
            cn.s = s;
            cn.s_end = s + m;
            cn.total = 0;
            cn.status = ST_OK;
#pragma unroll
            for (int k = 0; k < n; ++k) cn.ys[k] = have_ckpt ? a.ckpt[(sv.b * a.K + c) * n + k] : 0.0;
            WorkspaceSink<n> wsink{wsb, s};
            extern __shared__ float pred_lds[];
            cn.template run<PRED, ZREF>(model, sv.t, C, a.max_newton, a.max_newton_chunk, a.tol_a, a.tol_r, a.init,
                                        a.halving != 0,
                   wsink, PredictorRef{a.pred, a.pred_hidden, a.pred_steps, a.pred_base, pred_lds});
            if (active && cn.status != ST_OK) status = cn.status;
            __syncthreads(); // one wave per block: makes the workspace writes visible to the wave
        }

        // ---- transposed blocks and the in-lane reverse composition
        double Fi[T][n][n], wi[T][n], yl[T][n], hl[T], tl[T];  // I + Fi = D^{-1} (not transposed)
        AffineI<n, double> map;
        affine_identity(map);
        int ok = 1;
#pragma unroll
        for (int i = T - 1; i >= 0; --i) {
            const int j = q * T + i + 1;
            const bool v = active && j <= m;
            const int64_t k = s + (v ? j : 1);
            double gk[n];
#pragma unroll
            for (int e = 0; e < n; ++e) {
                if (RECOMPUTE) yl[i][e] = v ? wsb[(j - 1) * n + e] : 0.0;
                else yl[i][e] = v ? ld(yb + k * n + e) : 0.0;
                gk[e] = v ? ld(gb + k * n + e) : 0.0;
            }
            tl[i] = v ? ld(sv.t + k) : 0.0;
            hl[i] = v ? tl[i] - ld(sv.t + k - 1) : 0.0;
            if (v) {
                if constexpr (FE) {
                    // I + Fi = I + dt_{k+1} j(y_k); nothing follows the series' last step
                    double J[n][n];
                    const double h1 = (k < sv.Nb) ? ld(sv.t + k + 1) - tl[i] : 0.0;
                    model.jac(yl[i], tl[i], J);
#pragma unroll
                    for (int r = 0; r < n; ++r) {
#pragma unroll
                        for (int cc = 0; cc < n; ++cc) Fi[i][r][cc] = h1 * J[r][cc];
                        wi[i][r] = gk[r];
                    }
                } else {
                    double J[n][n], D[n][n];
                    model.jac(yl[i], tl[i], J);
#pragma unroll
                    for (int r = 0; r < n; ++r)
#pragma unroll
                        for (int cc = 0; cc < n; ++cc) D[r][cc] = ((r == cc) ? 1.0 : 0.0) - hl[i] * J[r][cc];
                    ok &= invert_plus(D, Fi[i]) ? 1 : 0;
                    const double zero[n] = {};
                    apply_ip_t(Fi[i], gk, zero, wi[i]);
                }
                AffineI<n, double> stp;
#pragma unroll
                for (int r = 0; r < n; ++r) {
#pragma unroll
                    for (int cc = 0; cc < n; ++cc) stp.F[r][cc] = Fi[i][cc][r];
                    stp.z[r] = wi[i][r];
                }
                if (i < T - 1) affine_after(stp, map);
                map = stp;
            }
        }
        seg_scan_down<n, S>(map);
        // lam at the first owned step of every lane, then the value entering from the right
        double vq[n], lin[n];
        apply_ip(map.F, lam, map.z, vq);
        vec_next(vq, lin);
        if (q == S - 1) {
#pragma unroll
            for (int k = 0; k < n; ++k) lin[k] = lam[k];
        }
        // FE: the state before each owned step (the parameter term is taken there)
        double ybefore[n];
        if constexpr (FE) {
            vec_prev(yl[T - 1], ybefore);
            if (q == 0 && active) {
                const bool have = !RECOMPUTE || c < a.K;  // a missing checkpoint already failed the series
#pragma unroll
                for (int e = 0; e < n; ++e)
                    ybefore[e] = !have ? 0.0 : RECOMPUTE ? a.ckpt[(sv.b * a.K + c) * n + e] : (double)ld(yb + s * n + e);
            }
        }
#pragma unroll
        for (int i = T - 1; i >= 0; --i) {
            const int j = q * T + i + 1;
            if (active && j <= m) {
                apply_ip_t(Fi[i], lin, wi[i], lin);
                double w[n];
#pragma unroll
                for (int k = 0; k < n; ++k) w[k] = hl[i] * lin[k];
                if constexpr (FE) {
                    double yp[n];
#pragma unroll
                    for (int k = 0; k < n; ++k) yp[k] = (i == 0) ? ybefore[k] : yl[i - 1][k];
                    model.vjp_p(yp, tl[i] - hl[i], w, gp);
                } else {
                    model.vjp_p(yl[i], tl[i], w, gp);
                }
            }
        }
        double first[n];
        vec_read(vq, base, first);
        ok = seg_and<S>(ok);
        if (active) {
#pragma unroll
            for (int k = 0; k < n; ++k) lam[k] = first[k];
            if (!ok && status == ST_OK) status = ST_SINGULAR;
            --c;
            if (c < 0) active = false;
        }
    }

    // dL/dy0 = g_0 + lam_1; dL/dp summed over the segment in a fixed order
#pragma unroll
    for (int k = 0; k < P; ++k) gp[k] = seg_sum<S>(gp[k]);
    if (sv.valid && q == 0) {
        const double nan = __builtin_nan("");
        if constexpr (FE) {
            // lam <- (I + dt_1 j(y_0))^T lam_1 (lam_1 = 0 when the series has no step)
            if (sv.Nb > 0) {
                double y0v[n], J[n][n], out[n];
#pragma unroll
                for (int e = 0; e < n; ++e) y0v[e] = RECOMPUTE ? a.ckpt[sv.b * a.K * n + e] : (double)ld(yb + e);
                const double t0 = ld(sv.t), h1 = ld(sv.t + 1) - t0;
                model.jac(y0v, t0, J);
#pragma unroll
                for (int e = 0; e < n; ++e) {
                    double acc = lam[e];
#pragma unroll
                    for (int r = 0; r < n; ++r) acc = fma(h1 * J[r][e], lam[r], acc);
                    out[e] = acc;
                }
#pragma unroll
                for (int e = 0; e < n; ++e) lam[e] = out[e];
            }
        }
#pragma unroll
        for (int k = 0; k < n; ++k) st(a.dLdy0 + sv.b * n + k, status == ST_OK ? ld(gb + k) + lam[k] : nan);
#pragma unroll
        for (int k = 0; k < P; ++k) st(a.dLdp + sv.b * P + k, status == ST_OK ? gp[k] : nan);
        a.status[sv.b] = status;
    }
}

} // namespace tvi
