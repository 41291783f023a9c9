// Block solver: the chunked backward-Euler Newton method (Algorithm 1) and its
// discrete adjoint (Appendix A) for state sizes n up to 40, where an n x n
// block no longer fits one lane's registers.
//
// One workgroup of kWaves wavefronts per series.  The steps of a chunk are
// dealt round-robin to the waves; a wave holds the block of one step with one
// row per lane (n <= 64 rows), padded to NP columns with the identity so that
// every register index is static.  Per Newton iteration:
//   1. residual pass: R_j = dy_j - dy_{j-1} - dt_j h(y_s + dy_j, t_{s+j})
//      (Eq. batched-backward-euler), ||R||^2 summed in a fixed order;
//   2. block pass: row i of D_j = I - dt_j j_j from the model, the block
//      inverted in registers by Gauss-Jordan elimination with partial pivoting
//      (rows stay in their lanes; the pivot order is kept and undone when the
//      inverse is written), M_j = D_j^{-1} and z_j = -M_j R_j to the
//      workspace;
//   3. the block lower-bidiagonal system (Section 3) as the affine recurrence
//      x_j = z_j + M_j x_{j-1}: the chunk is cut into segments of T steps;
//      each wave composes its segments' maps serially (Thomas's algorithm,
//      Alg. thomas), ceil(log2 S) parallel-cyclic-reduction levels compose the
//      S segment maps (Section 3.2, the normalized split with B = -I), and each
//      segment replays its steps from the value entering it (Section 3.3, the
//      hybrid).  T = chunk is Thomas's algorithm, T = 1 is pure PCR.
// The adjoint solves D_j^T lam_j - lam_{j+1} = g_j chunk by chunk in reverse:
// lam_j = D_j^{-T} g_j + D_j^{-T} lam_{j+1}, the same recurrence on the
// transposed inverses in reversed step order, then dL/dp = sum_j dt_j
// (dh/dp(y_j))^T lam_j as sums over steps of products of per-step factors.
#pragma once

#include "grad_input.hpp"
#include "solver.hpp"
#include "tvi.h"

namespace tvi {
namespace blk {

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * kWave;
constexpr int kMaxN = 40;
constexpr int kMaxChunk = 1024;

struct BlockArgs {
    SolveArgs<double> a;
    int32_t n;          // state size (<= NP)
    int32_t P;          // parameters per series
    int32_t T;          // steps per segment (T >= chunk: Thomas; 1: PCR)
    int32_t NF;         // factors per step (adjoint)
    int64_t ws_stride;  // workspace doubles per launch slot
    double *ws;         // workspace [B][ws_stride]
    GradInput gi;       // adjoint: how dL/dy is read
};

// Per-slot workspace, in doubles (row stride NP).
struct WsLayout {
    int64_t M, SA, SB, z, za, zb, dy, F, total;
};

__host__ __device__ inline WsLayout ws_layout(int NP, int C, int T, int NF)
{
    const int64_t S = (C + T - 1) / T;
    const int64_t blk = (int64_t)NP * NP;
    WsLayout w;
    int64_t o = 0;
    w.M = o;  o += (int64_t)C * blk;        // step maps
    w.SA = o; o += (T > 1 && S > 1 ? S : 0) * blk;  // segment maps (T = 1: the step maps; S = 1: none)
    w.SB = o; o += (S > 1 ? S : 0) * blk;   // the other buffer of the reduction levels
    w.z = o;  o += (int64_t)C * NP;
    w.za = o; o += (T > 1 && S > 1 ? S : 0) * NP;
    w.zb = o; o += (S > 1 ? S : 0) * NP;
    w.dy = o; o += (int64_t)(C + 1) * NP;   // Newton iterate, dy[0] = 0
    w.F = o;  o += (int64_t)C * NF;         // adjoint factors per step
    w.total = o;
    return w;
}

// LDS: per wave a block buffer of (NP+1) x (NP+1) doubles, a state vector,
// two vectors for the serial replay, the model's scratch; shared by the
// workgroup: the chunk start state, the carried adjoint vector, per-wave
// partial sums and flags.
template <int NP, int SCR>
struct Lds {
    static constexpr int kBlk = (NP + 1) * (NP + 1);
    static constexpr int kPiv = (NP + 1) / 2;  // the pivot order (NP ints) after vector 2
    static constexpr int kPerWave = kBlk + 3 * NP + kPiv + SCR;
    double wave[kWaves][kPerWave];
    double ys[NP];
    double lam[NP];
    double red[kWaves];
    int flag[kWaves];
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Row `lane` of D = I - dt j, padded with identity rows, from the lane's
// Jacobian row in LDS.
template <int NP>
__device__ __forceinline__ void load_block_row(const double *jrow, int lane, int n, double dt, double (&a)[NP])
{
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double e = (c == lane) ? 1.0 : 0.0;
        a[c] = lane < n ? fma(-dt, jrow[c], e) : e;
    }
}

// Inverse of the NP x NP block whose row `lane` is a[] (lanes >= NP hold
// nothing; rows n..NP-1 are identity rows), by Gauss-Jordan elimination with
// partial pivoting, without moving rows between lanes: step k takes as pivot
// the unused row with the largest |entry| in column k (ties: the lowest row).
// Every step shifts the rows left by one column and appends the new column of
// the inverse, so the pivot column is always a[0] and the step loop needs no
// unrolling.  Afterwards the lane that pivoted at step k holds row k of the
// inverse with its columns permuted: a[c] is entry (k, piv[c]).  The
// permutation is undone while writing the inverse into `blk` (row stride
// NP + 1), transposed when TR.  rowbuf: NP doubles of LDS for the pivot row,
// then the pivot order (NP ints).  Returns false (every lane) if a pivot is
// zero or not finite.
template <int NP, bool TR>
__device__ __forceinline__ bool gj_invert_to(double (&a)[NP], int lane, double *rowbuf, double *blk)
{
    bool used = lane >= NP;
    bool ok = true;
    int kk = 0;
    int *piv = reinterpret_cast<int *>(rowbuf + NP);
    for (int k = 0; k < NP; ++k) {
        const double cand = used ? -1.0 : fabs(a[0]);
        const bool nan = cand != cand;
        const double best = wave_max(nan ? -1.0 : cand);
        const unsigned long long at = __ballot(!used && cand == best);
        const int p = at ? __builtin_amdgcn_readfirstlane(__ffsll((long long)at) - 1) : 0;
        ok = ok && !wave_any(nan) && best > 0.0 && finite(best);
        if (lane == p) {
#pragma unroll
            for (int c = 0; c < NP; ++c) rowbuf[c] = a[c];
            piv[k] = p;
        }
        wave_sync();
        const double inv = 1.0 / rowbuf[0];
        if (lane == p) {
            used = true;
            kk = k;
#pragma unroll
            for (int c = 1; c < NP; ++c) a[c - 1] = a[c] * inv;
            a[NP - 1] = inv;
        } else {
            const double f = -a[0] * inv;
#pragma unroll
            for (int c = 1; c < NP; ++c) a[c - 1] = fma(f, rowbuf[c], a[c]);
            a[NP - 1] = f;
        }
        wave_sync();
    }
    if (lane < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            const int pc = piv[c];
            if (TR) blk[pc * (NP + 1) + kk] = a[c];
            else blk[kk * (NP + 1) + pc] = a[c];
        }
    }
    wave_sync();
    return ok;
}

// Workgroup context of one series.
template <int NP, int SCR>
struct Ctx {
    Lds<NP, SCR> *L;
    double *ws;   // this slot's workspace
    WsLayout lay;
    int w, lane, tid;
    __device__ double *M() const { return ws + lay.M; }
    __device__ double *z() const { return ws + lay.z; }
    __device__ double *blk() const { return L->wave[w]; }
    __device__ double *vec(int i) const { return L->wave[w] + Lds<NP, SCR>::kBlk + i * NP; }  // 0: state, 1-2: replay
    __device__ double *scr() const { return L->wave[w] + Lds<NP, SCR>::kBlk + 3 * NP + Lds<NP, SCR>::kPiv; }
    // the lane's row of blk (lanes >= NP, which hold no row, get the last one)
    __device__ double *jrow() const { return L->wave[w] + (lane < NP ? lane : NP - 1) * (NP + 1); }
};

// x_j = zz_j + MM_j x_{j-1} for j = j0 .. j0+len-1 from x_{j0-1} = vec(1)
// (one wave); each x_j overwrites zz_j.
template <int NP, int SCR>
__device__ void replay(const Ctx<NP, SCR> &cx, const double *MM, double *zz, int j0, int len)
{
    double *cur = cx.vec(1), *nxt = cx.vec(2);
    const int i = cx.lane;
    for (int j = j0; j < j0 + len; ++j) {
        double acc = 0.0;
        if (i < NP) {
            const double *row = MM + ((int64_t)j * NP + i) * NP;
            double acc4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NP; ++c) acc4[c & 3] = fma(row[c], cur[c], acc4[c & 3]);
            acc = zz[(int64_t)j * NP + i] + ((acc4[0] + acc4[1]) + (acc4[2] + acc4[3]));
            zz[(int64_t)j * NP + i] = acc;
            nxt[i] = acc;
        }
        wave_sync();
        double *t = cur; cur = nxt; nxt = t;
    }
}

// acc[c] = sum_l row[l] blk[l][c] for c = 0..NP (row: NP entries in global
// memory, blk: NP rows of NP + 1 in LDS, read by every lane alike).  The l
// loop is not unrolled, so only the accumulators stay live.
template <int NP>
__device__ __forceinline__ void row_times_blk(const double *row, const double *blk, double (&acc)[NP + 1])
{
#pragma unroll
    for (int c = 0; c <= NP; ++c) acc[c] = 0.0;
#pragma unroll 2
    for (int l = 0; l < NP; ++l) {
        const double r = row[l];
        const double *b = blk + l * (NP + 1);
#pragma unroll
        for (int c = 0; c <= NP; ++c) acc[c] = fma(r, b[c], acc[c]);
    }
}

// (P, p) <- (A, a) o (B, b): P = A B, p = A b + a (one wave; B staged in LDS).
template <int NP, int SCR>
__device__ void compose(const Ctx<NP, SCR> &cx, const double *A, const double *a, const double *Bm, const double *b,
                        double *Pm, double *p)
{
    double *blk = cx.blk();
    const int i = cx.lane;
    if (i < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) blk[i * (NP + 1) + c] = Bm[i * NP + c];
        blk[i * (NP + 1) + NP] = b[i];
    }
    wave_sync();
    if (i < NP) {
        double acc[NP + 1];
        row_times_blk<NP>(A + i * NP, blk, acc);
#pragma unroll
        for (int c = 0; c < NP; ++c) Pm[i * NP + c] = acc[c];
        p[i] = acc[NP] + a[i];
    }
    wave_sync();
}

// The map of steps j0 .. j0+len-1 of x_j = z_j + M_j x_{j-1} (one wave):
// P = M_last ... M_j0, p = its offset; Thomas's serial composition.
template <int NP, int SCR>
__device__ void compose_segment(const Ctx<NP, SCR> &cx, int j0, int len, double *Pm, double *p)
{
    double *blk = cx.blk();
    const double *M = cx.M(), *z = cx.z();
    const int i = cx.lane;
    if (i < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) blk[i * (NP + 1) + c] = M[((int64_t)j0 * NP + i) * NP + c];
        blk[i * (NP + 1) + NP] = z[(int64_t)j0 * NP + i];
    }
    wave_sync();
    for (int j = j0 + 1; j < j0 + len; ++j) {
        double acc[NP + 1];
        if (i < NP) {
            row_times_blk<NP>(M + ((int64_t)j * NP + i) * NP, blk, acc);
            acc[NP] += z[(int64_t)j * NP + i];
        }
        wave_sync();
        if (i < NP) {
#pragma unroll
            for (int c = 0; c <= NP; ++c) blk[i * (NP + 1) + c] = acc[c];
        }
        wave_sync();
    }
    if (i < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) Pm[i * NP + c] = blk[i * (NP + 1) + c];
        p[i] = blk[i * (NP + 1) + NP];
    }
    wave_sync();
}

// Solve x_j = z_j + M_j x_{j-1}, j = 0 .. m-1, from x_{-1} = xin (LDS,
// shared; null: zero), in segments of T steps; x overwrites z.  Every thread
// of the workgroup calls it.
template <int NP, int SCR>
__device__ void chain_solve(const Ctx<NP, SCR> &cx, int m, int T, const double *xin)
{
    const int S = (m + T - 1) / T;
    const int w = cx.w, i = cx.lane;
    double *M = cx.M(), *z = cx.z();
    if (S == 1) {  // Thomas's algorithm: one wave runs the whole chunk
        if (w == 0) {
            if (i < NP) cx.vec(1)[i] = xin ? xin[i] : 0.0;
            wave_sync();
            replay(cx, M, z, 0, m);
        }
        __syncthreads();
        return;
    }
    double *PA = M, *pa = z;
    if (T > 1) {
        PA = cx.ws + cx.lay.SA;
        pa = cx.ws + cx.lay.za;
        for (int g = w; g < S; g += kWaves)
            compose_segment(cx, g * T, min(T, m - g * T), PA + (int64_t)g * NP * NP, pa + (int64_t)g * NP);
        __syncthreads();
    }
    double *PB = cx.ws + cx.lay.SB, *pb = cx.ws + cx.lay.zb;
    for (int sig = 1; sig < S; sig <<= 1) {
        for (int g = w; g < S; g += kWaves) {
            double *Pg = PB + (int64_t)g * NP * NP, *pg = pb + (int64_t)g * NP;
            const double *Ag = PA + (int64_t)g * NP * NP, *ag = pa + (int64_t)g * NP;
            if (g >= sig) {
                compose(cx, Ag, ag, PA + (int64_t)(g - sig) * NP * NP, pa + (int64_t)(g - sig) * NP, Pg, pg);
            } else if (i < NP) {
#pragma unroll
                for (int c = 0; c < NP; ++c) Pg[i * NP + c] = Ag[i * NP + c];
                pg[i] = ag[i];
            }
        }
        __syncthreads();
        double *t = PA; PA = PB; PB = t;
        t = pa; pa = pb; pb = t;
    }
    // PA[g], pa[g]: the map from x_{-1} to the value at the end of segment g
    if (T == 1) {
        for (int g = w; g < S; g += kWaves) {
            if (i < NP) {
                double v = pa[(int64_t)g * NP + i];
                if (xin) {
                    const double *row = PA + ((int64_t)g * NP + i) * NP;
#pragma unroll
                    for (int c = 0; c < NP; ++c) v = fma(row[c], xin[c], v);
                }
                z[(int64_t)g * NP + i] = v;  // z may alias pa: each lane rewrites its own entry
            }
        }
        __syncthreads();
        return;
    }
    for (int g = w; g < S; g += kWaves) {
        if (i < NP) {
            double v = 0.0;
            if (g == 0) {
                v = xin ? xin[i] : 0.0;
            } else {
                v = pa[(int64_t)(g - 1) * NP + i];
                if (xin) {
                    const double *row = PA + ((int64_t)(g - 1) * NP + i) * NP;
#pragma unroll
                    for (int c = 0; c < NP; ++c) v = fma(row[c], xin[c], v);
                }
            }
            cx.vec(1)[i] = v;
        }
        wave_sync();
        replay(cx, M, z, g * T, min(T, m - g * T));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Forward kernel
// ---------------------------------------------------------------------------
template <class Model, int NP>
__global__ __launch_bounds__(kThreads) void block_forward_kernel(BlockArgs ba)
{
    using L_t = Lds<NP, Model::template scratch<NP>()>;
    extern __shared__ __align__(16) unsigned char smem[];
    L_t &L = *reinterpret_cast<L_t *>(smem);
    const SolveArgs<double> &a = ba.a;
    const SeriesView<double> sv(a, blockIdx.x);
    if (!sv.valid) return;  // uniform over the workgroup
    const int tid = threadIdx.x, w = tid / kWave, lane = tid & (kWave - 1);
    const int n = ba.n, C = a.chunk, T = ba.T;
    Ctx<NP, Model::template scratch<NP>()> cx{&L, ba.ws + (int64_t)blockIdx.x * ba.ws_stride,
                                               ws_layout(NP, C, T, ba.NF), w, lane, tid};
    Model model;
    model.init(n, a.params_shared ? a.params : a.params + sv.b * ba.P);
    const double *t = sv.t;
    double *y = a.y ? a.y + sv.p0 * n : nullptr;
    double *ck = a.ckpt ? a.ckpt + sv.b * a.K * n : nullptr;
    double *dy = cx.ws + cx.lay.dy, *z = cx.z(), *M = cx.M();

    if (tid < NP) L.ys[tid] = tid < n ? a.y0[sv.b * n + tid] : 0.0;
    __syncthreads();
    if (tid < n) {
        if (y) y[tid] = L.ys[tid];
        if (ck) ck[tid] = L.ys[tid];
    }

    const int64_t Nb = sv.Nb;
    int64_t s = 0, ck_next = 1, ck_at = C;
    int mcur = C, m = 0, it = 0, total = 0, status = ST_OK;
    bool active = Nb > 0, start = true, sing = false;
    double nrm0 = 0.0;
    const double tol_a2 = a.tol_a * a.tol_a, tol_r2 = a.tol_r * a.tol_r;

    while (active) {
        if (start) {
            m = (int)min((int64_t)mcur, min(ck_at, Nb) - s);
            // the extrapolated start needs h(y_s, t_s): wave 0 leaves it in its vector 1
            const double *slope = L.wave[0] + L_t::kBlk + NP;
            if (a.init == INIT_EXTRAP) {
                if (w == 0) {
                    double *yv = cx.vec(0);
                    if (lane < NP) yv[lane] = L.ys[lane];
                    wave_sync();
                    const double f = model.rate(yv, t[s], cx.scr(), cx.blk(), lane);
                    wave_sync();
                    if (lane < NP) cx.vec(1)[lane] = (lane < n) ? f : 0.0;
                }
                __syncthreads();
            }
            const double ts = t[s];
            for (int e = tid; e < (m + 1) * NP; e += kThreads) {
                const int j = e / NP, k = e - j * NP;
                dy[e] = (a.init == INIT_EXTRAP && k < n) ? (t[s + j] - ts) * slope[k] : 0.0;
            }
            it = 0;
            sing = false;
            start = false;
            __syncthreads();
        }

        // ---- residual and its norm
        double acc = 0.0;
        for (int j = 1 + w; j <= m; j += kWaves) {
            double *yv = cx.vec(0);
            const double *dj = dy + (int64_t)j * NP;
            if (lane < NP) yv[lane] = L.ys[lane] + dj[lane];
            wave_sync();
            const double tj = t[s + j], hj = tj - t[s + j - 1];
            const double f = model.rate(yv, tj, cx.scr(), cx.blk(), lane);
            if (lane < NP) {
                const double r = lane < n ? (dj[lane] - dj[lane - NP]) - hj * f : 0.0;
                z[(int64_t)(j - 1) * NP + lane] = r;
                acc = fma(r, r, acc);
            }
            wave_sync();
        }
        acc = seg_sum<kWave>(acc);
        if (lane == 0) L.red[w] = acc;
        __syncthreads();
        double nrm2 = 0.0;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) nrm2 += L.red[v];
        __syncthreads();

        int act;  // 1 converged, 2 failed, 3 correct
        int code = ST_OK;
        if (it == 0) nrm0 = nrm2;
        if (sing) { act = 2; code = ST_SINGULAR; }
        else if (!finite(nrm2)) { act = 2; code = ST_NONFINITE; }
        else if (nrm2 <= tol_a2 || nrm2 <= tol_r2 * nrm0) act = 1;
        else if (it >= a.max_newton) { act = 2; code = ST_NOT_CONVERGED; }
        else act = 3;

        if (act == 1) {
            for (int e = tid; e < m * n; e += kThreads) {
                const int j = e / n + 1, k = e - (j - 1) * n;
                if (y) y[(s + j) * n + k] = L.ys[k] + dy[(int64_t)j * NP + k];
            }
            __syncthreads();
            if (tid < NP) L.ys[tid] += dy[(int64_t)m * NP + tid];
            __syncthreads();
            s += m;
            const bool at_ck = s == ck_at;
            if ((at_ck || s >= Nb) && ck && ck_next < a.K && tid < n) ck[ck_next * n + tid] = L.ys[tid];
            if (at_ck) {
                mcur = C;
                ++ck_next;
                ck_at += C;
            }
            if (s >= Nb) active = false;
            start = true;
        } else if (act == 2) {
            if (a.halving && m > 1) {
                mcur = (m + 1) / 2;
                start = true;
            } else {
                status = code;
                active = false;
                if (y)
                    for (int64_t e = (s + 1) * n + tid; e < (Nb + 1) * n; e += kThreads) y[e] = __builtin_nan("");
            }
        } else {
            // ---- blocks, inverses and offsets
            bool ok = true;
            for (int j = 1 + w; j <= m; j += kWaves) {
                double *yv = cx.vec(0), *rv = cx.vec(1);
                if (lane < NP) {
                    yv[lane] = L.ys[lane] + dy[(int64_t)j * NP + lane];
                    rv[lane] = z[(int64_t)(j - 1) * NP + lane];
                }
                wave_sync();
                const double tj = t[s + j], hj = tj - t[s + j - 1];
                model.template rate_row<NP>(yv, tj, cx.scr(), cx.blk(), lane, cx.jrow());
                wave_sync();
                double row[NP];
                load_block_row<NP>(cx.jrow(), lane, n, hj, row);
                ok = gj_invert_to<NP, false>(row, lane, cx.vec(2), cx.blk()) && ok;
                if (lane < NP) {
                    const double *br = cx.blk() + lane * (NP + 1);
                    double *Mr = M + ((int64_t)(j - 1) * NP + lane) * NP;
                    double zz = 0.0;
#pragma unroll
                    for (int c = 0; c < NP; ++c) {
                        Mr[c] = br[c];
                        zz = fma(-br[c], rv[c], zz);
                    }
                    z[(int64_t)(j - 1) * NP + lane] = zz;
                }
                wave_sync();
            }
            if (lane == 0) L.flag[w] = ok ? 1 : 0;
            __syncthreads();
#pragma unroll
            for (int v = 0; v < kWaves; ++v) ok = ok && L.flag[v];
            // ---- the chunk's block-bidiagonal solve, then the update
            chain_solve(cx, m, T, nullptr);
            for (int e = tid; e < m * NP; e += kThreads) dy[e + NP] += z[e];
            __syncthreads();
            ++it;
            ++total;
            if (!ok) sing = true;
        }
    }
    if (tid == 0) {
        a.status[sv.b] = status;
        if (a.iters) a.iters[sv.b] = total;
    }
}

// ---------------------------------------------------------------------------
// Adjoint kernel (states from the stored trajectory)
// ---------------------------------------------------------------------------
template <class Model, int NP>
__global__ __launch_bounds__(kThreads) void block_adjoint_kernel(BlockArgs ba)
{
    constexpr int SCR = Model::template scratch<NP>();
    constexpr int kQ = (Model::template max_params<NP>() + kThreads - 1) / kThreads;
    using L_t = Lds<NP, SCR>;
    extern __shared__ __align__(16) unsigned char smem[];
    L_t &L = *reinterpret_cast<L_t *>(smem);
    const SolveArgs<double> &a = ba.a;
    const SeriesView<double> sv(a, blockIdx.x);
    if (!sv.valid) return;
    const int tid = threadIdx.x, w = tid / kWave, lane = tid & (kWave - 1);
    const int n = ba.n, C = a.chunk, T = ba.T, P = ba.P, NF = ba.NF;
    Ctx<NP, SCR> cx{&L, ba.ws + (int64_t)blockIdx.x * ba.ws_stride, ws_layout(NP, C, T, NF), w, lane, tid};
    Model model;
    model.init(n, a.params + sv.b * P);
    const double *t = sv.t;
    const double *y = a.y + sv.p0 * n;
    const double gsc = grad_scale(ba.gi);  // g = (given g) / (*gi.div)
    double *z = cx.z(), *M = cx.M(), *F = cx.ws + cx.lay.F;

    if (tid < NP) L.lam[tid] = 0.0;
    double gq[kQ];
#pragma unroll
    for (int r = 0; r < kQ; ++r) gq[r] = 0.0;
    bool ok = true;
    __syncthreads();

    const int64_t Nb = sv.Nb;
    for (int64_t c = (Nb + C - 1) / C - 1; c >= 0; --c) {
        const int64_t c0 = c * C;
        const int m = (int)min((int64_t)C, Nb - c0);
        // ---- transposed inverses in reversed order: slot r = m - j holds step j
        for (int j = 1 + w; j <= m; j += kWaves) {
            double *yv = cx.vec(0), *gv = cx.vec(1);
            if (lane < NP) {
                yv[lane] = lane < n ? y[(c0 + j) * n + lane] : 0.0;
                const double *gp = grad_at(a.g, ba.gi, sv.b, sv.p0, c0 + j, n);
                gv[lane] = (lane < n && gp) ? gsc * gp[lane] : 0.0;
            }
            wave_sync();
            const double tj = t[c0 + j], hj = tj - t[c0 + j - 1];
            model.template rate_row<NP>(yv, tj, cx.scr(), cx.blk(), lane, cx.jrow());
            wave_sync();
            double row[NP];
            load_block_row<NP>(cx.jrow(), lane, n, hj, row);
            ok = gj_invert_to<NP, true>(row, lane, cx.vec(2), cx.blk()) && ok;
            if (lane < NP) {
                const int r = m - j;
                const double *br = cx.blk() + lane * (NP + 1);
                double *Nr = M + ((int64_t)r * NP + lane) * NP;
                double zz = 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    Nr[k] = br[k];
                    zz = fma(br[k], gv[k], zz);
                }
                z[(int64_t)r * NP + lane] = zz;
            }
            wave_sync();
        }
        __syncthreads();
        // x_r = lam at step c0 + m - r, from lam at c0 + m + 1 (carried)
        chain_solve(cx, m, T, L.lam);
        // ---- per-step factors of the parameter products at w_j = dt_j lam_j
        for (int j = 1 + w; j <= m; j += kWaves) {
            double *yv = cx.vec(0), *wv = cx.vec(1);
            const double tj = t[c0 + j], hj = tj - t[c0 + j - 1];
            if (lane < NP) {
                yv[lane] = lane < n ? y[(c0 + j) * n + lane] : 0.0;
                wv[lane] = lane < n ? hj * z[(int64_t)(m - j) * NP + lane] : 0.0;
            }
            wave_sync();
            model.factors(yv, tj, wv, cx.scr(), cx.blk(), lane, F + (int64_t)(j - 1) * NF);
            wave_sync();
        }
        __syncthreads();
        // ---- dL/dp += sum over the chunk's steps, in step order
#pragma unroll
        for (int r = 0; r < kQ; ++r) {
            const int q = tid + r * kThreads;
            if (q < P) {
                int fa, fb;
                model.pair(q, fa, fb);
                double s = 0.0;
                for (int j = 0; j < m; ++j) s = fma(F[(int64_t)j * NF + fa], F[(int64_t)j * NF + fb], s);
                gq[r] += s;
            }
        }
        if (tid < NP) L.lam[tid] = z[(int64_t)(m - 1) * NP + tid];
        __syncthreads();
    }
    if (lane == 0) L.flag[w] = ok ? 1 : 0;
    __syncthreads();
    bool all = true;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) all = all && L.flag[v];
    const double nan = __builtin_nan("");
#pragma unroll
    for (int r = 0; r < kQ; ++r) {
        const int q = tid + r * kThreads;
        if (q < P) a.dLdp[sv.b * P + q] = all ? gq[r] : nan;
    }
    const double *g0 = grad_at(a.g, ba.gi, sv.b, sv.p0, 0, n);
    if (tid < n) a.dLdy0[sv.b * n + tid] = all ? (g0 ? gsc * g0[tid] : 0.0) + L.lam[tid] : nan;
    if (tid == 0) a.status[sv.b] = all ? ST_OK : ST_SINGULAR;
}

// Rate and state Jacobian of M independent states, one wave per state.
template <class Model, int NP>
__global__ __launch_bounds__(kThreads) void block_eval_kernel(int n, int P, int64_t Ms, const double *states,
                                                              const double *times, const double *params,
                                                              int shared, double *f, double *J)
{
    using L_t = Lds<NP, Model::template scratch<NP>()>;
    extern __shared__ __align__(16) unsigned char smem[];
    L_t &L = *reinterpret_cast<L_t *>(smem);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int64_t e = (int64_t)blockIdx.x * kWaves + w;
    if (e >= Ms) return;  // uniform over the wave; no workgroup barrier below
    Ctx<NP, Model::template scratch<NP>()> cx{&L, nullptr, WsLayout{}, w, lane, (int)threadIdx.x};
    Model model;
    model.init(n, shared ? params : params + e * P);
    double *yv = cx.vec(0);
    if (lane < NP) yv[lane] = lane < n ? states[e * n + lane] : 0.0;
    wave_sync();
    const double fv = model.template rate_row<NP>(yv, times ? times[e] : 0.0, cx.scr(), cx.blk(), lane, cx.jrow());
    wave_sync();
    if (lane < n) {
        if (f) f[e * n + lane] = fv;
        if (J)
            for (int c = 0; c < n; ++c) J[(e * n + lane) * n + c] = cx.jrow()[c];
    }
}

template <class Model, int NP>
inline size_t lds_bytes()
{
    return sizeof(Lds<NP, Model::template scratch<NP>()>);
}

struct EvalArgs {
    int n, P, shared;
    int64_t M;
    const double *states, *times, *params;
    double *f, *J;
};

template <class Model, int NP>
tvi_status launch_np(int pass, const BlockArgs &ba, const EvalArgs *ev, hipStream_t stream)
{
    const size_t shm = lds_bytes<Model, NP>();
    if (ev) {
        if (hipFuncSetAttribute((const void *)block_eval_kernel<Model, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
            return TVI_EHIP;
        const int64_t blocks = (ev->M + kWaves - 1) / kWaves;
        if (blocks > 0x7fffffffLL) return TVI_EINVAL;
        hipLaunchKernelGGL((block_eval_kernel<Model, NP>), dim3((unsigned)blocks), dim3(kThreads), shm, stream,
                           ev->n, ev->P, ev->M, ev->states, ev->times, ev->params, ev->shared, ev->f, ev->J);
        return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
    }
    const dim3 grid((unsigned)ba.a.B), block(kThreads);
    if (pass == 0) {
        if (hipFuncSetAttribute((const void *)block_forward_kernel<Model, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
            return TVI_EHIP;
        hipLaunchKernelGGL((block_forward_kernel<Model, NP>), grid, block, shm, stream, ba);
    } else {
        if (hipFuncSetAttribute((const void *)block_adjoint_kernel<Model, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
            return TVI_EHIP;
        hipLaunchKernelGGL((block_adjoint_kernel<Model, NP>), grid, block, shm, stream, ba);
    }
    return hipGetLastError() == hipSuccess ? TVI_OK : TVI_EHIP;
}

// The padded size a state of size n runs at.
inline int padded(int n) { return n <= 8 ? 8 : n <= 16 ? 16 : n <= 24 ? 24 : n <= 32 ? 32 : 40; }

// pass 0: forward, 1: adjoint, 2: model evaluation (ev)
template <class Model>
tvi_status launch_model(int pass, int n, const BlockArgs *ba, const EvalArgs *ev, hipStream_t stream)
{
    static const BlockArgs none{};
    const BlockArgs &b = ba ? *ba : none;
    const EvalArgs *e = pass == 2 ? ev : nullptr;
    switch (padded(n)) {
    case 8: return launch_np<Model, 8>(pass, b, e, stream);
    case 16: return launch_np<Model, 16>(pass, b, e, stream);
    case 24: return launch_np<Model, 24>(pass, b, e, stream);
    case 32: return launch_np<Model, 32>(pass, b, e, stream);
    default: return launch_np<Model, 40>(pass, b, e, stream);
    }
}

}  // namespace blk
}  // namespace tvi
