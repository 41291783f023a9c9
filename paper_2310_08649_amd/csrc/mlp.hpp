// Neural-ODE right-hand side h(y) = W3 tanh(W2 tanh(W1 y + b1) + b2) + b3
// (n = 8 states, 64 hidden units, shared parameters) evaluated on MFMA:
// v_mfma_f32_16x16x32_bf16 with hidden units along M and samples (time steps
// of a chunk) along N.
//
// Precision.  Every product that enters the Newton residual or the adjoint
// is computed from a three-way bf16 split of both operands (x = x0 + x1 + x2,
// each part a bf16 holding the next 8 bits of the float mantissa) with the
// six MFMAs x0y0 + x0y1 + x1y0 + x0y2 + x1y1 + x2y0 accumulated in float; the
// dropped terms are below float rounding, so this is float-accurate.  (A
// two-way split with three products keeps only about 16 bits.)  The Jacobian
// used only inside Newton's method may take plain bf16 products: an
// approximate Jacobian changes the convergence rate, not the root.
//
// Operand layout (16x16x32, lane l, group g = l / 16, r = l % 16): the A
// operand of a lane is row r of the 16-row tile, the B operand column r of
// the 16-column tile, each with eight k-elements e = 0..7; the accumulator
// holds D[4g + i][r], i = 0..3.  The contraction only needs A and B to use
// the same lane-to-k assignment, so a chained product takes its B operand
// straight from the previous accumulators: for K-step ks (32 hidden units,
// the previous M-tiles 2ks and 2ks+1) element e of lane l is the previous
// output element (tile 2ks + e/4, entry e%4), i.e. hidden unit
// k(ks, g, e) = 32 ks + 16 (e / 4) + 4 g + e % 4, and the weights are stored
// in LDS already permuted to that order.
#pragma once

#include "device.hpp"

namespace tvi {
namespace mlp {

constexpr int NS = 8;   // state size
constexpr int H = 64;   // hidden width
constexpr int P = H * NS + H + H * H + H + NS * H + NS;  // 5256
constexpr int kWaves = 4;
constexpr int kSPW = 32;                  // samples (chunk steps) per wave
constexpr int kMaxChunk = kWaves * kSPW;  // 128
constexpr int kThreads = kWaves * kWave;

// offsets of the parameter blocks in theta
constexpr int oW1 = 0, ob1 = H * NS, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + NS * H;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ f32x4 mma(const bf16x8 &a, const bf16x8 &b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Split {
    bf16x8 p0, p1, p2;
};

__device__ __forceinline__ Split split8(const float (&x)[8])
{
    Split s;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h0 = (__bf16)x[e];
        const float r1 = x[e] - (float)h0;
        const __bf16 h1 = (__bf16)r1;
        s.p0[e] = h0;
        s.p1[e] = h1;
        s.p2[e] = (__bf16)(r1 - (float)h1);
    }
    return s;
}

__device__ __forceinline__ Split split_lds(const float *x)
{
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = x[e];
    return split8(v);
}

// c += a * b: float-accurate (EXACT, six products) or plain bf16 (one product)
template <bool EXACT>
__device__ __forceinline__ f32x4 mma_acc(const Split &a, const Split &b, f32x4 c)
{
    if (EXACT) {
        c = mma(a.p0, b.p2, c);
        c = mma(a.p1, b.p1, c);
        c = mma(a.p2, b.p0, c);
        c = mma(a.p0, b.p1, c);
        c = mma(a.p1, b.p0, c);
    }
    return mma(a.p0, b.p0, c);
}

__device__ __forceinline__ int kchain(int ks, int g, int e) { return 32 * ks + 16 * (e >> 2) + 4 * g + (e & 3); }

// One operand tile of the network's forward pass, split once when the weights
// are loaded (x = p0 + p1 + p2): a lane reads its eight k-elements of each part
// with one 16-byte load (the parts stored apart: consecutive lanes, consecutive
// 16 bytes), and the plain bf16 products read p0 alone.
struct Tile {
    bf16x8 p0[kWave], p1[kWave], p2[kWave];
    __device__ __forceinline__ Split at(int l) const { return Split{p0[l], p1[l], p2[l]}; }
    __device__ __forceinline__ void put(int l, const float (&x)[8])
    {
        const Split s = split8(x);
        p0[l] = s.p0;
        p1[l] = s.p1;
        p2[l] = s.p2;
    }
};

// Weights in LDS, per (tile, lane) in operand order.  The forward pass's tiles
// are stored split; the adjoint's transposed tiles as float (split where used:
// the LDS holds no more).
struct Weights {
    Tile w1[4];                  // W1   [64 x 8]:  M-tiles 0..3, one K-step (k = 8 g + e, k < 8)
    Tile w2[4][2];               // W2   [64 x 64]: M-tiles, chained K-steps
    Tile w3[2];                  // W3   [8 x 64]:  one M-tile (rows 8..15 zero), chained K-steps
    float w3t[4][kWave][8];      // W3^T [64 x 8]:  M-tiles, one K-step (k = 8 g + e, k < 8)
    float w2t[4][2][kWave][8];   // W2^T [64 x 64]
    float w1p[2][4][8][NS];      // W1[k(ks, g, e)][c]: the Jacobian's first factor
    float b1[H], b2[H], b3[NS];
};

// Fill the operand tiles from theta (all threads of the block cooperate).
template <class IO>
__device__ void load_weights(Weights &W, const IO *th)
{
    const int t = threadIdx.x;
    for (int idx = t; idx < 4 * kWave; idx += kThreads) {
        const int mt = idx / kWave, l = idx % kWave, g = l >> 4, r = l & 15;
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            a[e] = k < NS ? (float)th[oW1 + (16 * mt + r) * NS + k] : 0.f;   // W1[m][k]
            b[e] = k < NS ? (float)th[oW3 + k * H + 16 * mt + r] : 0.f;     // W3^T[m][k] = W3[k][m]
        }
        W.w1[mt].put(l, a);
#pragma unroll
        for (int e = 0; e < 8; ++e) W.w3t[mt][l][e] = b[e];
    }
    for (int idx = t; idx < 8 * kWave; idx += kThreads) {
        const int mt = idx / (2 * kWave), ks = (idx / kWave) & 1, l = idx % kWave, g = l >> 4, r = l & 15;
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kchain(ks, g, e);
            a[e] = (float)th[oW2 + (16 * mt + r) * H + k];   // W2[m][k]
            b[e] = (float)th[oW2 + k * H + 16 * mt + r];     // W2^T[m][k] = W2[k][m]
        }
        W.w2[mt][ks].put(l, a);
#pragma unroll
        for (int e = 0; e < 8; ++e) W.w2t[mt][ks][l][e] = b[e];
    }
    for (int idx = t; idx < 2 * kWave; idx += kThreads) {
        const int ks = idx / kWave, l = idx % kWave, g = l >> 4, r = l & 15;
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = r < NS ? (float)th[oW3 + r * H + kchain(ks, g, e)] : 0.f;
        W.w3[ks].put(l, a);
    }
    for (int idx = t; idx < 2 * 4 * 8 * NS; idx += kThreads) {
        const int c = idx % NS, e = (idx / NS) % 8, g = (idx / (NS * 8)) % 4, ks = idx / (NS * 32);
        W.w1p[ks][g][e][c] = (float)th[oW1 + kchain(ks, g, e) * NS + c];
    }
    for (int idx = t; idx < H; idx += kThreads) {
        W.b1[idx] = (float)th[ob1 + idx];
        W.b2[idx] = (float)th[ob2 + idx];
    }
    if (t < NS) W.b3[t] = (float)th[ob3 + t];
}

// Activations of one wave's 32 samples (two 16-sample N-tiles u), in
// accumulator layout: a1[mt][u][i] is hidden unit 16 mt + 4 g + i of sample
// 16 u + r.
struct Acts {
    f32x4 a1[4][2], a2[4][2];
};

// Forward pass for the wave's samples.  ys(u) gives the state of the lane's
// column sample (8 floats, used by group 0 only).  Writes the rate of sample
// (16 u + r) rows 4g+i (g < 2) through put_f(u, row, value).
template <bool EXACT, class GetY, class PutF>
__device__ __forceinline__ void forward(const Weights &W, Acts &A, GetY get_y, PutF put_f)
{
    const int l = lane_id(), g = l >> 4;
    Split yb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        float y[8];
        get_y(u, y);
        if (g != 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) y[e] = 0.f;
        }
        yb[u] = split8(y);
    }
    // layer 1
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 bias;
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[i] = W.b1[16 * mt + 4 * g + i];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            f32x4 z = mma_acc<true>(W.w1[mt].at(l), yb[u], bias);
#pragma unroll
            for (int i = 0; i < 4; ++i) A.a1[mt][u][i] = tanhf(z[i]);
        }
    }
    // layer 2
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        Split bk[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = A.a1[2 * ks + (e >> 2)][u][e & 3];
            bk[ks] = split8(v);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 z;
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = W.b2[16 * mt + 4 * g + i];
            z = mma_acc<true>(W.w2[mt][0].at(l), bk[0], z);
            z = mma_acc<true>(W.w2[mt][1].at(l), bk[1], z);
#pragma unroll
            for (int i = 0; i < 4; ++i) A.a2[mt][u][i] = tanhf(z[i]);
        }
    }
    // layer 3
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        f32x4 z;
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = (4 * g + i < NS) ? W.b3[(4 * g + i) & (NS - 1)] : 0.f;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = A.a2[2 * ks + (e >> 2)][u][e & 3];
            z = mma_acc<true>(W.w3[ks].at(l), split8(v), z);
        }
        if (g < 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) put_f(u, 4 * g + i, z[i]);
        }
    }
    (void)EXACT;
}

// State Jacobians J = W3 diag(1 - a2^2) W2 diag(1 - a1^2) W1 of the wave's
// samples, column by column: for column c the B operand of the W2 product
// is (1 - a1^2) * W1[:, c] in the chained order, the product's accumulators
// scaled by (1 - a2^2) feed the W3 product.  put_j(u, row, c, value).
template <bool EXACT, class PutJ>
__device__ __forceinline__ void jacobian(const Weights &W, const Acts &A, PutJ put_j)
{
    const int l = lane_id(), g = l >> 4;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        float d1[4][4], d2[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                d1[mt][i] = 1.f - A.a1[mt][u][i] * A.a1[mt][u][i];
                d2[mt][i] = 1.f - A.a2[mt][u][i] * A.a2[mt][u][i];
            }
#pragma unroll 1
        for (int c = 0; c < NS; ++c) {
            Split bk[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = d1[2 * ks + (e >> 2)][e & 3] * W.w1p[ks][g][e][c];
                bk[ks] = split8(v);
            }
            f32x4 p2[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 z = {0.f, 0.f, 0.f, 0.f};
                z = mma_acc<EXACT>(W.w2[mt][0].at(l), bk[0], z);
                p2[mt] = mma_acc<EXACT>(W.w2[mt][1].at(l), bk[1], z);
            }
            f32x4 j = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = d2[2 * ks + (e >> 2)][e & 3] * p2[2 * ks + (e >> 2)][e & 3];
                j = mma_acc<EXACT>(W.w3[ks].at(l), split8(v), j);
            }
            if (g < 2) {
#pragma unroll
                for (int i = 0; i < 4; ++i) put_j(u, 4 * g + i, c, j[i]);
            }
        }
    }
}

} // namespace mlp
} // namespace tvi
