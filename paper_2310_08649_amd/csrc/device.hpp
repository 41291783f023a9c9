// Device building blocks for gfx950 (wave64): cross-lane moves, small dense
// block algebra held in registers, and the segmented scans that carry the
// parallel cyclic reduction of a block-bidiagonal chunk system (Section 3.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvi {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite(float x) { return __builtin_isfinite(x); }

// Read `x` from lane `src` (0..63) of the wave.  All lanes must execute it.
__device__ __forceinline__ double lane_read(double x, int src)
{
    const int addr = src << 2;
    int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
    int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int lane_read(int x, int src)
{
    return __builtin_amdgcn_ds_bpermute(src << 2, x);
}

__device__ __forceinline__ float lane_read(float x, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(x)));
}

// Wave-uniform "does any lane satisfy p".
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Sum of x over the S-lane segment of this lane (butterfly; every lane of the
// segment gets the same, order-fixed result).
template <int S, class R>
__device__ __forceinline__ R seg_sum(R x)
{
#pragma unroll
    for (int d = 1; d < S; d <<= 1) x += __shfl_xor(x, d, S);
    return x;
}

template <int S>
__device__ __forceinline__ int seg_and(int x)
{
#pragma unroll
    for (int d = 1; d < S; d <<= 1) x &= __shfl_xor(x, d, S);
    return x;
}

// ---------------------------------------------------------------------------
// n x n blocks in registers (row-major, compile-time n: every index is static,
// so nothing is spilled to scratch).
// ---------------------------------------------------------------------------
template <int N, class R>
__device__ __forceinline__ void set_identity(R (&A)[N][N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) A[i][k] = (i == k) ? R(1) : R(0);
}

// C = A * B
template <int N, class R>
__device__ __forceinline__ void matmul(const R (&A)[N][N], const R (&B)[N][N], R (&C)[N][N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            R s = A[i][0] * B[0][k];
#pragma unroll
            for (int l = 1; l < N; ++l) s = fma(A[i][l], B[l][k], s);
            C[i][k] = s;
        }
}

// y = A x + c   (y may alias c)
template <int N, class R>
__device__ __forceinline__ void matvec_add(const R (&A)[N][N], const R (&x)[N], const R (&c)[N], R (&y)[N])
{
    R t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R s = c[i];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(A[i][l], x[l], s);
        t[i] = s;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = t[i];
}

// y = A^T x + c
template <int N, class R>
__device__ __forceinline__ void matTvec_add(const R (&A)[N][N], const R (&x)[N], const R (&c)[N], R (&y)[N])
{
    R t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R s = c[i];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(A[l][i], x[l], s);
        t[i] = s;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = t[i];
}

// X = A^{-1} by Gauss-Jordan elimination with partial pivoting: for each
// column the row of largest magnitude among the remaining ones is moved to the
// pivot position by conditional (select) row exchanges, so every register
// index stays static.  A is destroyed.  Returns false if a pivot is zero or
// not finite.
template <int N, class R>
__device__ __forceinline__ bool invert(R (&A)[N][N], R (&X)[N][N])
{
    set_identity(X);
    bool ok = true;
#pragma unroll
    for (int c = 0; c < N; ++c) {
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const bool sw = fabs(A[r][c]) > fabs(A[c][c]);
#pragma unroll
            for (int k = c; k < N; ++k) {
                const R a = A[r][k], b = A[c][k];
                A[r][k] = sw ? b : a;
                A[c][k] = sw ? a : b;
            }
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const R a = X[r][k], b = X[c][k];
                X[r][k] = sw ? b : a;
                X[c][k] = sw ? a : b;
            }
        }
        const R piv = A[c][c];
        ok = ok && (piv != R(0)) && finite(piv);
        const R ip = R(1) / piv;
#pragma unroll
        for (int k = c; k < N; ++k) A[c][k] *= ip;
#pragma unroll
        for (int k = 0; k < N; ++k) X[c][k] *= ip;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (r == c) continue;
            const R f = A[r][c];
#pragma unroll
            for (int k = c; k < N; ++k) A[r][k] = fma(-f, A[c][k], A[r][k]);
#pragma unroll
            for (int k = 0; k < N; ++k) X[r][k] = fma(-f, X[c][k], X[r][k]);
        }
    }
    return ok;
}

// ---------------------------------------------------------------------------
// Affine maps v -> M v + z over a segment of S lanes.
//
// A block lower-bidiagonal system with sub-diagonal blocks -I,
//   D_j x_j - x_{j-1} = r_j,
// is the affine recurrence x_j = M_j x_{j-1} + z_j with M_j = D_j^{-1},
// z_j = D_j^{-1} r_j and x_0 = 0.  One level of parallel cyclic reduction at
// stride d replaces row j's dependence on x_{j-1..} by one on x_{j-d..}:
// z_j <- z_j + M_j z_{j-d},  M_j <- M_j M_{j-d}  (the split of Section 3.2
// with B = -I), i.e. a Kogge-Stone scan with map composition.
// ---------------------------------------------------------------------------
template <int N, class R = double>
struct Affine {
    R M[N][N];
    R z[N];
};

template <int N, class R>
__device__ __forceinline__ void affine_identity(Affine<N, R> &a)
{
    set_identity(a.M);
#pragma unroll
    for (int i = 0; i < N; ++i) a.z[i] = R(0);
}

// a <- a o b  (apply b first, then a):  M = Ma Mb,  z = Ma zb + za
template <int N, class R>
__device__ __forceinline__ void affine_after(Affine<N, R> &a, const Affine<N, R> &b)
{
    matvec_add(a.M, b.z, a.z, a.z);
    R t[N][N];
    matmul(a.M, b.M, t);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) a.M[i][k] = t[i][k];
}

template <int N, class R>
__device__ __forceinline__ void affine_read(const Affine<N, R> &a, int src, Affine<N, R> &out)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) out.M[i][k] = lane_read(a.M[i][k], src);
        out.z[i] = lane_read(a.z[i], src);
    }
}

// Inclusive prefix composition over the segment, lowest lane first:
// lane q ends with A_q o A_{q-1} o ... o A_0.
template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_up(Affine<N, R> &a)
{
    const int lane = lane_id();
    const int q = lane & (S - 1);
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
        Affine<N, R> o;
        affine_read(a, q >= d ? lane - d : lane, o);
        if (q >= d) affine_after(a, o);
    }
}

// Inclusive suffix composition, highest lane first:
// lane q ends with A_q o A_{q+1} o ... o A_{S-1}.
template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_down(Affine<N, R> &a)
{
    const int lane = lane_id();
    const int q = lane & (S - 1);
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
        Affine<N, R> o;
        affine_read(a, q + d < S ? lane + d : lane, o);
        if (q + d < S) affine_after(a, o);
    }
}

// ---------------------------------------------------------------------------
// The same maps kept as "identity plus small", x -> (I + F) x + z.  For blocks
// D = I - dt j with dt j small (non-stiff steps in float), I + F = D^{-1}
// with F = D^{-1} (dt j) small, so F and every composition carry full
// relative precision instead of losing it next to the identity.
// ---------------------------------------------------------------------------
template <int N, class R>
struct AffineI {
    R F[N][N];
    R z[N];
};

template <int N, class R>
__device__ __forceinline__ void affine_identity(AffineI<N, R> &a)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) a.F[i][k] = R(0);
        a.z[i] = R(0);
    }
}

// y = (I + F) x + c   (y may alias x or c)
template <int N, class R>
__device__ __forceinline__ void apply_ip(const R (&F)[N][N], const R (&x)[N], const R (&c)[N], R (&y)[N])
{
    R t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R s = c[i];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(F[i][l], x[l], s);
        t[i] = s + x[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = t[i];
}

// a <- a o b:  F = Fa + Fb + Fa Fb,  z = (I + Fa) zb + za
template <int N, class R>
__device__ __forceinline__ void affine_after(AffineI<N, R> &a, const AffineI<N, R> &b)
{
    apply_ip(a.F, b.z, a.z, a.z);
    R t[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            R s = a.F[i][k] + b.F[i][k];
#pragma unroll
            for (int l = 0; l < N; ++l) s = fma(a.F[i][l], b.F[l][k], s);
            t[i][k] = s;
        }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) a.F[i][k] = t[i][k];
}

template <int N, class R>
__device__ __forceinline__ void affine_read(const AffineI<N, R> &a, int src, AffineI<N, R> &out)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) out.F[i][k] = lane_read(a.F[i][k], src);
        out.z[i] = lane_read(a.z[i], src);
    }
}

template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_up(AffineI<N, R> &a)
{
    const int lane = lane_id();
    const int q = lane & (S - 1);
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
        AffineI<N, R> o;
        affine_read(a, q >= d ? lane - d : lane, o);
        if (q >= d) affine_after(a, o);
    }
}

template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_down(AffineI<N, R> &a)
{
    const int lane = lane_id();
    const int q = lane & (S - 1);
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
        AffineI<N, R> o;
        affine_read(a, q + d < S ? lane + d : lane, o);
        if (q + d < S) affine_after(a, o);
    }
}

// F with I + F = (I - E)^{-1}: F = (I - E)^{-1} E.  Returns false on a zero or
// non-finite pivot.
template <int N, class R>
__device__ __forceinline__ bool inverse_plus(const R (&E)[N][N], R (&F)[N][N])
{
    R D[N][N], X[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) D[i][k] = ((i == k) ? R(1) : R(0)) - E[i][k];
    const bool ok = invert(D, X);
    matmul(X, E, F);
    return ok;
}

// Vector of N doubles from lane src.
template <int N, class R>
__device__ __forceinline__ void vec_read(const R (&v)[N], int src, R (&out)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = lane_read(v[i], src);
}

// IO conversions
template <class IO>
__device__ __forceinline__ double ld(const IO *p) { return static_cast<double>(*p); }
template <class IO>
__device__ __forceinline__ void st(IO *p, double v) { *p = static_cast<IO>(v); }

} // namespace tvi
