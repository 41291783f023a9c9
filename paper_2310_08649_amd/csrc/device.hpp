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

// ---------------------------------------------------------------------------
// Register-to-register lane moves by DPP (data-parallel primitives: a source
// modifier of an ordinary VALU move, no LDS round trip).  GFX9 controls:
//   quad_perm [1,0,3,2] / [2,3,0,1]   exchange within quads
//   row_shr:d / row_shl:d             lane i of a 16-lane row reads i -/+ d
//   wave_shr:1 / wave_shl:1           lane i reads i -/+ 1 across the wave
//   row_half_mirror / row_mirror      lane i reads 7-i / 15-i within a row
//   row_bcast:15 (rows 1,3 read lanes 15,47), row_bcast:31 (rows 2,3 read 31)
// A lane whose source does not exist, or whose row is masked off, keeps `old`.
// Every lane of the wave must execute these.
// ---------------------------------------------------------------------------
namespace dpp {
constexpr int QUAD_XOR1 = 0xB1, QUAD_XOR2 = 0x4E;
constexpr int ROW_SHL = 0x100, ROW_SHR = 0x110;
constexpr int WAVE_SHL1 = 0x130, WAVE_SHR1 = 0x138;
constexpr int ROW_MIRROR = 0x140, ROW_HALF_MIRROR = 0x141;
constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
} // namespace dpp

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_mov(int old, int x)
{
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_mov(float old, float x)
{
    return __int_as_float(dpp_mov<CTRL, ROWS>(__float_as_int(old), __float_as_int(x)));
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_mov(double old, double x)
{
    const int lo = dpp_mov<CTRL, ROWS>(__double2loint(old), __double2loint(x));
    const int hi = dpp_mov<CTRL, ROWS>(__double2hiint(old), __double2hiint(x));
    return __hiloint2double(hi, lo);
}

// The same moves with zero fill: a lane whose source does not exist, or whose
// row is masked off, gets 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_zero(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_zero(float x)
{
    return __int_as_float(dpp_zero<CTRL, ROWS>(__float_as_int(x)));
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_zero(double x)
{
    const int lo = dpp_zero<CTRL, ROWS>(__double2loint(x));
    const int hi = dpp_zero<CTRL, ROWS>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// The value of x in lane `src` (wave-uniform src), for every lane.
__device__ __forceinline__ int lane_bcast(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ __forceinline__ float lane_bcast(float x, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ __forceinline__ double lane_bcast(double x, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}

// x of lane-1 / lane+1 (0 for lane 0 / lane 63).
template <class R>
__device__ __forceinline__ R lane_prev(R x) { return dpp_zero<dpp::WAVE_SHR1>(x); }
template <class R>
__device__ __forceinline__ R lane_next(R x) { return dpp_zero<dpp::WAVE_SHL1>(x); }

// Sum of x over the S-lane segment of this lane.  Exchanges within quads,
// half rows and rows, then the row sums by lane broadcast: every lane of a
// segment computes the same additions on the same operands (in swapped order
// at most), so all get the bitwise-same, order-fixed result.
template <int S, class R>
__device__ __forceinline__ R seg_sum(R x)
{
    if constexpr (S >= 2) x += dpp_mov<dpp::QUAD_XOR1>(x, x);
    if constexpr (S >= 4) x += dpp_mov<dpp::QUAD_XOR2>(x, x);
    if constexpr (S >= 8) x += dpp_mov<dpp::ROW_HALF_MIRROR>(x, x);
    if constexpr (S >= 16) x += dpp_mov<dpp::ROW_MIRROR>(x, x);
    if constexpr (S >= 32) {
        const R r0 = lane_bcast(x, 0), r1 = lane_bcast(x, 16), r2 = lane_bcast(x, 32), r3 = lane_bcast(x, 48);
        if constexpr (S == 32) x = (lane_id() < 32) ? r0 + r1 : r2 + r3;
        else x = (r0 + r1) + (r2 + r3);
    }
    return x;
}

// Logical and of x != 0 over the S-lane segment (one ballot).
template <int S>
__device__ __forceinline__ int seg_and(int x)
{
    const unsigned long long m = __ballot(x != 0);
    if constexpr (S == kWave) return m == ~0ull ? 1 : 0;
    const int base = lane_id() & ~(S - 1);
    const unsigned long long seg = (1ull << S) - 1ull;
    return ((m >> base) & seg) == seg ? 1 : 0;
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

// X <- A^{-1} X by Gauss-Jordan elimination with partial pivoting: for each
// column the row of largest magnitude among the remaining ones is moved to the
// pivot position by conditional (select) row exchanges, so every register
// index stays static.  A is destroyed.  Returns false if a pivot is zero or
// not finite.
//
// SKIP: the exchange's selects run only where some lane of the wave exchanges
// (blocks I - dt j rarely need one); by default for blocks of 4 x 4 and more,
// where the selects outnumber the test and branch.  RCP takes the pivot's
// reciprocal in double from the hardware estimate and one Newton step
// (r <- r + r (1 - p r)), within an ulp or so of 1/p, for a few instructions
// instead of a correctly rounded division; a zero or non-finite pivot is
// reported all the same.
template <class R>
__device__ __forceinline__ R pivot_reciprocal(R p)
{
    if constexpr (sizeof(R) == 8) {
        const double r0 = __builtin_amdgcn_rcp(p);
        return fma(r0, fma(-p, r0, 1.0), r0);
    } else {
        return R(1) / p;
    }
}

template <int N, class R, bool SKIP = (N >= 4), bool RCP = false>
__device__ __forceinline__ bool gj_solve(R (&A)[N][N], R (&X)[N][N])
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < N; ++c) {
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const bool sw = fabs(A[r][c]) > fabs(A[c][c]);
            if (!SKIP || wave_any(sw)) {
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
        }
        const R piv = A[c][c];
        ok = ok && (piv != R(0)) && finite(piv);
        const R ip = RCP ? pivot_reciprocal(piv) : R(1) / piv;
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

// X = A^{-1} (A destroyed).
template <int N, class R, bool SKIP = (N >= 4), bool RCP = false>
__device__ __forceinline__ bool invert(R (&A)[N][N], R (&X)[N][N])
{
    set_identity(X);
    return gj_solve<N, R, SKIP, RCP>(A, X);
}

// ---------------------------------------------------------------------------
// Affine maps over a segment of S lanes, kept as "identity plus F":
// x -> (I + F) x + z.
//
// A block lower-bidiagonal system with sub-diagonal blocks -I,
//   D_j x_j - x_{j-1} = r_j,
// is the affine recurrence x_j = M_j x_{j-1} + z_j with M_j = D_j^{-1} = I + F_j,
// z_j = D_j^{-1} r_j and x_0 = 0.  One level of parallel cyclic reduction at
// stride d replaces row j's dependence on x_{j-1..} by one on x_{j-d..}:
// z_j <- z_j + M_j z_{j-d},  M_j <- M_j M_{j-d}  (the split of Section 3.2
// with B = -I), i.e. a Kogge-Stone scan with map composition.
//
// Keeping F rather than M makes the identity map all zeros, so a lane move
// that fills missing sources with zero hands the lanes without a partner the
// identity, and every lane composes unconditionally.  For D = I - dt j with
// dt j small (non-stiff steps in float) F = D^{-1} (dt j) also keeps full
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


// F with I + F = (I - E)^{-1}: F = (I - E)^{-1} E.  Returns false on a zero or
// non-finite pivot.
template <int N, class R>
__device__ __forceinline__ bool inverse_plus(const R (&E)[N][N], R (&F)[N][N])
{
    R D[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            D[i][k] = ((i == k) ? R(1) : R(0)) - E[i][k];
            F[i][k] = E[i][k];
        }
    return gj_solve(D, F);  // one solve with right-hand side E
}

// Lane moves of a whole map, element by element (zero fill: identity).
template <int CTRL, int ROWS, int N, class R>
__device__ __forceinline__ void dpp_map(const AffineI<N, R> &a, AffineI<N, R> &o)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) o.F[i][k] = dpp_zero<CTRL, ROWS>(a.F[i][k]);
        o.z[i] = dpp_zero<CTRL, ROWS>(a.z[i]);
    }
}

template <int N, class R>
__device__ __forceinline__ void bcast_map(const AffineI<N, R> &a, int src, AffineI<N, R> &o)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) o.F[i][k] = lane_bcast(a.F[i][k], src);
        o.z[i] = lane_bcast(a.z[i], src);
    }
}

// o <- keep ? o : identity
template <int N, class R>
__device__ __forceinline__ void keep_or_identity(AffineI<N, R> &o, bool keep)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < N; ++k) o.F[i][k] = keep ? o.F[i][k] : R(0);
        o.z[i] = keep ? o.z[i] : R(0);
    }
}

// One Kogge-Stone level at stride D inside 16-lane rows (W = min(S, 16)).
// Row shifts zero-fill at row edges; narrower segments also mask their own edges.
template <int CTRL, int D, int S, bool UP, int N, class R>
__device__ __forceinline__ void scan_level(AffineI<N, R> &a, int q)
{
    constexpr int W = S < 16 ? S : 16;
    if constexpr (D < W) {
        AffineI<N, R> o;
        dpp_map<CTRL + D, 0xF>(a, o);
        if constexpr (S < 16) keep_or_identity(o, UP ? (q >= D) : (q + D < S));
        affine_after(a, o);
    }
}

// Levels of the segment scan: log2(S).
template <int S>
constexpr int scan_levels() { return S >= 64 ? 6 : S >= 32 ? 5 : S >= 16 ? 4 : S >= 8 ? 3 : S >= 4 ? 2 : S >= 2 ? 1 : 0; }

// Inclusive prefix composition over the segment, lowest lane first:
// lane q ends with A_q o A_{q-1} o ... o A_0.  Row shifts inside 16-lane rows,
// then the row totals by row broadcasts (rows 1, 3 take lanes 15, 47; rows 2,
// 3 take lane 31); masked rows receive the identity.
template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_up(AffineI<N, R> &a)
{
    const int q = lane_id() & (S - 1);
    scan_level<dpp::ROW_SHR, 1, S, true>(a, q);
    scan_level<dpp::ROW_SHR, 2, S, true>(a, q);
    scan_level<dpp::ROW_SHR, 4, S, true>(a, q);
    scan_level<dpp::ROW_SHR, 8, S, true>(a, q);
    if constexpr (S >= 32) {
        AffineI<N, R> o;
        dpp_map<dpp::ROW_BCAST15, 0xA>(a, o);
        affine_after(a, o);
    }
    if constexpr (S >= 64) {
        AffineI<N, R> o;
        dpp_map<dpp::ROW_BCAST31, 0xC>(a, o);
        affine_after(a, o);
    }
}

// Inclusive suffix composition, highest lane first:
// lane q ends with A_q o A_{q+1} o ... o A_{S-1}.  Row shifts, then rows 0
// and 2 take the totals of rows 1 and 3 (their first lanes), then rows 0 and
// 1 take the total of rows 2-3 (lane 32), by lane broadcasts.
template <int N, int S, class R>
__device__ __forceinline__ void seg_scan_down(AffineI<N, R> &a)
{
    const int lane = lane_id();
    const int q = lane & (S - 1);
    scan_level<dpp::ROW_SHL, 1, S, false>(a, q);
    scan_level<dpp::ROW_SHL, 2, S, false>(a, q);
    scan_level<dpp::ROW_SHL, 4, S, false>(a, q);
    scan_level<dpp::ROW_SHL, 8, S, false>(a, q);
    if constexpr (S >= 32) {
        AffineI<N, R> h1, h3;
        bcast_map(a, 16, h1);
        bcast_map(a, 48, h3);
        AffineI<N, R> o = (lane & 32) ? h3 : h1;
        keep_or_identity(o, !(lane & 16));
        affine_after(a, o);
    }
    if constexpr (S >= 64) {
        AffineI<N, R> o;
        bcast_map(a, 32, o);
        keep_or_identity(o, !(lane & 32));
        affine_after(a, o);
    }
}

// F of the inverse of the block D: I + F = D^{-1}, via Gauss-Jordan on D
// (partial pivoting).  Returns false on a zero or non-finite pivot.
template <int N, class R, bool SKIP = (N >= 4), bool RCP = false>
__device__ __forceinline__ bool invert_plus(R (&D)[N][N], R (&F)[N][N])
{
    if constexpr (N == 2) {
        // 2 x 2: the adjugate over the determinant (one division).  Elimination
        // with the pivot D00 forms the same determinant, D00 D11 - D01 D10.
        const R det = fma(D[0][0], D[1][1], -(D[0][1] * D[1][0]));
        const R id = RCP ? pivot_reciprocal(det) : R(1) / det;
        F[0][0] = fma(D[1][1], id, R(-1));
        F[0][1] = -D[0][1] * id;
        F[1][0] = -D[1][0] * id;
        F[1][1] = fma(D[0][0], id, R(-1));
        return det != R(0) && finite(det) && finite(id);
    } else {
        const bool ok = invert<N, R, SKIP, RCP>(D, F);
#pragma unroll
        for (int i = 0; i < N; ++i) F[i][i] -= R(1);
        return ok;
    }
}

// y = (I + F)^T x + c   (y may alias x or c)
template <int N, class R>
__device__ __forceinline__ void apply_ip_t(const R (&F)[N][N], const R (&x)[N], const R (&c)[N], R (&y)[N])
{
    R t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R s = c[i];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(F[l][i], x[l], s);
        t[i] = s + x[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = t[i];
}

// Vector from lane src (any lane of the wave; an LDS permute).
template <int N, class R>
__device__ __forceinline__ void vec_read(const R (&v)[N], int src, R (&out)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = lane_read(v[i], src);
}

// Vector of lane-1 / lane+1.
template <int N, class R>
__device__ __forceinline__ void vec_prev(const R (&v)[N], R (&out)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = lane_prev(v[i]);
}

template <int N, class R>
__device__ __forceinline__ void vec_next(const R (&v)[N], R (&out)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = lane_next(v[i]);
}

// IO conversions
template <class IO>
__device__ __forceinline__ double ld(const IO *p) { return static_cast<double>(*p); }
template <class IO>
__device__ __forceinline__ void st(IO *p, double v) { *p = static_cast<IO>(v); }

} // namespace tvi
