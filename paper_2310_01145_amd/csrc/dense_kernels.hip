// Dense engine of ParaIEKS (Alg. 2) for large state dimension D (the
// method-of-lines case).  At D = d(q+1) = 192 one tria operand is 2D x 2D
// (590 KB in FP32): no group of lanes can hold an element in registers, so
// one workgroup (4 wavefronts) owns one element operation at a time and the
// element's matrices stay in global memory (L2-resident while it works on
// them).  Every contraction runs on the matrix cores (v_mfma 16x16x4 in
// FP32 or FP64):
//   tria      blocked Householder LQ: panels of 16 reflectors are factored by
//             one wavefront in LDS, the compact-WY trailing update
//             M <- M - ((M Y) T) Y^T is two MFMA products per 16-row stripe;
//   products  16x16 MFMA tiles, one wavefront per tile;
//   solves    blocked triangular solves (MFMA update of the block column,
//             16 x 16 diagonal block per row in registers).
// The scans are Blelloch's two sweeps over the elements of every instance,
// one launch per level; launches use a fixed number of workgroups (each with
// its own scratch slot) that stride over the level's pairs.
//
// Formulas (preconditioned coordinates, increment form delta = Ybar - eta as
// in the row-per-lane kernels):
//   filtering element (eq. sqrt-filtering-elements, prior state 0):
//     Psi = tria([[H sqrtQ], [sqrtQ]]),  K = Psi21 Psi11^{-1},
//     A = Phi - K (H Phi),  b = u - K (H u - r),  sqrtC = Psi22,
//     sqrtJ = (H Phi)^T Psi11^{-T},  eta = sqrtJ Psi11^{-1} (r - H u);
//     step 1 has A = 0, eta = 0, sqrtJ = 0 (its prior is the known state).
//   filtering operator (eq. sqrt-associative-filtering):
//     Xi = tria([[sqrtC_i^T sqrtJ_j, I], [sqrtJ_j, 0]]),  G = sqrtC_i Xi11^{-T},
//     F = I - G Xi21^T,  A_ij = A_j F A_i,
//     b_ij = A_j F (b_i + sqrtC_i sqrtC_i^T eta_j) + b_j,
//     sqrtC_ij = tria([A_j G, sqrtC_j]),
//     eta_ij = A_i^T F^T (eta_j - sqrtJ_j sqrtJ_j^T b_i) + eta_i,
//     sqrtJ_ij = tria([A_i^T Xi22, sqrtJ_i]);
//     when the left operand is a prefix state (A = 0, eta = 0, J = 0) only
//     b_ij and sqrtC_ij are formed.
//   smoothing element (eq. sqrt-smoothing-elements):
//     Pi = tria([[Phi sqrtP, sqrtQ], [sqrtP, 0]]),  E = Pi21 Pi11^{-1},
//     g = m - E (Phi m + u_next),  sqrtL = Pi22;  the last step has E = 0.
//   smoothing operator (eq. sqrt-associative-smoothing):
//     E = E_i E_j,  g = E_i g_j + g_i,  sqrtL = tria([E_i sqrtL_j, sqrtL_i]).
#include <algorithm>

#include "dense.h"

namespace parapn {
namespace dense {

// Threads per workgroup: FP32 workgroups are two wavefronts (four fit a
// compute unit, 30 KB of LDS each at D = 192); FP64 ones need twice the LDS,
// so two per compute unit of four wavefronts each.  Per-element work is
// largely sequential (panel factorisations, row solves), so the number of
// elements in flight sets the throughput.
template <typename T>
__host__ __device__ constexpr int nt_of() { return sizeof(T) == 4 ? 128 : 256; }
constexpr int NB = 16;   // reflectors per panel
// MFMAs per batch of loads in the k loops (4 k-values each): 8 in FP32; 4 in
// FP64, where more loads in flight would cost a wavefront per SIMD
template <typename T>
__host__ __device__ constexpr int kstep_of() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T>
struct MF;
// MFMA 16x16x4 operand layout (both precisions): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator entry v of lane l is
// C[row(l / 16, v)][l % 16] with row(g, v) = 4g + v for f32 and 4v + g for
// f64 (measured on gfx950).
template <>
struct MF<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct MF<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * v + g; }
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }

// ---------------------------------------------------------------------------
// workgroup primitives on row-major matrices in global memory.  Each one
// assumes its inputs are complete and ends with a workgroup barrier.
// ---------------------------------------------------------------------------

// The primitives are not inlined, so a plain pointer parameter is "flat" to
// the compiler, and a flat access counts against the LDS wait counter too:
// every LDS wait would then also wait for the global loads and stores in
// flight.  Operands in global memory are therefore accessed through G<T>
// pointers and the LDS scratch through S<T> pointers.
template <typename T>
using G = __attribute__((address_space(1))) T;
template <typename T>
using S = __attribute__((address_space(3))) T;

// C (m x n) = alpha op(A) op(B) + beta C.  op(A) is m x k: A[i lda + p], or
// A[p lda + i] when ta; op(B) is k x n: B[p ldb + j], or B[j ldb + p] when tb.
// beta == 0: C is not read.  C must not overlap A or B.
template <typename T>
__device__ void wg_gemm(int m, int n, int k, T alpha, const T *A_, int lda, bool ta, const T *B_, int ldb, bool tb,
                        T beta, T *C_, int ldc)
{
    const G<T> *A = (const G<T> *)A_, *B = (const G<T> *)B_;
    G<T> *C = (G<T> *)C_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
    for (int t = wv; t < tm * tn; t += NW) {
        const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
        const int ia = i0 + li, jb = j0 + li;
        const bool rok = ia < m, cok = jb < n;
        typename MF<T>::v4 acc = {T(0), T(0), T(0), T(0)};
        // 4U values of k per step, all loads issued before the U MFMAs; lane
        // group g takes k = p0 + U g + u in MFMA u (the same k for A and B)
        constexpr int U = kstep_of<T>();
        int p0 = 0;
        for (; p0 + 4 * U <= k; p0 += 4 * U) {
            T a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + U * lg + u;
                a[u] = rok ? (ta ? A[(size_t)p * lda + ia] : A[(size_t)ia * lda + p]) : T(0);
                b[u] = cok ? (tb ? B[(size_t)jb * ldb + p] : B[(size_t)p * ldb + jb]) : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = MF<T>::mma(a[u], b[u], acc);
        }
        for (; p0 < k; p0 += 4) {
            const int p = p0 + lg;
            T a = T(0), b = T(0);
            if (rok && p < k) a = ta ? A[(size_t)p * lda + ia] : A[(size_t)ia * lda + p];
            if (cok && p < k) b = tb ? B[(size_t)jb * ldb + p] : B[(size_t)p * ldb + jb];
            acc = MF<T>::mma(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + MF<T>::row(lg, v), j = j0 + li;
            if (i < m && j < n) {
                T x = alpha * acc[v];
                if (beta != T(0)) x += beta * C[(size_t)i * ldc + j];
                C[(size_t)i * ldc + j] = x;
            }
        }
    }
    __syncthreads();
}

// y (m) = alpha op(A) x + beta y, op(A) m x k (A[i lda + j], or A[j lda + i]
// when ta).  beta == 0: y is not read.  y must not overlap A or x.
template <typename T>
__device__ void wg_gemv(int m, int k, T alpha, const T *A_, int lda, bool ta, const T *x_, T beta, T *y_)
{
    const G<T> *A = (const G<T> *)A_, *x = (const G<T> *)x_;
    G<T> *y = (G<T> *)y_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    for (int i = threadIdx.x; i < m; i += NT) {
        T s = T(0);
        if (ta)
            for (int j = 0; j < k; ++j) s += A[(size_t)j * lda + i] * x[j];
        else
            for (int j = 0; j < k; ++j) s += A[(size_t)i * lda + j] * x[j];
        y[i] = alpha * s + (beta != T(0) ? beta * y[i] : T(0));
    }
    __syncthreads();
}

// dst (m x n) = src, or zero where src is null
template <typename T>
__device__ void wg_copy(T *dst_, int ldd, const T *src_, int ldsrc, int m, int n)
{
    G<T> *dst = (G<T> *)dst_;
    const G<T> *src = (const G<T> *)src_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    for (int e = threadIdx.x; e < m * n; e += NT) {
        const int i = e / n, j = e - i * n;
        dst[(size_t)i * ldd + j] = src ? src[(size_t)i * ldsrc + j] : T(0);
    }
    __syncthreads();
}

template <typename T>
__device__ void wg_vcopy(T *dst_, const T *src_, int n)
{
    G<T> *dst = (G<T> *)dst_;
    const G<T> *src = (const G<T> *)src_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    for (int i = threadIdx.x; i < n; i += NT) dst[i] = src ? src[i] : T(0);
    __syncthreads();
}

// One wavefront: Householder LQ of the nb x w panel P (row stride w) in LDS.
// Row j's reflector H_j = I - tau_j v_j v_j^T (v_j[c] = 0 for c < j, 1 at j,
// stored in P[j][c > j]) zeroes row j right of the diagonal; the diagonal
// entry goes to P[j][j], and rows below get H_j applied.  Then the compact-WY
// factor Tm (NB x NB, upper triangular, zero outside nb x nb) with
// H_0 H_1 ... H_{nb-1} = I - Y Tm Y^T, Y = [v_0 .. v_{nb-1}].
template <typename T>
__device__ void panel_factor(T *P_, int nb, int w, T *Tm_, T *Z_, T *tau_)
{
    S<T> *P = (S<T> *)P_, *Tm = (S<T> *)Tm_, *Z = (S<T> *)Z_, *tau = (S<T> *)tau_;
    const int lane = threadIdx.x & 63;
    for (int j = 0; j < nb; ++j) {
        S<T> *pj = P + j * w;
        T s = T(0);
        for (int c = j + 1 + lane; c < w; c += 64) s += pj[c] * pj[c];
        s = wave_sum(s);
        const T al = pj[j];
        T be = al, tj = T(0), sc = T(0);
        if (s > T(0)) {
            const T nr = dsqrt(al * al + s);
            be = al > T(0) ? -nr : nr;
            tj = (be - al) / be;
            sc = T(1) / (al - be);
        }
        for (int c = j + 1 + lane; c < w; c += 64) pj[c] *= sc;
        wave_sync();
        if (lane == 0) {
            pj[j] = be;
            tau[j] = tj;
        }
        wave_sync();
        for (int r = j + 1; r < nb; ++r) {
            S<T> *pr = P + r * w;
            T dt = T(0);
            for (int c = j + 1 + lane; c < w; c += 64) dt += pr[c] * pj[c];
            dt = wave_sum(dt) + pr[j];
            const T f = tj * dt;
            for (int c = j + 1 + lane; c < w; c += 64) pr[c] -= f * pj[c];
            wave_sync();
            if (lane == 0) pr[j] -= f;
            wave_sync();
        }
    }
    // Z[i][j] = v_i . v_j (i < j); v_j vanishes left of j and is 1 at j
    for (int e = lane; e < NB * NB; e += 64) {
        const int i = e / NB, j = e - i * NB;
        T z = T(0);
        if (i < j && j < nb) {
            const S<T> *pi = P + i * w, *pj = P + j * w;
            z = pi[j];
            for (int c = j + 1; c < w; ++c) z += pi[c] * pj[c];
        }
        Z[e] = z;
        Tm[e] = T(0);
    }
    wave_sync();
    // T[j][j] = tau_j,  T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] Z[l][j]
    for (int j = 0; j < nb; ++j) {
        T v = T(0);
        if (lane < j) {
            for (int l = lane; l < j; ++l) v += Tm[lane * NB + l] * Z[l * NB + j];
            v = -tau[j] * v;
        }
        wave_sync();
        if (lane < j) Tm[lane * NB + j] = v;
        if (lane == j) Tm[j * NB + j] = tau[j];
        wave_sync();
    }
}

// LDS elements the workgroup primitives need for operands up to nmax columns
template <typename T>
__host__ __device__ constexpr int smem_elems(int nmax) { return NB * nmax + 2 * NB * NB + NB + (nt_of<T>() / 64) * 256; }

// tria in place: the m x n matrix M (row stride ld) becomes the lower-
// trapezoidal L (columns >= min(m, n) zero) with L L^T = M M^T, M = L Q.
// sm: smem_elems(n) elements of LDS.
template <typename T>
__device__ void wg_tria(T *M_, int m, int n, int ld, T *sm)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    G<T> *M = (G<T> *)M_;
    S<T> *P = (S<T> *)sm;
    S<T> *Tm = P + NB * n;
    S<T> *Z = Tm + NB * NB;
    S<T> *tau = Z + NB * NB;
    S<T> *Wb = tau + NB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    const int kmax = m < n ? m : n;
    for (int k0 = 0; k0 < kmax; k0 += NB) {
        const int nb = min(NB, kmax - k0), w = n - k0;
        for (int e = threadIdx.x; e < nb * w; e += NT) {
            const int j = e / w, c = e - j * w;
            P[e] = M[(size_t)(k0 + j) * ld + k0 + c];
        }
        __syncthreads();
        if (wv == 0) panel_factor((T *)P, nb, w, (T *)Tm, (T *)Z, (T *)tau);
        __syncthreads();
        // trailing rows: M_t <- M_t - ((M_t Y) Tm) Y^T over columns k0..n-1
        const int r0s = k0 + nb, nst = (m - r0s + 15) >> 4;
        S<T> *Wl = Wb + wv * 256;
        for (int st = wv; st < nst; st += NW) {
            const int r0 = r0s + (st << 4);
            const int ra = r0 + li;
            const G<T> *mrow = M + (size_t)ra * ld + k0;
            typename MF<T>::v4 acc = {T(0), T(0), T(0), T(0)};
            const bool rok = ra < m;
            constexpr int U = kstep_of<T>();
            for (int c0 = 0; c0 < w; c0 += 4 * U) {
                T a[U], b[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = c0 + U * lg + u;
                    a[u] = (rok && c < w) ? mrow[c] : T(0);
                    b[u] = T(0);
                    if (li < nb && c < w) b[u] = c < li ? T(0) : (c == li ? T(1) : P[li * w + c]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) acc = MF<T>::mma(a[u], b[u], acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) Wl[MF<T>::row(lg, v) * 16 + li] = acc[v];
            wave_sync();
            T wt[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T s = T(0);
                if (li < nb)
                    for (int l = 0; l <= li; ++l) s += Wl[MF<T>::row(lg, v) * 16 + l] * Tm[l * NB + li];
                wt[v] = s;
            }
            wave_sync();
#pragma unroll
            for (int v = 0; v < 4; ++v) Wl[MF<T>::row(lg, v) * 16 + li] = -wt[v];
            wave_sync();
            typename MF<T>::v4 nx;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + MF<T>::row(lg, v);
                nx[v] = (r < m && li < w) ? M[(size_t)r * ld + k0 + li] : T(0);
            }
            for (int c0 = 0; c0 < w; c0 += 16) {
                const int c = c0 + li;
                typename MF<T>::v4 cc = nx;
                // the next tile's loads are in flight during this tile's MFMAs
                if (c0 + 16 < w) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = r0 + MF<T>::row(lg, v);
                        nx[v] = (r < m && c + 16 < w) ? M[(size_t)r * ld + k0 + c + 16] : T(0);
                    }
                }
#pragma unroll
                for (int l0 = 0; l0 < 16; l0 += 4) {
                    const int l = l0 + lg;
                    const T a = Wl[li * 16 + l];
                    T b = T(0);
                    if (l < nb && c < w) b = c < l ? T(0) : (c == l ? T(1) : P[l * w + c]);
                    cc = MF<T>::mma(a, b, cc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + MF<T>::row(lg, v);
                    if (r < m && c < w) M[(size_t)r * ld + k0 + c] = cc[v];
                }
            }
            wave_sync();
        }
        // the panel rows: their L entries, zeros right of the diagonal
        for (int e = threadIdx.x; e < nb * w; e += NT) {
            const int j = e / w, c = e - j * w;
            M[(size_t)(k0 + j) * ld + k0 + c] = c <= j ? P[e] : T(0);
        }
        __syncthreads();
    }
}

// In place on X (m x k, row stride ldx), L lower k x k nonsingular:
// TRANS: X <- X L^{-T} (solves X L^T = B, column blocks left to right);
// else   X <- X L^{-1} (solves X L = B, column blocks right to left).
template <typename T, bool TRANS>
__device__ void wg_trsm(T *X_, int m, int k, int ldx, const T *L_, int ldl)
{
    G<T> *X = (G<T> *)X_;
    const G<T> *L = (const G<T> *)L_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    const int nblk = (k + 15) >> 4;
    for (int bi = 0; bi < nblk; ++bi) {
        const int jb = TRANS ? bi : nblk - 1 - bi;
        const int j0 = jb << 4, nbk = min(16, k - j0), j1 = j0 + nbk;
        if (TRANS) {
            if (j0 > 0)
                wg_gemm<T>(m, nbk, j0, T(-1), X_, ldx, false, L_ + (size_t)j0 * ldl, ldl, true, T(1), X_ + j0, ldx);
        } else {
            if (j1 < k)
                wg_gemm<T>(m, nbk, k - j1, T(-1), X_ + j1, ldx, false, L_ + (size_t)j1 * ldl + j0, ldl, false, T(1),
                           X_ + j0, ldx);
        }
        // the diagonal block, one row per thread (the row stays in L1)
        const G<T> *Lb = L + (size_t)j0 * ldl + j0;
        for (int r = threadIdx.x; r < m; r += NT) {
            G<T> *xr = X + (size_t)r * ldx + j0;
            if (sizeof(T) == 4 && TRANS && nbk == 16) {
                // a full block of the forward solve in registers (FP32 only:
                // in FP64 the block would push the combine kernel into spills)
                T x[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) x[c] = xr[c];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    T s = x[j];
#pragma unroll
                    for (int c = 0; c < j; ++c) s -= x[c] * Lb[(size_t)j * ldl + c];
                    x[j] = s / Lb[(size_t)j * ldl + j];
                }
#pragma unroll
                for (int c = 0; c < 16; ++c) xr[c] = x[c];
                continue;
            }
            if (TRANS) {
                for (int j = 0; j < nbk; ++j) {
                    T s = xr[j];
                    for (int c = 0; c < j; ++c) s -= xr[c] * Lb[(size_t)j * ldl + c];
                    xr[j] = s / Lb[(size_t)j * ldl + j];
                }
            } else {
                for (int j = nbk - 1; j >= 0; --j) {
                    T s = xr[j];
                    for (int c = j + 1; c < nbk; ++c) s -= xr[c] * Lb[(size_t)c * ldl + j];
                    xr[j] = s / Lb[(size_t)j * ldl + j];
                }
            }
        }
        __syncthreads();
    }
}

// z = L^{-1} v for lower k x k L (k <= NW * 256), one wavefront, column-
// oriented forward substitution through LDS; z may alias v.
template <typename T>
__device__ void wg_lower_solve_vec(const T *L_, int ldl, int k, const T *v_, T *z_, T *sm_)
{
    const G<T> *L = (const G<T> *)L_, *v = (const G<T> *)v_;
    G<T> *z = (G<T> *)z_;
    S<T> *sm = (S<T> *)sm_;
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    for (int i = threadIdx.x; i < k; i += NT) sm[i] = v[i];
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        for (int j = 0; j < k; ++j) {
            const T zj = sm[j] / L[(size_t)j * ldl + j];
            wave_sync();
            if (lane == 0) sm[j] = zj;
            for (int i = j + 1 + lane; i < k; i += 64) sm[i] -= L[(size_t)i * ldl + j] * zj;
            wave_sync();
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += NT) z[i] = sm[i];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the model
// ---------------------------------------------------------------------------
// Method-of-lines heat/reaction chain on d periodic grid points, dx = 1/d:
// f_i = nu (y_{i-1} - 2 y_i + y_{i+1}) / dx^2 + y_i (1 - y_i).
__device__ __forceinline__ double mol_f(const DenseModel &md, const double *y, int i)
{
    const int d = md.d;
    const double k = md.p[0] * (double)d * (double)d;
    const double um = y[(i + d - 1) % d], up = y[(i + 1) % d], u = y[i];
    return k * (um - 2.0 * u + up) + u * (1.0 - u);
}
__device__ __forceinline__ double mol_jac(const DenseModel &md, const double *y, int i, int j)
{
    const int d = md.d;
    const double k = md.p[0] * (double)d * (double)d;
    double v = 0.0;
    if (j == (i + d - 1) % d) v += k;
    if (j == (i + 1) % d) v += k;
    if (j == i) v += -2.0 * k + 1.0 - 2.0 * y[i];
    return v;
}

__host__ __device__ inline size_t dense_scratch_elems_dev(int D) { return (size_t)11 * D * D + 8 * D + 64; }

template <typename T>
struct Views {
    T *A, *b, *C, *e, *J, *E, *g, *L;
    __device__ Views(const DenseWork &w)
        : A((T *)w.A), b((T *)w.b), C((T *)w.C), e((T *)w.e), J((T *)w.J), E((T *)w.E), g((T *)w.g), L((T *)w.L)
    {
    }
};

__device__ __forceinline__ bool inactive(const DenseWork &w, int b) { return w.active && w.active[b] == 0; }

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// linearisation (EK1, Sec. 3.2.1) and the filtering element of every step
template <typename T>
__global__ __launch_bounds__(nt_of<T>()) void k_elements(DenseModel md, DenseWork w)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    Views<T> V(w);
    const int D = md.D, d = md.d, S = md.q + 1;
    const int64_t N = md.N, total = (int64_t)md.B * N;
    const size_t DD = (size_t)D * D;
    T *scr = (T *)w.scratch + (size_t)blockIdx.x * dense_scratch_elems_dev(D);
    T *Sst = scr;                         // (d + D) x D
    T *HJ = Sst + (size_t)(d + D) * D;    // d x d: -(h/q) F_y
    T *HP = HJ + (size_t)d * d;           // d x D: H Phi
    T *KT = HP + (size_t)d * D;           // D x d
    T *r = KT + (size_t)D * d;            // d
    T *u = r + d;                         // D
    T *v = u + D;                         // d
    T *z = v + d;                         // d
    double *y = (double *)(z + d + 8);    // d doubles (8 T of slack keeps it 8-byte aligned for float)
    y = (double *)(((uintptr_t)y + 7) & ~(uintptr_t)7);
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = (int)(item / N);
        const int64_t k = item - (int64_t)b * N;
        if (inactive(w, b)) continue;
        const double *tr = w.traj + (size_t)b * w.traj_stride;
        const double *eta = tr + (size_t)(k + 1) * D, *etap = tr + (size_t)k * D;
        for (int i = threadIdx.x; i < d; i += NT) y[i] = md.T0 * eta[i * S];
        __syncthreads();
        for (int i = threadIdx.x; i < d; i += NT) r[i] = (T)((mol_f(md, y, i) - md.T1 * eta[i * S + 1]) / md.T1);
        for (int e = threadIdx.x; e < d * d; e += NT) {
            const int i = e / d, j = e - i * d;
            HJ[e] = (T)(-md.hq * mol_jac(md, y, i, j));
        }
        for (int rho = threadIdx.x; rho < D; rho += NT) {
            const int i = rho / S, a = rho - i * S;
            double s = -eta[rho];
            for (int c = 0; c < S; ++c) s += md.phib[a * 5 + c] * etap[i * S + c];
            u[rho] = (T)s;
        }
        __syncthreads();
        // stack [[H sqrtQ], [sqrtQ]] and H Phi (H = E1 + HJ E0, blocks are I_d (x) block)
        for (int e = threadIdx.x; e < (d + D) * D; e += NT) {
            const int row = e / D, col = e - row * D, j = col / S, c = col - j * S;
            T x;
            if (row < d) {
                x = (T)(row == j ? md.sqb[5 + c] : 0.0) + HJ[row * d + j] * (T)md.sqb[c];
            } else {
                const int rr = row - d, i2 = rr / S, a = rr - i2 * S;
                x = i2 == j ? (T)md.sqb[a * 5 + c] : T(0);
            }
            Sst[e] = x;
        }
        for (int e = threadIdx.x; e < d * D; e += NT) {
            const int row = e / D, col = e - row * D, j = col / S, c = col - j * S;
            HP[e] = (T)(row == j ? md.phib[5 + c] : 0.0) + HJ[row * d + j] * (T)md.phib[c];
        }
        // v = H u - r
        for (int i = threadIdx.x; i < d; i += NT) {
            T s = u[i * S + 1] - r[i];
            for (int j = 0; j < d; ++j) s += HJ[i * d + j] * u[j * S];
            v[i] = s;
        }
        __syncthreads();
        wg_tria<T>(Sst, d + D, D, D, sm);
        T *K = Sst + (size_t)d * D;  // Psi21 -> K (D x d, row stride D)
        wg_trsm<T, false>(K, D, d, D, Sst, D);
        const size_t el = (size_t)item;
        T *Ao = V.A + el * DD, *bo = V.b + el * D, *Co = V.C + el * DD, *eo = V.e + el * D, *Jo = V.J + el * DD;
        // b = u - K v
        wg_vcopy<T>(bo, u, D);
        wg_gemv<T>(D, d, T(-1), K, D, false, v, T(1), bo);
        // sqrtC = Psi22, zero padded
        for (int e = threadIdx.x; e < D * D; e += NT) {
            const int row = e / D, c = e - row * D;
            Co[e] = c < D - d ? Sst[(size_t)(d + row) * D + d + c] : T(0);
        }
        if (k == 0) {
            for (int e = threadIdx.x; e < D * D; e += NT) {
                Ao[e] = T(0);
                Jo[e] = T(0);
            }
            for (int i = threadIdx.x; i < D; i += NT) eo[i] = T(0);
            __syncthreads();
            continue;
        }
        // A = Phi - K (H Phi)
        for (int e = threadIdx.x; e < D * D; e += NT) {
            const int row = e / D, col = e - row * D, i = row / S, a = row - i * S, j = col / S, c = col - j * S;
            Ao[e] = i == j ? (T)md.phib[a * 5 + c] : T(0);
        }
        // KT = (H Phi)^T
        for (int e = threadIdx.x; e < D * d; e += NT) {
            const int row = e / d, c = e - row * d;
            KT[e] = HP[(size_t)c * D + row];
        }
        __syncthreads();
        wg_gemm<T>(D, D, d, T(-1), K, D, false, HP, D, false, T(1), Ao, D);
        // sqrtJ = (H Phi)^T Psi11^{-T}
        wg_trsm<T, true>(KT, D, d, d, Sst, D);
        wg_copy<T>(Jo, D, KT, d, D, d);
        wg_copy<T>(Jo + d, D, (const T *)nullptr, 0, D, D - d);
        // eta = sqrtJ Psi11^{-1} (r - H u) = sqrtJ Psi11^{-1} (-v)
        wg_lower_solve_vec<T>(Sst, D, d, v, z, sm);
        wg_gemv<T>(D, d, T(-1), KT, d, false, z, T(0), eo);
    }
}

// filtering operator on one pair (left earlier, right later); the result
// replaces the right element.  state: the left operand is a prefix state.
template <typename T>
__device__ void fcombine_pair(const DenseModel &md, Views<T> &V, int64_t li_, int64_t ri_, bool state, T *scr,
                              T *sm)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    const int D = md.D, D2 = 2 * D;
    const size_t DD = (size_t)D * D;
    const T *Ai = V.A + li_ * DD, *bi = V.b + li_ * D, *Ci = V.C + li_ * DD, *ei = V.e + li_ * D,
            *Ji = V.J + li_ * DD;
    T *Aj = V.A + ri_ * DD, *bj = V.b + ri_ * D, *Cj = V.C + ri_ * DD, *ej = V.e + ri_ * D, *Jj = V.J + ri_ * DD;
    T *Sx = scr;            // 2D x 2D
    T *G = Sx + 4 * DD;     // D x D
    T *F = G + DD;          // D x D
    T *TM = F + DD;         // D x D
    T *X1 = TM + DD;        // D x 2D
    T *X2 = X1 + 2 * DD;    // D x 2D
    T *v1 = X2 + 2 * DD, *v2 = v1 + D, *v3 = v2 + D;
    // Xi stack [[C_i^T J_j, I], [J_j, 0]]
    for (int e = threadIdx.x; e < D2 * D2; e += NT) {
        const int row = e / D2, col = e - row * D2;
        if (row < D && col < D) continue;
        T x = T(0);
        if (row < D)
            x = (col - D == row) ? T(1) : T(0);
        else if (col < D)
            x = Jj[(size_t)(row - D) * D + col];
        Sx[e] = x;
    }
    wg_gemm<T>(D, D, D, T(1), Ci, D, true, Jj, D, false, T(0), Sx, D2);
    wg_tria<T>(Sx, D2, D2, D2, sm);
    // G = C_i Xi11^{-T};  F = I - G Xi21^T
    wg_copy<T>(G, D, Ci, D, D, D);
    for (int e = threadIdx.x; e < D * D; e += NT) {
        const int row = e / D, col = e - row * D;
        F[e] = row == col ? T(1) : T(0);
    }
    wg_trsm<T, true>(G, D, D, D, Sx, D2);
    wg_gemm<T>(D, D, D, T(-1), G, D, false, Sx + (size_t)D * D2, D2, true, T(1), F, D);
    // TM = A_j F;  b_ij = TM (b_i + C_i C_i^T e_j) + b_j
    wg_gemm<T>(D, D, D, T(1), Aj, D, false, F, D, false, T(0), TM, D);
    wg_gemv<T>(D, D, T(1), Ci, D, true, ej, T(0), v1);
    wg_vcopy<T>(v2, bi, D);
    wg_gemv<T>(D, D, T(1), Ci, D, false, v1, T(1), v2);
    wg_vcopy<T>(v3, bj, D);
    wg_gemv<T>(D, D, T(1), TM, D, false, v2, T(1), v3);
    // C_ij = tria([A_j G, C_j])
    wg_copy<T>(X1 + D, D2, Cj, D, D, D);
    wg_gemm<T>(D, D, D, T(1), Aj, D, false, G, D, false, T(0), X1, D2);
    wg_tria<T>(X1, D, D2, D2, sm);
    wg_copy<T>(Cj, D, X1, D2, D, D);
    wg_vcopy<T>(bj, v3, D);
    if (state) {
        for (int e = threadIdx.x; e < D * D; e += NT) {
            Aj[e] = T(0);
            Jj[e] = T(0);
        }
        for (int i = threadIdx.x; i < D; i += NT) ej[i] = T(0);
        __syncthreads();
        return;
    }
    // A_ij = TM A_i
    wg_gemm<T>(D, D, D, T(1), TM, D, false, Ai, D, false, T(0), Aj, D);
    // e_ij = A_i^T F^T (e_j - J_j J_j^T b_i) + e_i
    wg_gemv<T>(D, D, T(1), Jj, D, true, bi, T(0), v1);
    wg_vcopy<T>(v2, ej, D);
    wg_gemv<T>(D, D, T(-1), Jj, D, false, v1, T(1), v2);
    wg_gemv<T>(D, D, T(1), F, D, true, v2, T(0), v1);
    wg_vcopy<T>(v3, ei, D);
    wg_gemv<T>(D, D, T(1), Ai, D, true, v1, T(1), v3);
    // J_ij = tria([A_i^T Xi22, J_i])
    wg_copy<T>(X2 + D, D2, Ji, D, D, D);
    wg_gemm<T>(D, D, D, T(1), Ai, D, true, Sx + (size_t)D * D2 + D, D2, false, T(0), X2, D2);
    wg_tria<T>(X2, D, D2, D2, sm);
    wg_copy<T>(Jj, D, X2, D2, D, D);
    wg_vcopy<T>(ej, v3, D);
}

// Blelloch level of the filtering scan.  up: pairs (r - s, r) with
// r = 2s(p + 1) - 1 (pair 0's left operand starts at step 1: a state);
// down: r = 2s(p + 1) + s - 1, whose left operand is a complete prefix.
template <typename T>
__global__ __launch_bounds__(nt_of<T>()) void k_fcombine(DenseModel md, DenseWork w, int64_t s, int up, int64_t npairs)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    Views<T> V(w);
    T *scr = (T *)w.scratch + (size_t)blockIdx.x * dense_scratch_elems_dev(md.D);
    const int64_t total = (int64_t)md.B * npairs;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = (int)(item / npairs);
        const int64_t p = item - (int64_t)b * npairs;
        if (inactive(w, b)) continue;
        const int64_t r = up ? 2 * s * (p + 1) - 1 : 2 * s * (p + 1) + s - 1;
        const int64_t base = (int64_t)b * md.N;
        fcombine_pair<T>(md, V, base + r - s, base + r, !up || p == 0, scr, sm);
    }
}

// smoothing element of every step from its filtering marginal (m, sqrtP) in
// (b, C); with_L also stores sqrtL.
template <typename T>
__global__ __launch_bounds__(nt_of<T>()) void k_selements(DenseModel md, DenseWork w, int with_L)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    Views<T> V(w);
    const int D = md.D, D2 = 2 * D, S = md.q + 1;
    const size_t DD = (size_t)D * D;
    const int64_t N = md.N, total = (int64_t)md.B * N;
    T *scr = (T *)w.scratch + (size_t)blockIdx.x * dense_scratch_elems_dev(D);
    T *Sx = scr, *v1 = Sx + 4 * DD, *v2 = v1 + D;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = (int)(item / N);
        const int64_t k = item - (int64_t)b * N;
        if (inactive(w, b)) continue;
        const T *Pf = V.C + (size_t)item * DD, *mf = V.b + (size_t)item * D;
        T *Eo = V.E + (size_t)item * DD, *go = V.g + (size_t)item * D;
        if (k == N - 1) {
            for (int e = threadIdx.x; e < D * D; e += NT) {
                Eo[e] = T(0);
                if (with_L) V.L[(size_t)item * DD + e] = Pf[e];
            }
            for (int i = threadIdx.x; i < D; i += NT) go[i] = mf[i];
            __syncthreads();
            continue;
        }
        // [[Phi sqrtP, sqrtQ], [sqrtP, 0]]
        for (int e = threadIdx.x; e < D2 * D2; e += NT) {
            const int row = e / D2, col = e - row * D2;
            T x = T(0);
            if (row < D) {
                const int i = row / S, a = row - i * S;
                if (col < D) {
                    for (int c = 0; c < S; ++c) x += (T)md.phib[a * 5 + c] * Pf[(size_t)(i * S + c) * D + col];
                } else {
                    const int cc = col - D, j = cc / S, c = cc - j * S;
                    x = i == j ? (T)md.sqb[a * 5 + c] : T(0);
                }
            } else if (col < D) {
                x = Pf[(size_t)(row - D) * D + col];
            }
            Sx[e] = x;
        }
        // m- = Phi m + u_{n+1}, u_{n+1} = Phi eta_n - eta_{n+1} (step n = k + 1)
        const double *tr = w.traj + (size_t)b * w.traj_stride;
        const double *e0 = tr + (size_t)(k + 1) * D, *e1 = tr + (size_t)(k + 2) * D;
        for (int rho = threadIdx.x; rho < D; rho += NT) {
            const int i = rho / S, a = rho - i * S;
            double uu = -e1[rho];
            T pm = T(0);
            for (int c = 0; c < S; ++c) {
                uu += md.phib[a * 5 + c] * e0[i * S + c];
                pm += (T)md.phib[a * 5 + c] * mf[i * S + c];
            }
            v1[rho] = pm + (T)uu;
            v2[rho] = mf[rho];
        }
        __syncthreads();
        wg_tria<T>(Sx, D2, D2, D2, sm);
        T *Eb = Sx + (size_t)D * D2;  // Pi21 -> E
        wg_trsm<T, false>(Eb, D, D, D2, Sx, D2);
        wg_gemv<T>(D, D, T(-1), Eb, D2, false, v1, T(1), v2);
        wg_copy<T>(Eo, D, Eb, D2, D, D);
        if (with_L) wg_copy<T>(V.L + (size_t)item * DD, D, Eb + D, D2, D, D);
        wg_vcopy<T>(go, v2, D);
    }
}

// Blelloch level of the smoothing (suffix) scan, on reversed positions:
// position x is step index N-1-x.  The earlier element of a pair absorbs the
// later one; state: the later operand contains the last step (E = 0).
template <typename T>
__global__ __launch_bounds__(nt_of<T>()) void k_bcombine(DenseModel md, DenseWork w, int64_t s, int up, int64_t npairs,
                                                 int with_L)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    Views<T> V(w);
    const int D = md.D, D2 = 2 * D;
    const size_t DD = (size_t)D * D;
    T *scr = (T *)w.scratch + (size_t)blockIdx.x * dense_scratch_elems_dev(D);
    T *X1 = scr, *TM = X1 + 2 * DD, *v1 = TM + DD;
    const int64_t total = (int64_t)md.B * npairs;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = (int)(item / npairs);
        const int64_t p = item - (int64_t)b * npairs;
        if (inactive(w, b)) continue;
        const int64_t r = up ? 2 * s * (p + 1) - 1 : 2 * s * (p + 1) + s - 1;
        const int64_t base = (int64_t)b * md.N;
        const int64_t self = base + md.N - 1 - r, part = self + s;
        const bool state = !up || p == 0;
        T *Es = V.E + self * DD, *gs = V.g + self * D;
        const T *Ep = V.E + part * DD, *gp = V.g + part * D;
        wg_vcopy<T>(v1, gs, D);
        wg_gemv<T>(D, D, T(1), Es, D, false, gp, T(1), v1);
        if (with_L) {
            wg_copy<T>(X1 + D, D2, V.L + self * DD, D, D, D);
            wg_gemm<T>(D, D, D, T(1), Es, D, false, V.L + part * DD, D, false, T(0), X1, D2);
            wg_tria<T>(X1, D, D2, D2, sm);
            wg_copy<T>(V.L + self * DD, D, X1, D2, D, D);
        }
        if (!state) {
            wg_gemm<T>(D, D, D, T(1), Es, D, false, Ep, D, false, T(0), TM, D);
            wg_copy<T>(Es, D, TM, D, D, D);
        } else {
            wg_copy<T>(Es, D, (const T *)nullptr, 0, D, D);
        }
        wg_vcopy<T>(gs, v1, D);
    }
}

__device__ __forceinline__ double nan_max(double x, double u) { return (u > x || u != u) ? u : x; }

// trajectory update eta += delta (FP64) and the two maxima of the stopping
// test, per instance: blockIdx.y = instance
template <typename T>
__global__ __launch_bounds__(nt_of<T>()) void k_update(DenseModel md, DenseWork w)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    const int b = blockIdx.y;
    if (inactive(w, b)) return;
    const int D = md.D, S = md.q + 1;
    const int64_t n_el = md.N * D;
    double *tr = w.traj + (size_t)b * w.traj_stride + D;
    const T *g = (const T *)w.g + (size_t)b * n_el;
    double dmax = 0.0, mmax = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n_el; i += (int64_t)gridDim.x * NT) {
        const double dl = (double)g[i];
        const double nw = tr[i] + dl;
        tr[i] = nw;
        if ((int)(i % D) % S == 0) {
            dmax = nan_max(dmax, fabs(md.T0 * dl));
            mmax = nan_max(mmax, fabs(md.T0 * nw));
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        dmax = nan_max(dmax, __shfl_xor(dmax, o));
        mmax = nan_max(mmax, __shfl_xor(mmax, o));
    }
    __shared__ double red[2 * NW];
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = dmax;
        red[NW + (threadIdx.x >> 6)] = mmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) {
            dmax = nan_max(dmax, red[i]);
            mmax = nan_max(mmax, red[NW + i]);
        }
        atomicMax(w.dbits + 2 * b, (unsigned long long)__double_as_longlong(dmax));
        atomicMax(w.dbits + 2 * b + 1, (unsigned long long)__double_as_longlong(mmax));
    }
}

// cov [B][N+1][D][D] = T * (scanned sqrtL), row 0 zero
template <typename T>
__global__ void k_cov_out(DenseModel md, DenseWork w, T *cov)
{
    const int D = md.D;
    const int64_t per = (md.N + 1) * (int64_t)D * D;
    const int64_t total = per * md.B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / per);
        const int64_t rem = i - (int64_t)b * per;
        const int64_t n = rem / ((int64_t)D * D);
        const int rr = (int)((rem / D) % D);
        if (n == 0) {
            cov[i] = T(0);
            continue;
        }
        const double *Td = w.traj + (size_t)b * w.traj_stride + (size_t)(md.N + 1) * D;
        const T *Ls = (const T *)w.L + ((size_t)b * md.N + (n - 1)) * D * D;
        cov[i] = (T)(Td[rr] * (double)Ls[rem - n * (int64_t)D * D]);
    }
}

// Objective value (eq. objective-value) of every active instance's resident
// trajectory, in the preconditioned coordinates it is kept in.  The prior is
// d independent copies of one (q+1)-state process, so the weighted norm splits
// over the grid components i:
//   |eta_n - Phi eta_{n-1}|^2_{Q^-1} = sum_i |sqrtQb^-1 (eta_n[i] - Phib eta_{n-1}[i])|^2
// with the (q+1) x (q+1) blocks (FP64).  Halved and summed over n = 1..N into
// obj[2b + slot]: one thread per (step, component) pair, one FP64 atomic per
// workgroup.
__global__ __launch_bounds__(256) void k_objective(DenseModel md, const double *traj, int64_t ts, const int *active,
                                                   double *obj, int slot)
{
    __shared__ double wsum[4];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int S = md.q + 1, D = md.D, d = md.d;
    const double *tb = traj + (size_t)b * ts;
    const int64_t units = md.N * d;
    double v = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = u / d + 1;
        const int i = (int)(u % d);
        const double *a = tb + (n - 1) * D + i * S, *x = a + D;
        double w[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            if (r >= S) break;
            double t = x[r];
#pragma unroll
            for (int c = 0; c < 5; ++c)
                if (c < S) t -= md.phib[r * 5 + c] * a[c];
#pragma unroll
            for (int c = 0; c < 5; ++c)
                if (c < r) t -= md.sqb[r * 5 + c] * w[c];
            w[r] = t / md.sqb[r * 5 + r];
            v += w[r] * w[r];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wsum[k];
        atomicAdd(obj + 2 * b + slot, 0.5 * t);
    }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
template <typename T>
size_t smem_bytes(int D)
{
    return (size_t)smem_elems<T>(2 * D) * sizeof(T);
}

template <typename K>
hipError_t allow_smem(K kern, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

inline unsigned grid_of(int64_t items, int nwg) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, nwg)); }

template <typename T>
hipError_t set_smem(int D)
{
    const size_t sh = smem_bytes<T>(D);
    hipError_t e;
    if ((e = allow_smem(k_elements<T>, sh)) != hipSuccess) return e;
    if ((e = allow_smem(k_fcombine<T>, sh)) != hipSuccess) return e;
    if ((e = allow_smem(k_selements<T>, sh)) != hipSuccess) return e;
    return allow_smem(k_bcombine<T>, sh);
}

template <typename T>
hipError_t smoother_scan(const DenseModel &md, const DenseWork &w, int with_L, hipStream_t st)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    const size_t sh = smem_bytes<T>(md.D);
    const int64_t N = md.N;
    int64_t smax = 0;
    for (int64_t s = 1; 2 * s <= N; s *= 2) {
        const int64_t np = N / (2 * s);
        PARAPN_LAUNCH("dense_bcombine_up", st, k_bcombine<T>, dim3(grid_of(md.B * np, w.nwg)), dim3(NT), sh, st, md,
                      w, s, 1, np, with_L);
        smax = s;
    }
    for (int64_t s = smax; s >= 1; s /= 2) {
        const int64_t np = N >= 3 * s ? (N - 3 * s) / (2 * s) + 1 : 0;
        if (np == 0) continue;
        PARAPN_LAUNCH("dense_bcombine_down", st, k_bcombine<T>, dim3(grid_of(md.B * np, w.nwg)), dim3(NT), sh, st,
                      md, w, s, 0, np, with_L);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t iteration_t(const DenseModel &md, const DenseWork &w, hipStream_t st)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    hipError_t e = set_smem<T>(md.D);
    if (e != hipSuccess) return e;
    const size_t sh = smem_bytes<T>(md.D);
    const int64_t N = md.N, items = md.B * N;
    PARAPN_LAUNCH("dense_elements", st, k_elements<T>, dim3(grid_of(items, w.nwg)), dim3(NT), sh, st, md, w);
    int64_t smax = 0;
    for (int64_t s = 1; 2 * s <= N; s *= 2) {
        const int64_t np = N / (2 * s);
        PARAPN_LAUNCH("dense_fcombine_up", st, k_fcombine<T>, dim3(grid_of(md.B * np, w.nwg)), dim3(NT), sh, st, md,
                      w, s, 1, np);
        smax = s;
    }
    for (int64_t s = smax; s >= 1; s /= 2) {
        const int64_t np = N >= 3 * s ? (N - 3 * s) / (2 * s) + 1 : 0;
        if (np == 0) continue;
        PARAPN_LAUNCH("dense_fcombine_down", st, k_fcombine<T>, dim3(grid_of(md.B * np, w.nwg)), dim3(NT), sh, st,
                      md, w, s, 0, np);
    }
    PARAPN_LAUNCH("dense_selements", st, k_selements<T>, dim3(grid_of(items, w.nwg)), dim3(NT), sh, st, md, w, 0);
    e = smoother_scan<T>(md, w, 0, st);
    if (e != hipSuccess) return e;
    const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N * md.D + NT - 1) / NT, 1024));
    PARAPN_LAUNCH("dense_update", st, k_update<T>, dim3(bx, md.B), dim3(NT), 0, st, md, w);
    return hipGetLastError();
}

template <typename T>
hipError_t covariance_t(const DenseModel &md, const DenseWork &w, void *cov_out, hipStream_t st)
{
    constexpr int NT = nt_of<T>(), NW = NT / 64;
    (void)NW;
    hipError_t e = set_smem<T>(md.D);
    if (e != hipSuccess) return e;
    const size_t sh = smem_bytes<T>(md.D);
    PARAPN_LAUNCH("dense_selements", st, k_selements<T>, dim3(grid_of(md.B * md.N, w.nwg)), dim3(NT), sh, st, md, w,
                  1);
    e = smoother_scan<T>(md, w, 1, st);
    if (e != hipSuccess) return e;
    const int64_t total = md.B * (md.N + 1) * (int64_t)md.D * md.D;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(k_cov_out<T>, dim3(blocks), dim3(256), 0, st, md, w, (T *)cov_out);
    return hipGetLastError();
}

}  // namespace dense

size_t dense_scratch_elems(int D) { return dense::dense_scratch_elems_dev(D); }

// as many as the compute units hold at once (256 CUs: four FP32 or two FP64
// workgroups each, limited by LDS at D = 192)
int dense_workgroups(int fp64) { return fp64 ? 512 : 1024; }

hipError_t dense_iteration(int fp64, const DenseModel &m, const DenseWork &w, hipStream_t s)
{
    return fp64 ? dense::iteration_t<double>(m, w, s) : dense::iteration_t<float>(m, w, s);
}

hipError_t dense_covariance(int fp64, const DenseModel &m, const DenseWork &w, void *cov_out, hipStream_t s)
{
    return fp64 ? dense::covariance_t<double>(m, w, cov_out, s) : dense::covariance_t<float>(m, w, cov_out, s);
}

hipError_t dense_objective(const DenseModel &m, const DenseWork &w, double *obj, int slot, hipStream_t s)
{
    if (m.q + 1 > 5 || slot < 0 || slot > 1) return hipErrorInvalidValue;
    const int64_t units = m.N * m.d;
    const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((units + 255) / 256, 1024));
    PARAPN_LAUNCH("dense_objective", s, dense::k_objective, dim3(bx, m.B), dim3(256), 0, s, m, w.traj, w.traj_stride,
                  w.active, obj, slot);
    return hipGetLastError();
}

}  // namespace parapn
