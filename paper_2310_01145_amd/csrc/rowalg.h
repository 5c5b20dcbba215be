// Small dense linear algebra for one square-root element per group of lanes.
//
// Layout: a group of R lanes (R a power of two, R <= 64, so a group never
// straddles a wavefront) works on one element.  Lane r holds row r of every
// matrix in registers; rows another lane needs are broadcast through the
// group's LDS scratch.  Because a group lives inside one wavefront, a
// wavefront-scope fence plus a scheduling barrier orders an LDS write before
// the reads of the other lanes; no workgroup barrier is needed.
#pragma once

#include <hip/hip_runtime.h>

#define PARAPN_DEV __device__ __forceinline__

namespace parapn {

constexpr int pow2ceil(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

PARAPN_DEV void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

PARAPN_DEV float psqrt(float x) { return __builtin_sqrtf(x); }
PARAPN_DEV double psqrt(double x) { return __builtin_sqrt(x); }

// tria (Sec. 3.1.2): L lower-triangular with L L^T = M M^T, by Householder
// reflections applied from the right (a QR factorisation of M^T).  M is
// NR x NC with row r in v[] of lane r; lanes >= NR must hold zeros and stay
// zero.  The reflector of step k is formed by lane k with the stable choice
// that makes the diagonal non-negative (so L is the canonical factor), then
// broadcast through `tr` (2*(NC+1) scalars, double-buffered).  On exit lane r
// holds row r of L in v[0..NR-1]; columns >= NR are zero.
template <typename T, int NR, int NC>
PARAPN_DEV void tria_rows(T (&v)[NC], int lane, T *tr)
{
    constexpr int K = NR < NC ? NR : NC;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T *buf = tr + (k & 1) * (NC + 1);
        T nrm = T(0);
        if (lane == k) {
            T sig = T(0);
#pragma unroll
            for (int c = k + 1; c < NC; ++c) sig += v[c] * v[c];
            const T x0 = v[k];
            nrm = psqrt(x0 * x0 + sig);
            const T u0 = x0 <= T(0) ? x0 - nrm : -sig / (x0 + nrm);
            const T uu = u0 * u0 + sig;
            buf[0] = uu > T(0) ? T(2) / uu : T(0);
            buf[1 + k] = u0;
#pragma unroll
            for (int c = k + 1; c < NC; ++c) buf[1 + c] = v[c];
        }
        wave_sync();
        const T s = buf[0];
        T dot = T(0);
#pragma unroll
        for (int c = k; c < NC; ++c) dot += v[c] * buf[1 + c];
        dot *= s;
#pragma unroll
        for (int c = k; c < NC; ++c) v[c] -= dot * buf[1 + c];
        if (lane == k) {
            v[k] = nrm;
#pragma unroll
            for (int c = k + 1; c < NC; ++c) v[c] = T(0);
        }
    }
    wave_sync();
}

// x (1 x n) such that x L = b, L lower-triangular n x n at L[i*ld + j]
template <typename T, int n>
PARAPN_DEV void solve_xL(T (&x)[n], const T (&b)[n], const T *L, int ld)
{
#pragma unroll
    for (int j = n - 1; j >= 0; --j) {
        T s = b[j];
#pragma unroll
        for (int k = j + 1; k < n; ++k) s -= x[k] * L[k * ld + j];
        x[j] = s / L[j * ld + j];
    }
}

// x (1 x n) such that x L^T = b, i.e. L x^T = b^T (forward substitution)
template <typename T, int n>
PARAPN_DEV void solve_xLt(T (&x)[n], const T (&b)[n], const T *L, int ld)
{
#pragma unroll
    for (int j = 0; j < n; ++j) {
        T s = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= x[k] * L[j * ld + k];
        x[j] = s / L[j * ld + j];
    }
}

// write row `lane` (if lane < NR) of an NR x NC matrix to buf with stride ld
template <typename T, int NR, int NC>
PARAPN_DEV void put_rows(T *buf, int ld, int lane, const T (&v)[NC])
{
    if (lane < NR) {
#pragma unroll
        for (int c = 0; c < NC; ++c) buf[lane * ld + c] = v[c];
    }
}

// out[c] = sum_k a[k] * B[k*ld + c]   (row vector times matrix in LDS)
template <typename T, int K, int NC>
PARAPN_DEV void row_times(T (&out)[NC], const T (&a)[K], const T *B, int ld)
{
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T ak = a[k];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += ak * B[k * ld + c];
    }
}

// out[c] = sum_k A[k*ld + r] * B[k*ldb + c]   (row r of A^T B, both in LDS)
template <typename T, int K, int NC>
PARAPN_DEV void rowT_times(T (&out)[NC], int r, const T *A, int lda, const T *B, int ldb)
{
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T ak = A[k * lda + r];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += ak * B[k * ldb + c];
    }
}

}  // namespace parapn
