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

// FP32: the hardware square root (1 ulp), without the rescaling a correctly
// rounded sqrt adds for tiny arguments
PARAPN_DEV float psqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
PARAPN_DEV double psqrt(double x) { return __builtin_sqrt(x); }

// tria (Sec. 3.1.2): L lower-triangular with L L^T = M M^T, by Householder
// reflections applied from the right (a QR factorisation of M^T).  M is
// NR x NC with row r in v[] of lane r; lanes >= NR must hold zeros and stay
// zero.  The reflector of step k is formed by lane k with the stable choice
// that makes the diagonal non-negative (so L is the canonical factor), then
// broadcast through `tr` (2*(NC+1) scalars, double-buffered).  On exit lane r
// holds row r of L in v[0..NR-1]; columns >= NR are zero.
// Value of x on lane K of the caller's group, for groups of R = 8 or 16
// lanes: a group is one 16-lane DPP row, or half of one, so the broadcast is
// a row_newbcast (lane K, or lane 8 + K for the upper half) with no LDS round
// trip.  Every lane of the group must be active; with R = 8 the other half of
// the row may be inactive (its value is never selected).
template <int R, int K>
PARAPN_DEV int gbcast_i(int x)
{
    static_assert(R == 8 || R == 16, "DPP broadcast needs groups of 8 or 16 lanes");
    static_assert(K >= 0 && K < R, "lane out of the group");
    // bound_ctrl set: no old value to preserve (the source lane is always an
    // active lane of the caller's group; a read of the inactive other half of
    // a row with R = 8 gives 0 and is not selected)
    if constexpr (R == 16) {
        return __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xF, 0xF, true);
    } else {
        const int lo = __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_update_dpp(0, x, 0x158 + K, 0xF, 0xF, true);
        return (threadIdx.x & 8) ? hi : lo;
    }
}

template <int R, int K>
PARAPN_DEV float gbcast(float x)
{
    return __builtin_bit_cast(float, gbcast_i<R, K>(__builtin_bit_cast(int, x)));
}

template <int R, int K>
PARAPN_DEV double gbcast(double x)
{
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = gbcast_i<R, K>((int)(b & 0xffffffffLL));
    const int hi = gbcast_i<R, K>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// reciprocals: the hardware's 1-ulp estimate in FP32, a division in FP64
PARAPN_DEV float recip(float x) { return __builtin_amdgcn_rcpf(x); }
PARAPN_DEV double recip(double x) { return 1.0 / x; }
PARAPN_DEV float two_over(float x) { return 2.0f * __builtin_amdgcn_rcpf(x); }
PARAPN_DEV double two_over(double x) { return 2.0 / x; }

// One reflection of tria_rows in registers only (groups of 8 or 16 lanes):
// every lane forms the reflector quantities of its own row, the group takes
// lane k's by DPP broadcast; sums use two partial accumulators to halve the
// dependency chains.
// Reflector of row x = v[k..NC-1] (every lane for its own row): returns the
// new diagonal |x|, and u0, the scale 2/(u.u) and the tail a so that the
// reflector is u = (u0, a[k+1..]).  SAFE (FP32 only): x is first divided by
// max|x| (the reflection does not depend on the scale of u), so neither a
// huge nor a tiny remaining tail over- or underflows its squares -- an
// underflowed norm would leave a zero on the diagonal of the factor.
template <typename T, int NC, bool SAFE>
PARAPN_DEV T reflector(const T (&v)[NC], int k, T &u0, T &sc, T (&a)[NC])
{
    T m = T(1);
    if constexpr (SAFE) {
        static_assert(sizeof(T) == 4, "scaled reflectors are for FP32");
        T m0 = __builtin_fabsf(v[k]), m1 = T(0);
#pragma unroll
        for (int c = k + 1; c < NC; ++c) {
            if ((c - k) & 1)
                m1 = __builtin_fmaxf(m1, __builtin_fabsf(v[c]));
            else
                m0 = __builtin_fmaxf(m0, __builtin_fabsf(v[c]));
        }
        m = __builtin_fmaxf(m0, m1);
        const T scale = m > T(0) ? recip(m) : T(0);
#pragma unroll
        for (int c = k; c < NC; ++c) a[c] = v[c] * scale;
    } else {
#pragma unroll
        for (int c = k; c < NC; ++c) a[c] = v[c];
    }
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int c = k + 1; c < NC; ++c) {
        if ((c - k) & 1)
            s0 += a[c] * a[c];
        else
            s1 += a[c] * a[c];
    }
    const T sig = s0 + s1;
    const T x0 = a[k];
    const T nrm = psqrt(x0 * x0 + sig);
    u0 = x0 <= T(0) ? x0 - nrm : -sig * recip(x0 + nrm);
    const T uu = u0 * u0 + sig;
    sc = uu > T(0) ? two_over(uu) : T(0);
    return nrm * m;
}

template <typename T, int NR, int NC, int R, bool SAFE, int k>
PARAPN_DEV void tria_dpp_step(T (&v)[NC], int lane)
{
    constexpr int K = NR < NC ? NR : NC;
    if constexpr (k < K) {
        T u0, sc, a[NC];
        const T nrm = reflector<T, NC, SAFE>(v, k, u0, sc, a);
        const T sk = gbcast<R, k>(sc);
        const T uk = gbcast<R, k>(u0);
        T w[NC];
#pragma unroll
        for (int c = k + 1; c < NC; ++c) w[c] = gbcast<R, k>(a[c]);
        T d0 = v[k] * uk, d1 = T(0);
#pragma unroll
        for (int c = k + 1; c < NC; ++c) {
            if ((c - k) & 1)
                d1 += v[c] * w[c];
            else
                d0 += v[c] * w[c];
        }
        const T dot = (d0 + d1) * sk;
        // lane k applies its own reflector too: that maps its row to
        // (|x|, 0, ..., 0) up to rounding; the strict upper triangle is
        // cleared once at the end
        (void)nrm;
        v[k] = v[k] - dot * uk;
#pragma unroll
        for (int c = k + 1; c < NC; ++c) v[c] = v[c] - dot * w[c];
        tria_dpp_step<T, NR, NC, R, SAFE, k + 1>(v, lane);
    }
}

// exact zeros above the diagonal (the register version leaves rounding
// residues there)
template <typename T, int NC>
PARAPN_DEV void canonical_upper(T (&v)[NC], int lane)
{
#pragma unroll
    for (int c = 1; c < NC; ++c) v[c] = c > lane ? T(0) : v[c];
}

// Two independent trias (NR rows each) in lock step: one reflection of each
// per step, so the dependency chains of the two overlap.
template <typename T, int NR, int NC1, int NC2, int R, bool SAFE, int k>
PARAPN_DEV void tria2_dpp_step(T (&v1)[NC1], T (&v2)[NC2], int lane)
{
    constexpr int K1 = NR < NC1 ? NR : NC1, K2 = NR < NC2 ? NR : NC2;
    constexpr int K = K1 > K2 ? K1 : K2;
    if constexpr (k < K) {
        (void)lane;
        if constexpr (k < K1) {
            T u0, sc, a[NC1];
            const T nrm = reflector<T, NC1, SAFE>(v1, k, u0, sc, a);
            const T sk = gbcast<R, k>(sc);
            const T uk = gbcast<R, k>(u0);
            T w[NC1];
#pragma unroll
            for (int c = k + 1; c < NC1; ++c) w[c] = gbcast<R, k>(a[c]);
            T d0 = v1[k] * uk, d1 = T(0);
#pragma unroll
            for (int c = k + 1; c < NC1; ++c) {
                if ((c - k) & 1)
                    d1 += v1[c] * w[c];
                else
                    d0 += v1[c] * w[c];
            }
            const T dot = (d0 + d1) * sk;
            (void)nrm;
            v1[k] = v1[k] - dot * uk;
#pragma unroll
            for (int c = k + 1; c < NC1; ++c) v1[c] = v1[c] - dot * w[c];
        }
        if constexpr (k < K2) {
            T u0, sc, a[NC2];
            const T nrm = reflector<T, NC2, SAFE>(v2, k, u0, sc, a);
            const T sk = gbcast<R, k>(sc);
            const T uk = gbcast<R, k>(u0);
            T w[NC2];
#pragma unroll
            for (int c = k + 1; c < NC2; ++c) w[c] = gbcast<R, k>(a[c]);
            T d0 = v2[k] * uk, d1 = T(0);
#pragma unroll
            for (int c = k + 1; c < NC2; ++c) {
                if ((c - k) & 1)
                    d1 += v2[c] * w[c];
                else
                    d0 += v2[c] * w[c];
            }
            const T dot = (d0 + d1) * sk;
            (void)nrm;
            v2[k] = v2[k] - dot * uk;
#pragma unroll
            for (int c = k + 1; c < NC2; ++c) v2[c] = v2[c] - dot * w[c];
        }
        tria2_dpp_step<T, NR, NC1, NC2, R, SAFE, k + 1>(v1, v2, lane);
    }
}

// tria for groups of R lanes: registers and DPP for R = 8 or 16, else the
// LDS version below
template <typename T, int NR, int NC, int R, bool SAFE = false>
PARAPN_DEV void tria_rows_g(T (&v)[NC], int lane, T *tr);

template <typename T, int NR, int NC, bool SAFE = false>
PARAPN_DEV void tria_rows(T (&v)[NC], int lane, T *tr)
{
    constexpr int K = NR < NC ? NR : NC;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T *buf = tr + (k & 1) * (NC + 1);
        T nrm = T(0);
        if (lane == k) {
            T u0, sc, a[NC];
            nrm = reflector<T, NC, SAFE>(v, k, u0, sc, a);
            buf[0] = sc;
            buf[1 + k] = u0;
#pragma unroll
            for (int c = k + 1; c < NC; ++c) buf[1 + c] = a[c];
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

// In FP32 every row is first scaled by a power of two (exactly) so that its
// largest entry is below 1, and the result scaled back: tria(S M) = S tria(M)
// for a positive diagonal S, and the reflections preserve each row's norm,
// so squares of large entries stay in range.  SAFE additionally scales each
// reflector (small remaining tails).  FP64 runs on the rows as they are.
template <typename T, int NR, int NC, int R, bool SAFE>
PARAPN_DEV void tria_rows_g(T (&v)[NC], int lane, T *tr)
{
    int e = 0;
    if constexpr (sizeof(T) == 4 && !SAFE) {
        T m = T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) m = __builtin_fmaxf(m, __builtin_fabsf(v[c]));
        e = m > T(0) ? __builtin_amdgcn_frexp_expf(m) : 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = __builtin_amdgcn_ldexpf(v[c], -e);
    }
    if constexpr (R == 8 || R == 16) {
        tria_dpp_step<T, NR, NC, R, SAFE, 0>(v, lane);
        canonical_upper<T, NC>(v, lane);
        wave_sync();  // callers' LDS traffic stays ordered around the call, as with the LDS version
    } else {
        tria_rows<T, NR, NC, SAFE>(v, lane, tr);
    }
    if constexpr (sizeof(T) == 4 && !SAFE) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = __builtin_amdgcn_ldexpf(v[c], e);
    }
}

// tria of two independent NR-row matrices (same layout rules as tria_rows_g)
template <typename T, int NR, int NC1, int NC2, int R, bool SAFE = false>
PARAPN_DEV void tria2_rows_g(T (&v1)[NC1], T (&v2)[NC2], int lane, T *tr)
{
    if constexpr (R == 8 || R == 16) {
        int e1 = 0, e2 = 0;
        if constexpr (sizeof(T) == 4 && !SAFE) {
            T m1 = T(0), m2 = T(0);
#pragma unroll
            for (int c = 0; c < NC1; ++c) m1 = __builtin_fmaxf(m1, __builtin_fabsf(v1[c]));
#pragma unroll
            for (int c = 0; c < NC2; ++c) m2 = __builtin_fmaxf(m2, __builtin_fabsf(v2[c]));
            e1 = m1 > T(0) ? __builtin_amdgcn_frexp_expf(m1) : 0;
            e2 = m2 > T(0) ? __builtin_amdgcn_frexp_expf(m2) : 0;
#pragma unroll
            for (int c = 0; c < NC1; ++c) v1[c] = __builtin_amdgcn_ldexpf(v1[c], -e1);
#pragma unroll
            for (int c = 0; c < NC2; ++c) v2[c] = __builtin_amdgcn_ldexpf(v2[c], -e2);
        }
        tria2_dpp_step<T, NR, NC1, NC2, R, SAFE, 0>(v1, v2, lane);
        canonical_upper<T, NC1>(v1, lane);
        canonical_upper<T, NC2>(v2, lane);
        wave_sync();
        if constexpr (sizeof(T) == 4 && !SAFE) {
#pragma unroll
            for (int c = 0; c < NC1; ++c) v1[c] = __builtin_amdgcn_ldexpf(v1[c], e1);
#pragma unroll
            for (int c = 0; c < NC2; ++c) v2[c] = __builtin_amdgcn_ldexpf(v2[c], e2);
        }
    } else {
        tria_rows_g<T, NR, NC1, R, SAFE>(v1, lane, tr);
        tria_rows_g<T, NR, NC2, R, SAFE>(v2, lane, tr);
    }
}

// x (1 x n) such that x L = b, L lower-triangular n x n at L[i*ld + j]
template <typename T, int n>
PARAPN_DEV void solve_xL(T (&x)[n], const T (&b)[n], const T *L, int ld)
{
    T inv[n];
#pragma unroll
    for (int j = 0; j < n; ++j) inv[j] = recip(L[j * ld + j]);
#pragma unroll
    for (int j = n - 1; j >= 0; --j) {
        T s = b[j];
#pragma unroll
        for (int k = j + 1; k < n; ++k) s -= x[k] * L[k * ld + j];
        x[j] = s * inv[j];
    }
}

// x (1 x n) such that x L^T = b, i.e. L x^T = b^T (forward substitution)
template <typename T, int n>
PARAPN_DEV void solve_xLt(T (&x)[n], const T (&b)[n], const T *L, int ld)
{
    T inv[n];
#pragma unroll
    for (int j = 0; j < n; ++j) inv[j] = recip(L[j * ld + j]);
#pragma unroll
    for (int j = 0; j < n; ++j) {
        T s = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= x[k] * L[j * ld + k];
        x[j] = s * inv[j];
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
