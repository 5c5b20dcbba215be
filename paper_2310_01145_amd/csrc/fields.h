// Vector-field registry shared by the device kernels (evaluated on dual
// numbers for f and its Jacobian, Sec. 3.2.1) and the host initialisation
// (evaluated on truncated Taylor series for mu0, eq. mu0).  Every field is
// written once, generic over the number type V, which must support +, -, *
// with V and with plain scalars.
#pragma once

#include <hip/hip_runtime.h>

#define PARAPN_HD __host__ __device__ __forceinline__

namespace parapn {

enum FieldId : int {
    F_LOGISTIC = 0,
    F_FHN = 1,
    F_LORENZ = 2,
    F_LV = 3,
    F_MOL = 4,
    F_AFFINE = 5,
    F_RIGID = 6,
    F_VDP = 7,
    // one grid point of the method-of-lines chain solved as its own d = 1
    // problem (approximate Jacobians decouple the chain's state-space model;
    // the linearisation reads the neighbours' trajectories)
    F_MOL_COMPONENT = 8,
};

// ODE dimension a field requires (0 = any d, checked against params elsewhere)
PARAPN_HD int field_fixed_dim(int field)
{
    switch (field) {
    case F_LOGISTIC: return 1;
    case F_FHN: return 2;
    case F_LORENZ: return 3;
    case F_LV: return 2;
    case F_RIGID: return 3;
    case F_VDP: return 2;
    case F_AFFINE: return 0;
    default: return -1;
    }
}

PARAPN_HD int field_n_params(int field, int d)
{
    switch (field) {
    case F_LOGISTIC: return 0;
    case F_FHN: return 3;
    case F_LORENZ: return 3;
    case F_LV: return 4;
    case F_RIGID: return 0;
    case F_VDP: return 1;
    case F_AFFINE: return d * d + d;
    default: return -1;
    }
}

// f(y) for a field of compile-time dimension d; returns false when the field
// does not exist in dimension d.  p holds the field parameters.
template <int d, class V, class P>
PARAPN_HD bool field_eval(int field, const P *p, const V *y, V *f)
{
    if (field == F_AFFINE) {
        for (int i = 0; i < d; ++i) {
            V s = y[0] * p[i * d];
            for (int j = 1; j < d; ++j) s = s + y[j] * p[i * d + j];
            f[i] = s + p[d * d + i];
        }
        return true;
    }
    if constexpr (d == 1) {
        if (field == F_LOGISTIC) {
            f[0] = y[0] * (P(1) - y[0]);
            return true;
        }
    } else if constexpr (d == 2) {
        if (field == F_FHN) {
            // V' = c (V - V^3/3 + R),  R' = -(V - a + b R)/c
            const P a = p[0], b = p[1], c = p[2];
            f[0] = (y[0] - y[0] * y[0] * y[0] * (P(1) / P(3)) + y[1]) * c;
            f[1] = (y[0] - a + y[1] * b) * (P(-1) / c);
            return true;
        }
        if (field == F_LV) {
            const P al = p[0], be = p[1], ga = p[2], de = p[3];
            V xy = y[0] * y[1];
            f[0] = y[0] * al - xy * be;
            f[1] = xy * de - y[1] * ga;
            return true;
        }
        if (field == F_VDP) {
            const P mu = p[0];
            f[0] = y[1];
            f[1] = ((P(1) - y[0] * y[0]) * y[1] - y[0]) * mu;
            return true;
        }
    } else if constexpr (d == 3) {
        if (field == F_LORENZ) {
            const P s = p[0], r = p[1], b = p[2];
            f[0] = (y[1] - y[0]) * s;
            f[1] = y[0] * (r - y[2]) - y[1];
            f[2] = y[0] * y[1] - y[2] * b;
            return true;
        }
        if (field == F_RIGID) {
            f[0] = y[1] * y[2] * P(-2);
            f[1] = y[0] * y[2] * P(1.25);
            f[2] = y[0] * y[1] * P(-0.5);
            return true;
        }
    }
    return false;
}

// Forward-mode dual number with N tangent directions.
template <typename T, int N>
struct Dual {
    T v;
    T g[N];
};

template <typename T, int N>
PARAPN_HD Dual<T, N> operator+(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v + b.v;
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator-(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v - b.v;
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator*(const Dual<T, N> &a, const Dual<T, N> &b)
{
    Dual<T, N> r;
    r.v = a.v * b.v;
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator+(const Dual<T, N> &a, T s)
{
    Dual<T, N> r = a;
    r.v = a.v + s;
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator+(T s, const Dual<T, N> &a)
{
    return a + s;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator-(const Dual<T, N> &a, T s)
{
    Dual<T, N> r = a;
    r.v = a.v - s;
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator-(T s, const Dual<T, N> &a)
{
    Dual<T, N> r;
    r.v = s - a.v;
    for (int i = 0; i < N; ++i) r.g[i] = -a.g[i];
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator*(const Dual<T, N> &a, T s)
{
    Dual<T, N> r;
    r.v = a.v * s;
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * s;
    return r;
}
template <typename T, int N>
PARAPN_HD Dual<T, N> operator*(T s, const Dual<T, N> &a)
{
    return a * s;
}

}  // namespace parapn
