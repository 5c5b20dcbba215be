// ParaRTS (Alg. 1) and the per-iteration work of ParaIEKS (Alg. 2) on gfx950.
//
// One group of R lanes (R = next power of two >= 2D) owns one element of the
// scan; lane r holds row r of every D x D block (rowalg.h).  The associative
// scans are hierarchical reduce-then-scan:
//   step level   each group folds b1 consecutive elements, built on the fly,
//                into one aggregate (the paper's operators);
//   upper levels groups fold bu aggregates at a time until at most btop
//                remain, which one group scans sequentially from the initial
//                state; prefix states then flow back down;
//   step level   each group walks its b1 steps again from its exclusive prefix
//                state and writes the per-step marginals.
// Every exclusive prefix of the filtering scan is a Gaussian state (A = 0,
// eta = 0, J = 0: it does not depend on an earlier state), so prefix states
// are stored as (mean, factor) only, and applying a state to the next element
// is the filtering operator with those zeros substituted -- which is exactly a
// Kalman predict + update step.  Suffixes of the smoothing scan always contain
// the last element (E_N = 0), so suffix states are (mean, factor) as well.
//
// Two representations keep FP32 from losing the dynamics at small steps.
// In preconditioned coordinates a step's transition acts on the trajectory
// as the identity plus O(h); a matrix entry near 1 rounded to FP32 carries
// only eps/h of relative precision in that O(h) part, and composing the
// rounded steps over N steps drifts by ~N eps.  So every filtering element
// and aggregate stores A - I in place of A, and the operator is evaluated in
// that form (below), which rounds each term relative to its own size.  On
// the smoothing side the element offset g = m^f - E m^- is a difference of two
// nearly equal means; instead the reverse scan runs on the smoothing
// correction c_n = m^s_n - m^f_n:
//   c_n = E_n c_{n+1} + E_n k_{n+1},   c_N = 0,
// where k_{n+1} = m^f_{n+1} - m^-_{n+1} is the Kalman update of step n+1 --
// the same recursion (and the same associative operator) with offset
// E_n k_{n+1}; the element records carry m^f_n beside it and the smoothed
// mean is m^f_n + c_n.  Both forms are exact rewritings of the paper's
// element and operator equations.
#include <hip/hip_runtime.h>

#include "fields.h"
#include "parapn_internal.h"
#include "rowalg.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace parapn {

constexpr int pow2floor(int x)
{
    int p = 1;
    while (2 * p <= x) p <<= 1;
    return p;
}

// Configuration of one (precision, d, q).  Filter-side kernels give each
// element 2D rows (R = next power of two >= 2D lanes); the smoother-side
// kernels only need D rows and use RS lanes.
template <typename T_, int d_, int q_, int RS_ = 0, bool LM_ = false>
struct Cfg {
    using T = T_;
    static constexpr int d = d_, q = q_, S = q_ + 1, D = d_ * (q_ + 1);
    // Levenberg-Marquardt damping: d more observation rows (E0 of the
    // increment, observed as 0) with noise, carried in NZ extra columns of the
    // update trias
    static constexpr bool LM = LM_;
    static constexpr int DO = LM_ ? 2 * d_ : d_;
    static constexpr int NZ = LM_ ? d_ : 0;
    static constexpr int D2 = 2 * D;
    static constexpr int DP = D * (D + 1) / 2;
    static constexpr int B1 = 8;  // steps per group in the smoother's step-level kernels (prefetched)
    static constexpr int R = RS_ ? RS_ : pow2ceil(D2);  // lanes per group
    static constexpr int LDM = D + 1;       // LDS row stride of D-wide blocks
    static constexpr int LDB = D2 + 1;      // LDS row stride of 2D-wide blocks
    // per-group LDS layout (in T units).  The smoother side (RS_ != 0) only
    // uses TR, M0, M1 and V0; its other regions have size zero.
    static constexpr int F1 = RS_ ? 0 : 1;
    static constexpr int TR = 0;
    static constexpr int BIG = TR + 2 * (D2 + 1);
    static constexpr int M0 = BIG + F1 * D2 * LDB;
    static constexpr int M1 = M0 + D * LDM;
    static constexpr int M2 = M1 + D * LDM;
    static constexpr int M3 = M2 + F1 * D * LDM;
    static constexpr int M4 = M3 + F1 * D * LDM;
    static constexpr int M5 = M4 + F1 * D * LDM;
    static constexpr int V0 = M5 + F1 * D * LDM;
    static constexpr int V1 = V0 + LDM;
    static constexpr int V2 = V1 + F1 * LDM;
    static constexpr int V3 = V2 + F1 * LDM;
    static constexpr int V4 = V3 + F1 * LDM;
    static constexpr int V5 = V4 + F1 * LDM;
    static constexpr int HO = V5 + F1 * LDM;         // H   (DO x LDM)
    static constexpr int HPO = HO + F1 * DO * LDM;   // H Phi (DO x LDM)
    static constexpr int DVO = HPO + F1 * DO * LDM;  // residual r (DO), then the damping std
    static constexpr int UO = DVO + F1 * (DO + 1);   // prior offset u (D)
    static constexpr int SH = UO + F1 * LDM;
    // block: groups per block chosen so that a block's LDS stays <= 64 KiB
    static constexpr int FE_ = 3 * D * D + 2 * D;
    // filter side: at most 16 groups per block (the tree width the workspace sizing covers)
    static constexpr int GPB_MAX = RS_ ? 256 / R : (256 / R < 16 ? 256 / R : 16);
    // room for the group scratch plus (filter side) one exchanged element per
    // group in the tree kernels; a block stays within 64 KiB of LDS
    static constexpr int GPB_FIT = (65536 / (int)sizeof(T) - 2 * D * LDM) / (SH + (RS_ ? 0 : FE_));
    static constexpr int GPB_P = pow2floor(GPB_FIT < GPB_MAX ? GPB_FIT : GPB_MAX);
    static constexpr int GPB = GPB_P >= 2 ? GPB_P : 2;
    static constexpr int NT = GPB * R;
    // tree width of the upper scan levels (one leaf per group of a block)
    static constexpr int W = GPB;
    // record sizes (T units)
    static constexpr int FE = 3 * D * D + 2 * D;  // filter element / aggregate: A, b, sqrtC, eta, sqrtJ
    static constexpr int FS = D + D * D;          // filter state: mean, factor
    static constexpr int SE = D * D + 2 * D;      // smoothing element (E, g) and the filtering mean
    static constexpr int SA = 2 * D * D + D;      // smoothing aggregate: E, g, sqrtL
    static constexpr int SS = D + D * D;          // smoother state: mean, factor
    // FP32 with the IWP(4) prior: every Householder reflector is formed from
    // its row scaled to unit max (the preconditioned quantities span a range
    // whose squares leave FP32); other configurations scale whole rows once
    static constexpr bool SAFE = sizeof(T_) == 4 && (q_ >= 4 || LM_);
    // stored records carry one trailing flag (request boundary)
    static constexpr int FEF = FE + 1, SEF = SE + 1, SAF = SA + 1;
    static_assert(R <= 64, "a group must fit in one wavefront");
};

// ---------------------------------------------------------------------------
// record <-> row registers
// ---------------------------------------------------------------------------
template <class C>
struct FRow {
    using T = typename C::T;
    T A[C::D];
    T b;
    T sC[C::D];
    T eta;
    T sJ[C::D];
    T flag;  // nonzero: contains the first step of a request (nothing before it matters)
};

template <class C>
struct SRow {  // a (mean, factor) row: filter/smoother state
    using T = typename C::T;
    T m;
    T P[C::D];
};

template <class C>
struct ERow {  // smoothing element / aggregate row
    using T = typename C::T;
    T E[C::D];
    T g;
    T L[C::D];
    T flag;  // nonzero: contains the last step of a request (nothing after it matters)
};

template <class C>
PARAPN_DEV void zero(FRow<C> &e)
{
#pragma unroll
    for (int c = 0; c < C::D; ++c) e.A[c] = e.sC[c] = e.sJ[c] = 0;
    e.b = e.eta = e.flag = 0;
}

template <class C, bool FLAG = true>
PARAPN_DEV FRow<C> load_frow(const typename C::T *rec, int r)
{
    constexpr int D = C::D;
    FRow<C> e;
    zero(e);
    if (FLAG) e.flag = rec[C::FE];
    if (r < D) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            e.A[c] = rec[r * D + c];
            e.sC[c] = rec[D * D + D + r * D + c];
            e.sJ[c] = rec[2 * D * D + 2 * D + r * D + c];
        }
        e.b = rec[D * D + r];
        e.eta = rec[2 * D * D + D + r];
    }
    return e;
}

template <class C, bool FLAG = true>
PARAPN_DEV void store_frow(typename C::T *rec, int r, const FRow<C> &e)
{
    constexpr int D = C::D;
    if (FLAG && r == 0) rec[C::FE] = e.flag;
    if (r < D) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            rec[r * D + c] = e.A[c];
            rec[D * D + D + r * D + c] = e.sC[c];
            rec[2 * D * D + 2 * D + r * D + c] = e.sJ[c];
        }
        rec[D * D + r] = e.b;
        rec[2 * D * D + D + r] = e.eta;
    }
}

template <class C>
PARAPN_DEV SRow<C> load_state(const typename C::T *rec, int r)
{
    constexpr int D = C::D;
    SRow<C> s;
    s.m = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) s.P[c] = 0;
    if (r < D) {
        s.m = rec[r];
#pragma unroll
        for (int c = 0; c < D; ++c) s.P[c] = rec[D + r * D + c];
    }
    return s;
}

template <class C>
PARAPN_DEV void store_state(typename C::T *rec, int r, const SRow<C> &s)
{
    constexpr int D = C::D;
    if (r < D) {
        rec[r] = s.m;
#pragma unroll
        for (int c = 0; c < D; ++c) rec[D + r * D + c] = s.P[c];
    }
}

// packed lower-triangular rows: row r occupies [r(r+1)/2, r(r+1)/2 + r]
template <class C>
PARAPN_DEV void load_packed(typename C::T (&v)[C::D], const typename C::T *p, int r)
{
#pragma unroll
    for (int c = 0; c < C::D; ++c) v[c] = 0;
    if (r < C::D) {
        const typename C::T *row = p + r * (r + 1) / 2;
#pragma unroll
        for (int c = 0; c < C::D; ++c)
            if (c <= r) v[c] = row[c];
    }
}

template <class C>
PARAPN_DEV void store_packed(typename C::T *p, int r, const typename C::T (&v)[C::D])
{
    if (r < C::D) {
        typename C::T *row = p + r * (r + 1) / 2;
#pragma unroll
        for (int c = 0; c < C::D; ++c)
            if (c <= r) row[c] = v[c];
    }
}

// ---------------------------------------------------------------------------
// the observation of one step, placed in the group's LDS:
//   H (d x D), H Phi (d x D), d (d)
// ---------------------------------------------------------------------------
// The scans solve for the Gauss-Newton increment delta = Ybar - eta of the
// preconditioned state relative to the current trajectory eta (same
// posterior, shifted coordinates).  Per step n the linearised model is
//   delta_n = Phi delta_{n-1} + u_n + w_n,    u_n = Phi eta_{n-1} - eta_n,
//   Hbar_n delta_n = r_n,   Hbar_n = E1 - (h/q) F_y E0,
//   r_n = (f(y_n) - y'_n) / T1,   y_n = T0 E0 eta_n,  y'_n = T1 E1 eta_n,
// i.e. the EK1 model of Sec. 3.2.1 written around eta (the F_y y terms of d_n
// cancel exactly against Hbar eta).  u_n and r_n are formed in FP64 from the
// FP64 trajectory and then rounded to the path's precision.  In memory mode
// (ParaRTS on a given linear model) u = 0 and r = d.
// The request fields the step kernels use, held in registers: the kernels
// store through pointers the compiler cannot separate from the request table,
// and fields read through it would be reloaded after every such store.
// Device memory reached through pointers read from tables is "flat" to the
// compiler, and a flat access also counts against the LDS wait counter: every
// LDS wait after a flat store then waits for that store to reach memory.
// Pointers known to address global memory are cast to this type.
typedef __attribute__((address_space(1))) double gdouble;

struct ReqView {
    const double *p;
    gdouble *traj;
    unsigned long long *dbits;
    double T0, T1, invT1, hq, lm_s;
    int64_t N, row;
    int field, lin;
};

PARAPN_DEV ReqView view_of(const ReqDev &q)
{
    ReqView v;
    v.p = q.p;
    v.traj = (gdouble *)q.traj;
    v.dbits = q.dbits;
    v.T0 = q.T0;
    v.T1 = q.T1;
    v.invT1 = q.invT1;
    v.hq = q.hq;
    v.lm_s = q.lm_s;
    v.N = q.N;
    v.row = q.row;
    v.field = q.field;
    v.lin = q.lin;
    return v;
}

template <class C>
PARAPN_DEV void obs_setup(const Pack &pk, const ReqView &o, int64_t n, int lane, typename C::T *sh,
                          const typename C::T *cphi)
{
    using T = typename C::T;
    constexpr int d = C::d, D = C::D, S = C::S, LDM = C::LDM;
    T hrow[D];
#pragma unroll
    for (int c = 0; c < D; ++c) hrow[c] = 0;
    T rval = 0, uval = 0;
    if (pk.mode == 0) {
        const gdouble *tn = o.traj + n * D;
        const gdouble *tp = tn - D;
        bool component = false;
        if constexpr (d == 1) {
            if (o.field == F_MOL_COMPONENT) {
                // f_i = nu (y_{i-1} - 2 y_i + y_{i+1}) / dx^2 + y_i (1 - y_i), its
                // diagonal Jacobian entry -2 nu / dx^2 + 1 - 2 y_i
                component = true;
                const double k = o.p[0];
                const double y = o.T0 * tn[0], ym = o.T0 * tn[(int64_t)o.p[1]], yp = o.T0 * tn[(int64_t)o.p[2]];
                const double fv = k * (ym - 2.0 * y + yp) + y * (1.0 - y);
                const double jv = o.lin == 2 ? 1.0 - 2.0 * k - 2.0 * y : 0.0;
                if (lane == 0) {
                    hrow[0] -= (T)(o.hq * jv);
                    hrow[1] += T(1);
                    rval = (T)((fv - o.T1 * tn[1]) * o.invT1);
                }
            }
        }
        if (!component) {
            Dual<double, d> yd[d], fd[d];
#pragma unroll
            for (int i = 0; i < d; ++i) {
                yd[i].v = o.T0 * tn[i * S];
#pragma unroll
                for (int j = 0; j < d; ++j) yd[i].g[j] = (i == j) ? 1.0 : 0.0;
            }
            field_eval<d>(o.field, o.p, yd, fd);
#pragma unroll
            for (int i = 0; i < d; ++i)
                if (lane == i) {
#pragma unroll
                    for (int j = 0; j < d; ++j) {
                        // EK0 drops F_y, DiagonalEK1 its off-diagonal entries
                        const bool keep = o.lin == 0 || (o.lin == 2 && j == i);
                        hrow[j * S] -= keep ? (T)(o.hq * fd[i].g[j]) : T(0);
                    }
                    hrow[i * S + 1] += T(1);
                    rval = (T)((fd[i].v - o.T1 * tn[i * S + 1]) * o.invT1);
                }
        }
        if constexpr (C::LM) {
            // damping rows: E0 of the increment is observed as 0
#pragma unroll
            for (int i = 0; i < d; ++i)
                if (lane == d + i) hrow[i * S] = T(1);
        }
        if (lane < D) {
            double u = -tn[lane];
#pragma unroll
            for (int k = 0; k < D; ++k) u += (double)cphi[lane * LDM + k] * tp[k];
            uval = (T)u;
        }
    } else if (lane < d) {
        const T *hr = (const T *)pk.H + ((n - 1) * d + lane) * D;
#pragma unroll
        for (int c = 0; c < D; ++c) hrow[c] = hr[c];
        rval = ((const T *)pk.dv)[(n - 1) * d + lane];
    }
    if (lane < C::DO) {
        T hp[D];
        row_times<T, D, D>(hp, hrow, cphi, LDM);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            sh[C::HO + lane * LDM + c] = hrow[c];
            sh[C::HPO + lane * LDM + c] = hp[c];
        }
        sh[C::DVO + lane] = rval;
    }
    if (C::LM && lane == 0) sh[C::DVO + C::DO] = (T)o.lm_s;
    if (lane < D) sh[C::UO + lane] = uval;
    wave_sync();
}

// ---------------------------------------------------------------------------
// square-root filtering element of a step n >= 1 with m_{n-1} = 0,
// P_{n-1} = 0 (eq. sqrt-filtering-elements, sqrt R = 0), so the predicted
// mean is the prior offset m- = u_n and the predicted factor is sqrtQ:
//   Psi = tria([[H sqrtQ], [sqrtQ]]),  K = Psi21 Psi11^{-1},
//   A = (I - K H) Phi,  b = m- - K (H m- - r),  sqrtC = Psi22,
//   sqrtJ = Phi^T H^T Psi11^{-T} (D x d, zero padded),
//   eta = sqrtJ Psi11^{-1} (r - H m-).
// The returned row holds A - I (the representation the scans use).
// The initial distribution is not folded in here: it enters the scan as the
// exclusive prefix state of step 1.
// ---------------------------------------------------------------------------
template <class C>
PARAPN_DEV FRow<C> filter_element(int lane, typename C::T *sh, const typename C::T *cphi, const typename C::T *csq)
{
    using T = typename C::T;
    constexpr int d = C::d, D = C::D, DO = C::DO, NZ = C::NZ, LDM = C::LDM, LDB = C::LDB;
    // tria([[H sqrtQ, sqrtR], [sqrtQ, 0]]); sqrtR = 0 except the damping rows
    T w[D + NZ];
#pragma unroll
    for (int c = 0; c < D + NZ; ++c) w[c] = 0;
    if (lane < DO) {
        T hrow[D], t[D];
#pragma unroll
        for (int c = 0; c < D; ++c) hrow[c] = sh[C::HO + lane * LDM + c];
        row_times<T, D, D>(t, hrow, csq, LDM);
#pragma unroll
        for (int c = 0; c < D; ++c) w[c] = t[c];
        if constexpr (NZ > 0) {
            const T sn = sh[C::DVO + DO];
#pragma unroll
            for (int i = 0; i < NZ; ++i)
                if (lane == d + i) w[D + i] = sn;
        }
    } else if (lane < DO + D) {
#pragma unroll
        for (int c = 0; c < D; ++c) w[c] = csq[(lane - DO) * LDM + c];
    }
    tria_rows_g<T, DO + D, D + NZ, C::R, C::SAFE>(w, lane, sh + C::TR);
    T *Psi = sh + C::BIG;
    put_rows<T, DO + D, D + NZ>(Psi, LDB, lane, w);
    wave_sync();
    FRow<C> e;
    zero(e);
    if (lane < D) {
        const T *HP = sh + C::HPO;
        const T *dv = sh + C::DVO;
        const T *um = sh + C::UO;
        T p21[DO], K[DO], hpc[DO], x[DO], dvv[DO], u[DO];
#pragma unroll
        for (int i = 0; i < DO; ++i) {
            p21[i] = Psi[(DO + lane) * LDB + i];
            hpc[i] = HP[i * LDM + lane];
            T hu = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) hu += sh[C::HO + i * LDM + k] * um[k];
            dvv[i] = dv[i] - hu;  // r - H m-
        }
        solve_xL<T, DO>(K, p21, Psi, LDB);
        T b = um[lane];
#pragma unroll
        for (int i = 0; i < DO; ++i) b += K[i] * dvv[i];
        e.b = b;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            // A - I = (Phi - I) - K H Phi; Phi - I has exact integer entries
            T a = cphi[lane * LDM + c] - (c == lane ? T(1) : T(0));
#pragma unroll
            for (int i = 0; i < DO; ++i) a -= K[i] * HP[i * LDM + c];
            e.A[c] = a;
            e.sC[c] = (c < D - d) ? Psi[(DO + lane) * LDB + DO + c] : T(0);
        }
        solve_xLt<T, DO>(x, hpc, Psi, LDB);
        solve_xLt<T, DO>(u, dvv, Psi, LDB);
        T et = 0;
#pragma unroll
        for (int i = 0; i < DO; ++i) {
            e.sJ[i] = x[i];
            et += x[i] * u[i];
        }
        e.eta = et;
    }
    wave_sync();
    return e;
}

// ---------------------------------------------------------------------------
// filtering operator a_i (x)_f a_j (eq. sqrt-associative-filtering), with
//   Xi = tria([[sqrtC_i^T sqrtJ_j, I], [sqrtJ_j, 0]]),
//   G = sqrtC_i Xi11^{-T},  F = I - G Xi21^T:
//   A_ij = A_j F A_i,  b_ij = A_j F (b_i + sqrtC_i sqrtC_i^T eta_j) + b_j,
//   sqrtC_ij = tria([A_j G, sqrtC_j]),
//   eta_ij = A_i^T F^T (eta_j - sqrtJ_j sqrtJ_j^T b_i) + eta_i,
//   sqrtJ_ij = tria([A_i^T Xi22, sqrtJ_i]).
// (F^T = I - Xi21 Xi11^{-1} sqrtC_i^T, the factor of the eta formula.)
// Evaluated on the stored differences Ai~ = A_i - I, Aj~ = A_j - I and
// F~ = F - I = -G Xi21^T: with P = A_j F - I = Aj~ + F~ + Aj~ F~,
//   A_ij - I = P + Ai~ + P Ai~,   b_ij = b_j + v + P v,
//   A_j G = G + Aj~ G,   A_i^T Xi22 = Xi22 + Ai~^T Xi22,
//   eta_ij = eta_i + y + Ai~^T y  with  y = z + F~^T z,
// (v = b_i + sqrtC_i sqrtC_i^T eta_j, z = eta_j - sqrtJ_j sqrtJ_j^T b_i).
// ---------------------------------------------------------------------------
// NJ: number of leading columns of sqrtJ_j that can be nonzero (D for an
// aggregate, d for a single step's element, whose sqrtJ is D x d).  The
// remaining columns of the first block of the Xi stack are zero and are left
// out of the tria; Xi11, Xi21 are unchanged and Xi22 keeps its NJ columns.
template <class C, int NJ>
PARAPN_DEV void xi_and_G_F(int lane, typename C::T *sh, const typename C::T (&sCi)[C::D],
                           const typename C::T (&sJj)[C::D], typename C::T (&G)[C::D], typename C::T (&F)[C::D])
{
    using T = typename C::T;
    constexpr int D = C::D, D2 = C::D2, LDM = C::LDM, LDB = C::LDB, NC = NJ + D;
    T *M0 = sh + C::M0, *M1 = sh + C::M1;
    put_rows<T, D, D>(M0, LDM, lane, sCi);
    put_rows<T, D, D>(M1, LDM, lane, sJj);
    wave_sync();
    T w[NC];
    if (lane < D) {
        T t[NJ];
        rowT_times<T, D, NJ>(t, lane, M0, LDM, M1, LDM);
#pragma unroll
        for (int c = 0; c < NJ; ++c) w[c] = t[c];
#pragma unroll
        for (int c = 0; c < D; ++c) w[NJ + c] = (c == lane) ? T(1) : T(0);
    } else if (lane < D2) {
#pragma unroll
        for (int c = 0; c < NJ; ++c) w[c] = M1[(lane - D) * LDM + c];
#pragma unroll
        for (int c = 0; c < D; ++c) w[NJ + c] = 0;
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = 0;
    }
    tria_rows_g<T, D2, NC, C::R, C::SAFE>(w, lane, sh + C::TR);
    T *Xi = sh + C::BIG;
    put_rows<T, D2, NC>(Xi, LDB, lane, w);
    wave_sync();
    // G row = sqrtC_i row * Xi11^{-T};  F~ row = -G row * Xi21^T
    solve_xLt<T, D>(G, sCi, Xi, LDB);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T f = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) f -= G[k] * Xi[(D + c) * LDB + k];
        F[c] = f;
    }
}

// NJ, NCJ: leading columns of sqrtJ_j and sqrtC_j that can be nonzero
// (D, D for aggregates; d, D - d for a single step's element).
template <class C, int NJ, int NCJ>
PARAPN_DEV FRow<C> filter_combine(int lane, typename C::T *sh, const FRow<C> &ei, const FRow<C> &ej)
{
    using T = typename C::T;
    constexpr int D = C::D, LDM = C::LDM, LDB = C::LDB;
    T G[D], F[D];
    xi_and_G_F<C, NJ>(lane, sh, ei.sC, ej.sJ, G, F);
    T *M0 = sh + C::M0, *M1 = sh + C::M1, *M2 = sh + C::M2, *M3 = sh + C::M3, *M4 = sh + C::M4;
    T *V0 = sh + C::V0, *V1 = sh + C::V1, *V2 = sh + C::V2, *V3 = sh + C::V3, *V4 = sh + C::V4, *V5 = sh + C::V5;
    const T *Xi = sh + C::BIG;
    // vectors: wv = sqrtC_i^T eta_j, u = sqrtJ_j^T b_i   (M0 = sqrtC_i, M1 = sqrtJ_j)
    if (lane < D) {
        V0[lane] = ej.eta;
        V1[lane] = ei.b;
    }
    put_rows<T, D, D>(M2, LDM, lane, F);
    put_rows<T, D, D>(M3, LDM, lane, ei.A);
    put_rows<T, D, D>(M4, LDM, lane, G);
    wave_sync();
    if (lane < D) {
        T wv = 0, uu = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) wv += M0[k * LDM + lane] * V0[k];
        if (lane < NJ)
#pragma unroll
            for (int k = 0; k < D; ++k) uu += M1[k * LDM + lane] * V1[k];
        V2[lane] = wv;
        V3[lane] = uu;
    }
    wave_sync();
    FRow<C> o;
    zero(o);
    // P = A_j F - I = Aj~ + F~ + Aj~ F~  (M2 holds F~)
    T ajf[D];
    row_times<T, D, D>(ajf, ej.A, M2, LDM);
#pragma unroll
    for (int c = 0; c < D; ++c) ajf[c] += ej.A[c] + F[c];
    if (lane < D) {
        // v = b_i + sqrtC_i wv ;  z = eta_j - sqrtJ_j u
        T v = ei.b, z = ej.eta;
#pragma unroll
        for (int c = 0; c < D; ++c) v += ei.sC[c] * V2[c];
#pragma unroll
        for (int c = 0; c < NJ; ++c) z -= ej.sJ[c] * V3[c];
        V4[lane] = v;
        V5[lane] = z;
    }
    wave_sync();
    if (lane < D) {
        // A_ij - I = P + Ai~ + P Ai~  (M3 holds Ai~)
        row_times<T, D, D>(o.A, ajf, M3, LDM);
#pragma unroll
        for (int c = 0; c < D; ++c) o.A[c] += ajf[c] + ei.A[c];
        // b_ij = b_j + v + P v,  y = z + F~^T z
        T pv = 0;
        T y = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            pv += ajf[k] * V4[k];
            y += M2[k * LDM + lane] * V5[k];
        }
        o.b = ej.b + (V4[lane] + pv);
        V0[lane] = V5[lane] + y;  // eta_j no longer needed
    }
    wave_sync();
    // sqrtC_ij = tria([A_j G, sqrtC_j]) and sqrtJ_ij = tria([A_i^T Xi22,
    // sqrtJ_i]) (Xi22 has NJ columns), two independent trias run together
    {
        T w[D + NCJ], wj[NJ + D];
        if (lane < D) {
            // A_j G = G + Aj~ G
            T t[D];
            row_times<T, D, D>(t, ej.A, M4, LDM);
#pragma unroll
            for (int c = 0; c < D; ++c) w[c] = t[c] + G[c];
#pragma unroll
            for (int c = 0; c < NCJ; ++c) w[D + c] = ej.sC[c];
            // A_i^T Xi22 = Xi22 + Ai~^T Xi22
            T tj[NJ];
            rowT_times<T, D, NJ>(tj, lane, M3, LDM, Xi + D * LDB + D, LDB);
#pragma unroll
            for (int c = 0; c < NJ; ++c) wj[c] = tj[c] + Xi[(D + lane) * LDB + D + c];
#pragma unroll
            for (int c = 0; c < D; ++c) wj[NJ + c] = ei.sJ[c];
            // eta_ij = eta_i + y + Ai~^T y
            T et = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) et += M3[k * LDM + lane] * V0[k];
            o.eta = ei.eta + (V0[lane] + et);
        } else {
#pragma unroll
            for (int c = 0; c < D + NCJ; ++c) w[c] = 0;
#pragma unroll
            for (int c = 0; c < NJ + D; ++c) wj[c] = 0;
        }
        tria2_rows_g<T, D, D + NCJ, NJ + D, C::R, C::SAFE>(w, wj, lane, sh + C::TR);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            o.sC[c] = lane < D ? w[c] : T(0);
            o.sJ[c] = lane < D ? wj[c] : T(0);
        }
    }
    wave_sync();
    return o;
}

// state (mean m, factor P) followed by aggregate a_j (holding A_j - I): the
// filtering operator with A_i = 0, eta_i = 0, sqrtJ_i = 0; returns the new
// (b_ij, sqrtC_ij).
template <class C>
PARAPN_DEV SRow<C> state_apply(int lane, typename C::T *sh, const SRow<C> &s, const FRow<C> &ej)
{
    using T = typename C::T;
    constexpr int D = C::D, D2 = C::D2, LDM = C::LDM;
    T G[D], F[D];
    xi_and_G_F<C, C::D>(lane, sh, s.P, ej.sJ, G, F);
    T *M0 = sh + C::M0, *M2 = sh + C::M2, *M4 = sh + C::M4;
    T *V0 = sh + C::V0, *V2 = sh + C::V2, *V4 = sh + C::V4;
    if (lane < D) V0[lane] = ej.eta;
    put_rows<T, D, D>(M2, LDM, lane, F);
    put_rows<T, D, D>(M4, LDM, lane, G);
    wave_sync();
    if (lane < D) {
        T wv = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) wv += M0[k * LDM + lane] * V0[k];
        V2[lane] = wv;
    }
    wave_sync();
    // P = A_j F - I = Aj~ + F~ + Aj~ F~
    T ajf[D];
    row_times<T, D, D>(ajf, ej.A, M2, LDM);
#pragma unroll
    for (int c = 0; c < D; ++c) ajf[c] += ej.A[c] + F[c];
    T v = 0;
    if (lane < D) {
        v = s.m;
#pragma unroll
        for (int c = 0; c < D; ++c) v += s.P[c] * V2[c];
        V4[lane] = v;
    }
    wave_sync();
    SRow<C> o;
    o.m = 0;
    if (lane < D) {
        // b = b_j + v + P v
        T pv = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) pv += ajf[k] * V4[k];
        o.m = ej.b + (v + pv);
    }
    T w[D2];
    if (lane < D) {
        // A_j G = G + Aj~ G
        T t[D];
        row_times<T, D, D>(t, ej.A, M4, LDM);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            w[c] = t[c] + G[c];
            w[D + c] = ej.sC[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < D2; ++c) w[c] = 0;
    }
    tria_rows_g<T, D, D2, C::R, C::SAFE>(w, lane, sh + C::TR);
#pragma unroll
    for (int c = 0; c < D; ++c) o.P[c] = lane < D ? w[c] : T(0);
    return o;
}

// One Kalman step from the filtering marginal (m, sqrtP) of step n-1 --
// the filtering operator applied to a prefix state, which has A = 0, eta = 0,
// J = 0 -- together with the smoothing element of step n-1
// (eq. sqrt-smoothing-elements).  The stacked tria
//   Pi = tria([[Phi sqrtP, sqrtQ], [sqrtP, 0]])   (2D x 2D)
// gives Pi11 = tria([Phi sqrtP, sqrtQ]), the predicted factor of step n (its
// first D reflections are the prediction's), and
//   E_{n-1} = Pi21 Pi11^{-1},  sqrtL_{n-1} = Pi22,
// with the predicted mean m- = Phi m + u_n.  The update is
//   Psi = tria([[H sqrtP-], [sqrtP-]]),  K = Psi21 Psi11^{-1},
//   k = K (r - H m-),  m = m- + k,  sqrtP = Psi22.
// The element's offset is kept in correction form, E_{n-1} k (the paper's
// g_{n-1} = m - E_{n-1} m- is m + E_{n-1} k minus E_{n-1} applied to the
// smoothed mean, see the top of this file).  The smoothing element (E,
// E k) and the filtering mean m of step n-1 come back in lanes D..2D-1 (row
// lane - D; the mean in mf_prev).
// qf (lane 0; 0 elsewhere): the quadratic form r^T S^-1 r of the step's
// innovation r over the d ODE rows, S = Psi11 Psi11^T (the prediction-error
// term of the quasi-maximum-likelihood diffusion, Sec. 2.4).
template <class C>
PARAPN_DEV SRow<C> kf_step_se(int lane, typename C::T *sh, const SRow<C> &s, const typename C::T *cphi,
                              const typename C::T *csq, ERow<C> &eo, typename C::T &mf_prev, typename C::T &qf)
{
    using T = typename C::T;
    constexpr int d = C::d, D = C::D, D2 = C::D2, LDM = C::LDM, LDB = C::LDB;
    T *M0 = sh + C::M0, *V0 = sh + C::V0, *V1 = sh + C::V1, *V2 = sh + C::V2;
    put_rows<T, D, D>(M0, LDM, lane, s.P);
    if (lane < D) V0[lane] = s.m;
    wave_sync();
    T mp = 0;
    T w[D2];
    if (lane < D) {
        T phirow[D], t[D];
#pragma unroll
        for (int k = 0; k < D; ++k) phirow[k] = cphi[lane * LDM + k];
        row_times<T, D, D>(t, phirow, M0, LDM);
        mp = sh[C::UO + lane];
#pragma unroll
        for (int k = 0; k < D; ++k) mp += phirow[k] * V0[k];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            w[c] = t[c];
            w[D + c] = csq[lane * LDM + c];
        }
    } else if (lane < D2) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            w[c] = M0[(lane - D) * LDM + c];
            w[D + c] = 0;
        }
    } else {
#pragma unroll
        for (int c = 0; c < D2; ++c) w[c] = 0;
    }
    tria_rows_g<T, D2, D2, C::R, C::SAFE>(w, lane, sh + C::TR);
    T *Pi = sh + C::BIG;
    put_rows<T, D2, D2>(Pi, LDB, lane, w);
    if (lane < D) V1[lane] = mp;
    wave_sync();
    eo.g = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) eo.E[c] = eo.L[c] = 0;
    if (lane >= D && lane < D2) {
        T p21[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            p21[c] = w[c];
            eo.L[c] = w[D + c];
        }
        solve_xL<T, D>(eo.E, p21, Pi, LDB);
    }
    // update with the predicted factor Pi11 (rows 0..D-1 of Pi):
    // tria([[H Pi11, sqrtR], [Pi11, 0]])
    constexpr int DO = C::DO, NZ = C::NZ;
    T x[D + NZ];
#pragma unroll
    for (int c = 0; c < D + NZ; ++c) x[c] = 0;
    if (lane < DO) {
        T hrow[D], t[D];
#pragma unroll
        for (int c = 0; c < D; ++c) hrow[c] = sh[C::HO + lane * LDM + c];
        row_times<T, D, D>(t, hrow, Pi, LDB);
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = t[c];
        if constexpr (NZ > 0) {
            const T sn = sh[C::DVO + DO];
#pragma unroll
            for (int i = 0; i < NZ; ++i)
                if (lane == d + i) x[D + i] = sn;
        }
    } else if (lane < DO + D) {
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = Pi[(lane - DO) * LDB + c];
    }
    wave_sync();
    tria_rows_g<T, DO + D, D + NZ, C::R, C::SAFE>(x, lane, sh + C::TR);
    T *Psi = sh + C::BIG;
    put_rows<T, DO + D, D + NZ>(Psi, LDB, lane, x);
    wave_sync();
    SRow<C> o;
    o.m = 0;
    qf = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) o.P[c] = 0;
    if (lane < D) {
        T res[DO], p21[DO], K[DO];
#pragma unroll
        for (int i = 0; i < DO; ++i) {
            T r = sh[C::DVO + i];
#pragma unroll
            for (int k = 0; k < D; ++k) r -= sh[C::HO + i * LDM + k] * V1[k];
            res[i] = r;
            p21[i] = Psi[(DO + lane) * LDB + i];
        }
        solve_xL<T, DO>(K, p21, Psi, LDB);
        T k = 0;
#pragma unroll
        for (int i = 0; i < DO; ++i) k += K[i] * res[i];
        o.m = mp + k;
        V2[lane] = k;
        if (lane == 0) {
            // Psi11^-1 r over the leading d rows (their block of the factor is
            // the factor of their block of S)
            T x[d], acc = 0;
#pragma unroll
            for (int i = 0; i < d; ++i) {
                T v = res[i];
#pragma unroll
                for (int j = 0; j < i; ++j) v -= Psi[i * LDB + j] * x[j];
                x[i] = v / Psi[i * LDB + i];
                acc += x[i] * x[i];
            }
            qf = acc;
        }
#pragma unroll
        for (int c = 0; c < D - d; ++c) o.P[c] = Psi[(DO + lane) * LDB + DO + c];
    }
    wave_sync();
    mf_prev = 0;
    if (lane >= D && lane < D2) {
        T g = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) g += eo.E[c] * V2[c];
        eo.g = g;
        mf_prev = V0[lane - D];
    }
    wave_sync();
    return o;
}

// ---------------------------------------------------------------------------
// smoothing side (eq. sqrt-smoothing-elements, eq. sqrt-associative-smoothing)
// ---------------------------------------------------------------------------
// acc (x)_s b : E = E_acc E_b, g = E_acc g_b + g_acc, sqrtL = tria([E_acc sqrtL_b, sqrtL_acc])
template <class C, bool WITH_L>
PARAPN_DEV ERow<C> smoother_combine(int lane, typename C::T *sh, const ERow<C> &a, const ERow<C> &b)
{
    using T = typename C::T;
    constexpr int D = C::D, D2 = C::D2, LDM = C::LDM;
    T *M0 = sh + C::M0, *M1 = sh + C::M1, *V0 = sh + C::V0;
    put_rows<T, D, D>(M0, LDM, lane, b.E);
    if (WITH_L) put_rows<T, D, D>(M1, LDM, lane, b.L);
    if (lane < D) V0[lane] = b.g;
    wave_sync();
    ERow<C> o;
    o.g = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) o.E[c] = o.L[c] = 0;
    if (lane < D) {
        row_times<T, D, D>(o.E, a.E, M0, LDM);
        T g = a.g;
#pragma unroll
        for (int k = 0; k < D; ++k) g += a.E[k] * V0[k];
        o.g = g;
    }
    if (WITH_L) {
        T w[D2];
        if (lane < D) {
            T t[D];
            row_times<T, D, D>(t, a.E, M1, LDM);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                w[c] = t[c];
                w[D + c] = a.L[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < D2; ++c) w[c] = 0;
        }
        tria_rows_g<T, D, D2, C::R, C::SAFE>(w, lane, sh + C::TR);
#pragma unroll
        for (int c = 0; c < D; ++c) o.L[c] = lane < D ? w[c] : T(0);
    }
    wave_sync();
    return o;
}

// element/aggregate applied to the suffix state after it:
//   m = E m_next + g,  sqrtP = tria([E sqrtP_next, sqrtL])
template <class C, bool WITH_L>
PARAPN_DEV SRow<C> smoother_apply(int lane, typename C::T *sh, const ERow<C> &a, const SRow<C> &s)
{
    using T = typename C::T;
    constexpr int D = C::D, D2 = C::D2, LDM = C::LDM;
    T *M0 = sh + C::M0, *V0 = sh + C::V0;
    if (WITH_L) put_rows<T, D, D>(M0, LDM, lane, s.P);
    if (lane < D) V0[lane] = s.m;
    wave_sync();
    SRow<C> o;
    o.m = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) o.P[c] = 0;
    if (lane < D) {
        T m = a.g;
#pragma unroll
        for (int k = 0; k < D; ++k) m += a.E[k] * V0[k];
        o.m = m;
    }
    if (WITH_L) {
        T w[D2];
        if (lane < D) {
            T t[D];
            row_times<T, D, D>(t, a.E, M0, LDM);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                w[c] = t[c];
                w[D + c] = a.L[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < D2; ++c) w[c] = 0;
        }
        tria_rows_g<T, D, D2, C::R, C::SAFE>(w, lane, sh + C::TR);
#pragma unroll
        for (int c = 0; c < D; ++c) o.P[c] = lane < D ? w[c] : T(0);
    }
    wave_sync();
    return o;
}

// ---------------------------------------------------------------------------
// request boundaries inside a pack
// ---------------------------------------------------------------------------
// A request's first filtering element is p(Y1 | Z1), which does not depend on
// anything earlier (A = 0, eta = 0, J = 0), and its last smoothing element is
// p(Y_N | Z_{1:N}) (E = 0).  Folding across a boundary with the plain
// operators would give the same result up to 0 * x terms; the flags make the
// boundary exact even when a neighbouring request holds NaN or Inf.
template <class C, int NJ, int NCJ>
PARAPN_DEV FRow<C> fcombine(int lane, typename C::T *sh, const FRow<C> &ei, const FRow<C> &ej)
{
    if (ej.flag != 0) return ej;
    FRow<C> o = filter_combine<C, NJ, NCJ>(lane, sh, ei, ej);
    o.flag = ei.flag;
    return o;
}

template <class C>
PARAPN_DEV SRow<C> sapply(int lane, typename C::T *sh, const SRow<C> &st, const FRow<C> &ej)
{
    if (ej.flag != 0) {
        SRow<C> o;
        o.m = ej.b;
#pragma unroll
        for (int c = 0; c < C::D; ++c) o.P[c] = ej.sC[c];
        return o;
    }
    return state_apply<C>(lane, sh, st, ej);
}

template <class C, bool WITH_L>
PARAPN_DEV ERow<C> scombine(int lane, typename C::T *sh, const ERow<C> &a, const ERow<C> &b)
{
    if (a.flag != 0) return a;
    ERow<C> o = smoother_combine<C, WITH_L>(lane, sh, a, b);
    o.flag = b.flag;
    return o;
}

template <class C, bool WITH_L>
PARAPN_DEV SRow<C> sm_apply(int lane, typename C::T *sh, const ERow<C> &a, const SRow<C> &st)
{
    if (a.flag != 0) {
        SRow<C> o;
        o.m = a.g;
#pragma unroll
        for (int c = 0; c < C::D; ++c) o.P[c] = a.L[c];
        return o;
    }
    return smoother_apply<C, WITH_L>(lane, sh, a, st);
}

// request owning step-level chunk c (requests are ordered by chunk index)
template <bool FORWARD>
PARAPN_DEV int find_req(const ReqDev *reqs, int nreq, int64_t c)
{
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t first = FORWARD ? reqs[mid].fchunk : reqs[mid].schunk;
        if (first <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// request taking part in level launch l that owns pack-wide block or group b:
// the last request whose first index at l is <= b (requests that take no part
// in launch l own an empty range, and are never the last such request)
PARAPN_DEV int find_tab(const ScanTab *t, int nreq, int l, int64_t b)
{
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[mid].first[l] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <class C>
struct KArgs {
    using T = typename C::T;
    Pack pk;
    const T *Phi, *sQ, *init;
};

#define PARAPN_GROUP_SETUP(C)                                                \
    using T = typename C::T;                                                 \
    __shared__ T smem[C::GPB * C::SH + 2 * C::D * C::LDM];                   \
    T *cphi = smem + C::GPB * C::SH;                                         \
    T *csq = cphi + C::D * C::LDM;                                           \
    const int lane = threadIdx.x & (C::R - 1);                               \
    const int grp = threadIdx.x / C::R;                                      \
    T *sh = smem + grp * C::SH;                                              \
    (void)sh;                                                                \
    (void)lane

template <class C>
PARAPN_DEV void load_consts(typename C::T *cphi, typename C::T *csq, const typename C::T *Phi,
                            const typename C::T *sQ)
{
    constexpr int D = C::D;
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
        const int r = i / D, c = i % D;
        cphi[r * C::LDM + c] = Phi[i];
        csq[r * C::LDM + c] = sQ[i];
    }
    __syncthreads();
}

template <class C>
PARAPN_DEV SRow<C> init_state(const typename C::T *init, int lane)
{
    return load_state<C>(init, lane);
}

// step level, forward reduce: the aggregate of one chunk of a request's
// steps, a_s (x)_f ... (x)_f a_{e-1}, the elements built on the fly.  A
// request's first element is the initial state combined with its step-1
// element (the paper's a_1 = p(Y1 | Z1)) and carries the boundary flag.
template <class C>
__global__ __launch_bounds__(C::NT) void k_fwd_reduce1(KArgs<C> a, typename C::T *agg)
{
    PARAPN_GROUP_SETUP(C);
    load_consts<C>(cphi, csq, a.Phi, a.sQ);
    const int64_t chunk = (int64_t)blockIdx.x * C::GPB + grp;
    if (chunk >= a.pk.nf) return;
    const int ri = find_req<true>(a.pk.reqs, a.pk.nreq, chunk);
    const ReqView q = view_of(a.pk.reqs[ri]);
    const int b1 = a.pk.reqs[ri].b1;
    const int64_t lc = chunk - a.pk.reqs[ri].fchunk;
    const int64_t fbase = a.pk.ftab[ri].base;
    const int64_t s = 1 + lc * b1;
    const int64_t e = s + b1 <= q.N + 1 ? s + b1 : q.N + 1;
    FRow<C> acc;
    zero(acc);
    // the transition and noise factor of step n: the block's constants, or a
    // time-varying model's Phi_n, sqrtQ_n (padded rows) read from memory.  The
    // two cases are separate inlined copies of the loop, so no pointer in it
    // may address either memory.
    auto fold = [&](const T *phi0, const T *sq0, int64_t stride) __attribute__((always_inline)) {
        for (int64_t n = s; n < e; ++n) {
            const T *pn = phi0 + (n - 1) * stride, *qn = sq0 + (n - 1) * stride;
            obs_setup<C>(a.pk, q, n, lane, sh, pn);
            FRow<C> el = filter_element<C>(lane, sh, pn, qn);
            if (n == 1) {
                SRow<C> st = state_apply<C>(lane, sh, init_state<C>(a.init, lane), el);
                zero(el);
                el.b = st.m;
#pragma unroll
                for (int c = 0; c < C::D; ++c) {
                    el.sC[c] = st.P[c];
                    el.A[c] = (c == lane) ? T(-1) : T(0);  // A = 0
                }
                el.flag = 1;
            }
            if (n == s)
                acc = el;
            else
                acc = filter_combine<C, C::DO, C::D - C::d>(lane, sh, acc, el);
        }
    };
    if (a.pk.phin)
        fold((const T *)a.pk.phin, (const T *)a.pk.sqn, C::D * C::LDM);
    else
        fold(cphi, csq, 0);
    store_frow<C>(agg + (fbase + lc) * C::FEF, lane, acc);
}

// Upper levels of the forward scan as in-workgroup trees: one leaf
// aggregate per group, W leaves per block.  The up-sweep combines pairs at
// doubling strides (depth log2 W) and keeps every left child for the
// down-sweep; the down-sweep gives each right child the state of its parent
// followed by its left sibling (Blelloch's schedule).  Node index of a left
// child at stride s (s = 1, 2, ..) within a block: off(s) + g / (2s) with
// off(s) = W - W/s, W - 1 nodes per block.
template <class C>
PARAPN_DEV int tree_node(int s, int g)
{
    return C::W - C::W / s + g / (2 * s);
}

// Request, block within its level, and level of one block of a tree launch:
// launch level >= 1 folds level `level` into level+1 for every request that
// has it; level 0 is the top (one block per request, on its last level).
struct TreePos {
    int r;
    int l;
    int64_t lb;
};

PARAPN_DEV TreePos tree_pos(const ScanTab *tab, int nreq, int level)
{
    TreePos p;
    if (level > 0) {
        p.r = find_tab(tab, nreq, level, blockIdx.x);
        p.l = level;
        p.lb = (int64_t)blockIdx.x - tab[p.r].first[level];
    } else {
        p.r = blockIdx.x;
        p.l = tab[p.r].L;
        p.lb = 0;
    }
    return p;
}

template <class C>
__global__ __launch_bounds__(C::NT) void k_fwd_tree_up(Pack pk, typename C::T *agg, typename C::T *part, int level)
{
    PARAPN_GROUP_SETUP(C);
    __shared__ T xch[C::GPB * C::FEF];
    const TreePos tp = tree_pos(pk.ftab, pk.nreq, level);
    const ScanTab &t = pk.ftab[tp.r];
    const T *in = agg + (t.base + t.off[tp.l]) * C::FEF;
    const int64_t nin = t.n[tp.l];
    T *pp = part + (t.pbase + t.poff[tp.l] + tp.lb * (C::W - 1)) * C::FEF;
    const int64_t leaf = tp.lb * C::W + grp;
    FRow<C> acc;
    if (leaf < nin)
        acc = load_frow<C>(in + leaf * C::FEF, lane);
    else
        zero(acc);
    for (int s = 1; s < C::W; s <<= 1) {
        if (grp % (2 * s) == s && leaf < nin) store_frow<C>(xch + grp * C::FEF, lane, acc);
        __syncthreads();
        if (grp % (2 * s) == 0 && leaf < nin) {
            store_frow<C>(pp + tree_node<C>(s, grp) * C::FEF, lane, acc);
            if (leaf + s < nin) {
                FRow<C> r = load_frow<C>(xch + (grp + s) * C::FEF, lane);
                acc = fcombine<C, C::D, C::D>(lane, sh, acc, r);
            }
        }
        __syncthreads();
    }
    if (grp == 0 && level > 0) store_frow<C>(agg + (t.base + t.off[tp.l + 1] + tp.lb) * C::FEF, lane, acc);
}

// down-sweep of one tree: the block's incoming state is the prefix state of
// its node one level up (the top tree starts from the initial state)
template <class C>
__global__ __launch_bounds__(C::NT) void k_fwd_tree_down(Pack pk, const typename C::T *part, typename C::T *pref,
                                                         const typename C::T *init, int level)
{
    PARAPN_GROUP_SETUP(C);
    __shared__ T xch[C::GPB * C::FS];
    const TreePos tp = tree_pos(pk.ftab, pk.nreq, level);
    const ScanTab &t = pk.ftab[tp.r];
    const int64_t nin = t.n[tp.l];
    const T *pp = part + (t.pbase + t.poff[tp.l] + tp.lb * (C::W - 1)) * C::FEF;
    const int64_t leaf = tp.lb * C::W + grp;
    SRow<C> st = level > 0 ? load_state<C>(pref + (t.base + t.off[tp.l + 1] + tp.lb) * C::FS, lane)
                           : load_state<C>(init, lane);
    for (int s = C::W / 2; s >= 1; s >>= 1) {
        if (grp % (2 * s) == 0 && leaf + s < nin) {
            FRow<C> left = load_frow<C>(pp + tree_node<C>(s, grp) * C::FEF, lane);
            SRow<C> r = sapply<C>(lane, sh, st, left);
            store_state<C>(xch + (grp + s) * C::FS, lane, r);
        }
        __syncthreads();
        if (grp % (2 * s) == s && leaf < nin) st = load_state<C>(xch + grp * C::FS, lane);
        __syncthreads();
    }
    if (leaf < nin) store_state<C>(pref + (t.base + t.off[tp.l] + leaf) * C::FS, lane, st);
}

// step level, forward down-sweep: Kalman steps from the chunk's prefix state
// (a request's first chunk starts from the initial state).  The smoothing
// element of a step is formed from its filtering marginal inside the next
// step's Kalman step, so a chunk covering steps s..e-1 writes the elements
// (E, E k, m^f) and sqrtL of steps s-1..e-2; the chunk holding step N also
// writes the last element (E = 0, offset 0, m^f_N, sqrtL = sqrtP^f_N,
// boundary flag).
// Filtering marginals are written only when mf is given.
template <class C>
__global__ __launch_bounds__(C::NT) void k_fwd_down1(KArgs<C> a, const typename C::T *pref, typename C::T *se,
                                                     typename C::T *sL, typename C::T *mf, typename C::T *sPf)
{
    PARAPN_GROUP_SETUP(C);
    load_consts<C>(cphi, csq, a.Phi, a.sQ);
    constexpr int D = C::D;
    const int64_t chunk = (int64_t)blockIdx.x * C::GPB + grp;
    const bool valid = chunk < a.pk.nf;
    double qsum = 0.0;  // lane 0: the chunk's innovation quadratic forms
    unsigned long long *qdst = nullptr;
    if (valid) {
        const int ri = find_req<true>(a.pk.reqs, a.pk.nreq, chunk);
        const ReqView q = view_of(a.pk.reqs[ri]);
        qdst = q.dbits;
        const int b1 = a.pk.reqs[ri].b1;
        const int64_t lc = chunk - a.pk.reqs[ri].fchunk;
        const int64_t s = 1 + lc * b1;
        const int64_t e = s + b1 <= q.N + 1 ? s + b1 : q.N + 1;
        SRow<C> st = s == 1 ? init_state<C>(a.init, lane)
                            : load_state<C>(pref + (a.pk.ftab[ri].base + lc) * C::FS, lane);
        if (s == 1 && mf && lane < D) {
            mf[q.row * D + lane] = st.m;
            store_packed<C>(sPf + q.row * C::DP, lane, st.P);
        }
        // as in k_fwd_reduce1: the constant or the time-varying model, each
        // in its own inlined copy of the loop
        auto walk = [&](const T *phi0, const T *sq0, int64_t stride) __attribute__((always_inline)) {
            for (int64_t n = s; n < e; ++n) {
                const T *pn = phi0 + (n - 1) * stride, *qn = sq0 + (n - 1) * stride;
                obs_setup<C>(a.pk, q, n, lane, sh, pn);
                ERow<C> eo;
                T mfp, qf;
                st = kf_step_se<C>(lane, sh, st, pn, qn, eo, mfp, qf);
                qsum += (double)qf;
                const int64_t row = q.row + n - 1;
                if (lane >= D && lane < C::D2) {
                    const int r = lane - D;
                    T *rec = se + row * C::SEF;
#pragma unroll
                    for (int c = 0; c < D; ++c) rec[r * D + c] = eo.E[c];
                    rec[D * D + r] = eo.g;
                    rec[D * D + D + r] = mfp;
                    if (r == 0) rec[C::SE] = 0;
                    store_packed<C>(sL + row * C::DP, r, eo.L);
                }
                if (mf && lane < D) {
                    mf[(row + 1) * D + lane] = st.m;
                    store_packed<C>(sPf + (row + 1) * C::DP, lane, st.P);
                }
            }
        };
        if (a.pk.phin)
            walk((const T *)a.pk.phin, (const T *)a.pk.sqn, D * C::LDM);
        else
            walk(cphi, csq, 0);
        if (e == q.N + 1 && lane < D) {
            const int64_t row = q.row + q.N;
            T *rec = se + row * C::SEF;
#pragma unroll
            for (int c = 0; c < D; ++c) rec[lane * D + c] = 0;
            rec[D * D + lane] = 0;
            rec[D * D + D + lane] = st.m;
            if (lane == 0) rec[C::SE] = 1;
            store_packed<C>(sL + row * C::DP, lane, st.P);
        }
    }
    // Block-level sums, then one atomic per counter slot present in the block
    // (a block's chunks are consecutive, so requests -- and requests sharing
    // a slot -- form runs).
    __shared__ double qred[C::GPB];
    __shared__ unsigned long long *qptr[C::GPB];
    if (lane == 0) {
        qred[grp] = qsum;
        qptr[grp] = qdst;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *cur = nullptr;
        double x = 0.0;
        for (int g = 0; g <= C::GPB; ++g) {
            unsigned long long *r = g < C::GPB ? qptr[g] : nullptr;
            if (r != cur) {
                if (cur) atomicAdd((double *)cur + 2, x);
                cur = r;
                x = 0.0;
            }
            if (r) x += qred[g];
        }
    }
}

template <class C, bool WITH_L>
PARAPN_DEV ERow<C> load_selem(const typename C::T *se, const typename C::T *sL, int64_t n, int lane)
{
    constexpr int D = C::D;
    ERow<C> e;
    e.g = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) e.E[c] = e.L[c] = 0;
    e.flag = se[n * C::SEF + C::SE];
    if (lane < D) {
        const typename C::T *rec = se + n * C::SEF;
#pragma unroll
        for (int c = 0; c < D; ++c) e.E[c] = rec[lane * D + c];
        e.g = rec[D * D + lane];
    }
    if (WITH_L) load_packed<C>(e.L, sL + n * C::DP, lane);
    return e;
}

template <class C>
PARAPN_DEV ERow<C> load_sagg(const typename C::T *rec, int lane)
{
    constexpr int D = C::D;
    ERow<C> e;
    e.g = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) e.E[c] = e.L[c] = 0;
    e.flag = rec[C::SA];
    if (lane < D) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            e.E[c] = rec[lane * D + c];
            e.L[c] = rec[D * D + D + lane * D + c];
        }
        e.g = rec[D * D + lane];
    }
    return e;
}

template <class C>
PARAPN_DEV void store_sagg(typename C::T *rec, int lane, const ERow<C> &e)
{
    constexpr int D = C::D;
    if (lane == 0) rec[C::SA] = e.flag;
    if (lane < D) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            rec[lane * D + c] = e.E[c];
            rec[D * D + D + lane * D + c] = e.L[c];
        }
        rec[D * D + lane] = e.g;
    }
}


// step level, smoother reduce over one chunk of a request's steps:
// b_s (x)_s ... (x)_s b_{e-1}
template <class C, bool WITH_L>
__global__ __launch_bounds__(C::NT) void k_bwd_reduce1(KArgs<C> a, const typename C::T *se,
                                                       const typename C::T *sL, typename C::T *agg)
{
    PARAPN_GROUP_SETUP(C);
    const int64_t chunk = (int64_t)blockIdx.x * C::GPB + grp;
    if (chunk >= a.pk.ns) return;
    const int ri = find_req<false>(a.pk.reqs, a.pk.nreq, chunk);
    const ReqView q = view_of(a.pk.reqs[ri]);
    const int64_t lc = chunk - a.pk.reqs[ri].schunk;
    const int64_t s = lc * C::B1;
    const int cnt = (int)(s + C::B1 <= q.N + 1 ? C::B1 : q.N + 1 - s);
    const int64_t row0 = q.row + s;
    // the chunk's elements are loaded up front so the fold does not wait on
    // memory (unless they would not fit in registers: factors at large D)
    constexpr bool PREFETCH = !WITH_L || C::D <= 8;
    constexpr int NB = PREFETCH ? C::B1 : 1;
    ERow<C> els[NB];
    if (PREFETCH) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (i < cnt) els[i] = load_selem<C, WITH_L>(se, sL, row0 + i, lane);
    }
    ERow<C> acc = load_selem<C, WITH_L>(se, sL, row0, lane);
#pragma unroll
    for (int i = 1; i < C::B1; ++i)
        if (i < cnt)
            acc = scombine<C, WITH_L>(lane, sh, acc,
                                      PREFETCH ? els[i % NB] : load_selem<C, WITH_L>(se, sL, row0 + i, lane));
    store_sagg<C>(agg + (a.pk.stab[ri].base + lc) * C::SAF, lane, acc);
}

// reverse launch l >= 1: one group per node of level l+1 of each request
// that has it, folding bu consecutive level-l aggregates
template <class C, bool WITH_L>
__global__ __launch_bounds__(C::NT) void k_bwd_reduce(Pack pk, typename C::T *agg, int level)
{
    PARAPN_GROUP_SETUP(C);
    const int64_t g = (int64_t)blockIdx.x * C::GPB + grp;
    if (g >= pk.sgroups[level]) return;
    const ScanTab &t = pk.stab[find_tab(pk.stab, pk.nreq, level, g)];
    const int64_t lg = g - t.first[level];
    const T *in = agg + (t.base + t.off[level]) * C::SAF;
    const int64_t nin = t.n[level];
    const int64_t s = lg * pk.bu;
    const int64_t e = s + pk.bu <= nin ? s + pk.bu : nin;
    ERow<C> acc = load_sagg<C>(in + s * C::SAF, lane);
    for (int64_t i = s + 1; i < e; ++i) {
        ERow<C> el = load_sagg<C>(in + i * C::SAF, lane);
        acc = scombine<C, WITH_L>(lane, sh, acc, el);
    }
    store_sagg<C>(agg + (t.base + t.off[level + 1] + lg) * C::SAF, lane, acc);
}

// top: one block (one group) per request: exclusive suffix scan, from the
// right, of the aggregates of its last level; the state after its last
// aggregate is irrelevant because that aggregate holds the request's last
// element
template <class C, bool WITH_L>
__global__ __launch_bounds__(C::R) void k_bwd_top(Pack pk, const typename C::T *agg, typename C::T *suf)
{
    PARAPN_GROUP_SETUP(C);
    if (grp != 0) return;
    const ScanTab &t = pk.stab[blockIdx.x];
    const int l = t.L;
    const T *a = agg + (t.base + t.off[l]) * C::SAF;
    T *o = suf + (t.base + t.off[l]) * C::SS;
    SRow<C> st;
    st.m = 0;
#pragma unroll
    for (int c = 0; c < C::D; ++c) st.P[c] = 0;
    for (int64_t i = t.n[l] - 1; i >= 0; --i) {
        store_state<C>(o + i * C::SS, lane, st);
        if (i > 0) {
            ERow<C> el = load_sagg<C>(a + i * C::SAF, lane);
            st = sm_apply<C, WITH_L>(lane, sh, el, st);
        }
    }
}

template <class C, bool WITH_L>
__global__ __launch_bounds__(C::NT) void k_bwd_down(Pack pk, const typename C::T *agg, typename C::T *suf,
                                                    int level)
{
    PARAPN_GROUP_SETUP(C);
    const int64_t g = (int64_t)blockIdx.x * C::GPB + grp;
    if (g >= pk.sgroups[level]) return;
    const ScanTab &t = pk.stab[find_tab(pk.stab, pk.nreq, level, g)];
    const int64_t lg = g - t.first[level];
    const T *a = agg + (t.base + t.off[level]) * C::SAF;
    T *o = suf + (t.base + t.off[level]) * C::SS;
    const int64_t nin = t.n[level];
    const int64_t s = lg * pk.bu;
    const int64_t e = s + pk.bu <= nin ? s + pk.bu : nin;
    SRow<C> st = load_state<C>(suf + (t.base + t.off[level + 1] + lg) * C::SS, lane);
    for (int64_t i = e - 1; i >= s; --i) {
        store_state<C>(o + i * C::SS, lane, st);
        if (i > s) {
            ERow<C> el = load_sagg<C>(a + i * C::SAF, lane);
            st = sm_apply<C, WITH_L>(lane, sh, el, st);
        }
    }
}

// step level, smoother down-sweep over one chunk of a request's steps from
// its suffix state.  The scan carries the smoothing correction c = m^s - m^f;
// the smoothed mean is the stored m^f plus c.  UPDATE: add the smoothed
// increments to the request's
// FP64 trajectory (the next linearisation point) and accumulate, in double,
//   delta = max |T0 E0 increment|  and  max |T0 E0 trajectory|
// into the request's counters; otherwise write the smoothed means to mout
// (packed rows).  Returns the group's request and its two maxima (lanes
// hold partial maxima).
template <class C, bool WITH_L, bool UPDATE>
PARAPN_DEV int bwd_down1_group(const KArgs<C> &a, int64_t chunk, int lane, typename C::T *sh,
                               const typename C::T *se, const typename C::T *sL, const typename C::T *suf,
                               typename C::T *mout, typename C::T *sPs, double &dmax, double &mmax)
{
    using T = typename C::T;
    constexpr int D = C::D;
    const int ri = find_req<false>(a.pk.reqs, a.pk.nreq, chunk);
    const ReqView q = view_of(a.pk.reqs[ri]);
    const int64_t lc = chunk - a.pk.reqs[ri].schunk;
    const int64_t sbase = a.pk.stab[ri].base;
    const int64_t s = lc * C::B1;
    const int cnt = (int)(s + C::B1 <= q.N + 1 ? C::B1 : q.N + 1 - s);
    const int64_t row0 = q.row + s;
    constexpr bool PREFETCH = !WITH_L || C::D <= 8;
    constexpr int NB = PREFETCH ? C::B1 : 1;
    ERow<C> els[NB];
    if (PREFETCH) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (i < cnt) els[i] = load_selem<C, WITH_L>(se, sL, row0 + i, lane);
    }
    double told[C::B1];
    if (UPDATE) {
#pragma unroll
        for (int i = 0; i < C::B1; ++i) told[i] = (i < cnt && lane < D) ? q.traj[(s + i) * D + lane] : 0.0;
    }
    // filtering means of the chunk's steps (the scan below yields m^s - m^f)
    T mfv[C::B1];
#pragma unroll
    for (int i = 0; i < C::B1; ++i) mfv[i] = (i < cnt && lane < D) ? se[(row0 + i) * C::SEF + D * D + D + lane] : T(0);
    SRow<C> st = load_state<C>(suf + (sbase + lc) * C::SS, lane);
#pragma unroll
    for (int i = C::B1 - 1; i >= 0; --i) {
        if (i >= cnt) continue;
        const int64_t n = s + i;
        st = sm_apply<C, WITH_L>(lane, sh,
                                 PREFETCH ? els[i % NB] : load_selem<C, WITH_L>(se, sL, row0 + i, lane), st);
        if (lane < D) {
            if (UPDATE) {
                const double inc = (double)mfv[i] + (double)st.m;
                const double nw = told[i] + inc;
                if (lane % C::S == 0) {
                    const double df = fabs(q.T0 * inc);
                    dmax = (df > dmax || df != df) ? df : dmax;
                    const double am = fabs(q.T0 * nw);
                    mmax = (am > mmax || am != am) ? am : mmax;
                }
                q.traj[n * D + lane] = nw;
            } else {
                mout[(row0 + i) * D + lane] = mfv[i] + st.m;
            }
            if (WITH_L) store_packed<C>(sPs + (row0 + i) * C::DP, lane, st.P);
        }
    }
    return ri;
}

PARAPN_DEV double nan_max(double x, double u) { return (u > x || u != u) ? u : x; }

template <class C, bool WITH_L, bool UPDATE>
__global__ __launch_bounds__(C::NT) void k_bwd_down1(KArgs<C> a, const typename C::T *se, const typename C::T *sL,
                                                     const typename C::T *suf, typename C::T *mout,
                                                     typename C::T *sPs)
{
    PARAPN_GROUP_SETUP(C);
    const int64_t chunk = (int64_t)blockIdx.x * C::GPB + grp;
    const bool valid = chunk < a.pk.ns;
    double dmax = 0.0, mmax = 0.0;
    int ri = -1;
    if (valid) ri = bwd_down1_group<C, WITH_L, UPDATE>(a, chunk, lane, sh, se, sL, suf, mout, sPs, dmax, mmax);
    if (UPDATE) {
        // Block-level maxima, then one atomic pair per request present in the
        // block (a block's chunks are consecutive, so its requests form runs):
        // a few thousand atomics per launch instead of two per group.
        // Non-negative doubles order like their bit patterns; NaN sorts above
        // everything.
        // group maxima first, across the group's lanes (XOR shuffles stay
        // inside the group: R is a power of two within one wavefront)
#pragma unroll
        for (int off = C::R / 2; off >= 1; off >>= 1) {
            dmax = nan_max(dmax, __shfl_xor(dmax, off));
            mmax = nan_max(mmax, __shfl_xor(mmax, off));
        }
        __shared__ double red[C::GPB * 2];
        __shared__ int rq[C::GPB];
        if (lane == 0) {
            red[grp] = dmax;
            red[C::GPB + grp] = mmax;
            rq[grp] = ri;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int cur = -1;
            double x = 0.0, y = 0.0;
            for (int g = 0; g <= C::GPB; ++g) {
                const int r = g < C::GPB ? rq[g] : -1;
                if (r != cur) {
                    if (cur >= 0) {
                        unsigned long long *db = a.pk.reqs[cur].dbits;
                        atomicMax(db, (unsigned long long)__double_as_longlong(x));
                        atomicMax(db + 1, (unsigned long long)__double_as_longlong(y));
                    }
                    cur = r;
                    x = y = 0.0;
                }
                if (r < 0) continue;
                x = nan_max(x, red[g]);
                y = nan_max(y, red[C::GPB + g]);
            }
        }
    }
}

// batched filtering operator for the ABI entry point
template <class C>
__global__ __launch_bounds__(C::NT) void k_filter_combine_batch(const typename C::T *aa, const typename C::T *cc,
                                                                typename C::T *out, int64_t count)
{
    PARAPN_GROUP_SETUP(C);
    const int64_t k = (int64_t)blockIdx.x * C::GPB + grp;
    if (k >= count) return;
    FRow<C> ei = load_frow<C, false>(aa + k * C::FE, lane);
    FRow<C> ej = load_frow<C, false>(cc + k * C::FE, lane);
    // the operator works on A - I
#pragma unroll
    for (int c = 0; c < C::D; ++c)
        if (c == lane) {
            ei.A[c] -= T(1);
            ej.A[c] -= T(1);
        }
    FRow<C> o = filter_combine<C, C::D, C::D>(lane, sh, ei, ej);
#pragma unroll
    for (int c = 0; c < C::D; ++c)
        if (c == lane) o.A[c] += T(1);
    store_frow<C, false>(out + k * C::FE, lane, o);
}


// ---------------------------------------------------------------------------
// starting trajectory from a coarse grid (remark on other initial state
// trajectories, Sec. 3.2.2)
// ---------------------------------------------------------------------------
// One wavefront per request runs the sequential extended Kalman smoother on
// the request's coarse grid: M steps of H = s h, in the coordinates of H
// with the IWP prior's h-independent Phi, Q, in FP64 and covariance form
// (the sequential recursion is latency-bound: every lane owns entries of the
// D x D covariance, so a step is a few short dot products, not a chain of
// reflections).  Filter step n: predict m- = Phi m, P- = Phi P Phi^T + Q;
// linearise the vector field at the predicted mean (EK1, Sec. 3.2.1):
//   Hbar = E1 - (H/q) F_y E0,  r = (f(T0 E0 m-) - T1 E1 m-) / T1;
// update with U = P- Hbar^T, S = Hbar U = L_S L_S^T:
//   K = U S^-1,  z = S^-1 r,  m = m- + K r,  P = (I - K Hbar) P- (I - K Hbar)^T
// (the Joseph form: the plain P- - K S K^T loses the small eigenvalues of the
// rank-deficient noiseless-data covariance to cancellation).
// Smoother (the RTS means, written without inverting P-): with
// nu_{M+1} = 0 and t_n = Phi^T nu_{n+1},
//   m^s_n = m^f_n + P_n t_n,   nu_n = Hbar_n^T (z_n - K_n^T t_n) + t_n
//                                   = A_n^T t_n + c_n,
// A_n = I - K_n Hbar_n (the Joseph factor), c_n = Hbar_n^T z_n; this is
// m^s_n = m^f_n + G_n (m^s_{n+1} - m-_{n+1}) with the RTS gain
// G_n = P_n Phi^T (P-_{n+1})^-1 and nu_{n+1} = (P-_{n+1})^-1 (m^s_{n+1} -
// m-_{n+1}).  Per coarse node the records hold m^f_n, P_n, and for n >= 1
// the 2d columns of A_n that differ from I and c_n; the smoothed means go to
// the node array.
// Sequential EK1 filter (covariance form, FP64) on the coarse grid, one
// wavefront per request, then the RTS means.  The coarse prior is the IWP:
// Phi = I_d (x) Phi1 and Q = I_d (x) Q1 with (q+1)-blocks, so a product with
// Phi or Q touches q+1 terms, and Hbar = E1 - (H/q) F_y E0 has d+1 nonzeros
// per row.  With U = P- Hbar^T, S = Hbar U and K = U S^-1 the update is the
// Joseph form (I - K Hbar) P- (I - K Hbar)^T (noiseless data), whose factor
// differs from I in 2d columns only: both products cost O(D^2 d).  (The
// algebraically equal P- - K U^T - U K^T + K S K^T loses definiteness within
// a few dozen steps on FitzHugh-Nagumo: its terms are large and cancel.)
template <int d, int q>
__global__ __launch_bounds__(64) void k_coarse_eks(const ReqDev *reqs, const CoarseDev *cds, const double *Phi,
                                                   const double *Q)
{
    constexpr int S = q + 1, D = d * S, DD = D * D, EPL = (DD + 63) / 64;
    constexpr int REC = coarse_record_doubles(d, q);
    __shared__ double sP[DD], sA[DD], sPp[DD], sm[D], smp[D], sU[D * d], sK[D * d], snu[D];
    const int lane = threadIdx.x;
    const ReqDev &rq = reqs[blockIdx.x];
    const CoarseDev cd = cds[blockIdx.x];
    const int field = rq.field;
    // the parameters in registers: the loop stores to global memory, so
    // values read through the request table would be reloaded every step
    double prm[kMaxParams];
#pragma unroll
    for (int i = 0; i < kMaxParams; ++i) prm[i] = rq.p[i];
    // one (q+1)-block of Phi (uniform: every lane holds it, indexed only by
    // compile-time constants), and each lane's own rows of Phi and entries of Q
    // for the P- entries it forms (loaded once: an array indexed by lane-
    // dependent values would live in scratch memory, and waiting for a scratch
    // load inside the loop waits for every global store before it)
    double p1[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) p1[i][j] = Phi[i * D + j];
    double prow[EPL][S], pcol[EPL][S], qv[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int e = lane + 64 * k, ee = e < DD ? e : 0;
        const int i = ee / D, j = ee % D, ri = i % S, rj = j % S;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            prow[k][l] = Phi[ri * D + l];
            pcol[k][l] = Phi[rj * D + l];
        }
        qv[k] = (i / S == j / S) ? Q[(i % S) * D + (j % S)] : 0.0;
    }
    // the lane's row of Phi1 for m- = Phi m (lane < D holds component lane)
    double prl[S];
#pragma unroll
    for (int l = 0; l < S; ++l) prl[l] = Phi[(lane % S) * D + l];
    gdouble *rec = (gdouble *)cd.gain, *node = (gdouble *)cd.node;
    for (int e = lane; e < DD; e += 64) sP[e] = 0.0;
    if (lane < D) sm[lane] = cd.mu0c[lane];
    wave_sync();
    bool bad = false;
    for (int64_t n = 1; n <= cd.M; ++n) {
        gdouble *rp = rec + (n - 1) * REC;  // node n-1: m^f, P
        if (lane < D) rp[lane] = sm[lane];
        for (int e = lane; e < DD; e += 64) rp[D + e] = sP[e];
        // A = Phi P, m- = Phi m
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int e = lane + 64 * k;
            if (e < DD) {
                const int i = e / D, j = e % D, bi = i / S;
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) acc += prow[k][l] * sP[(bi * S + l) * D + j];
                sA[e] = acc;
            }
        }
        if (lane < D) {
            const int bi = lane / S;
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < S; ++l) acc += prl[l] * sm[bi * S + l];
            smp[lane] = acc;
        }
        wave_sync();
        // P- = A Phi^T + Q (kept in registers for the update, and in LDS)
        double pp[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int e = lane + 64 * k;
            pp[k] = 0.0;
            if (e < DD) {
                const int i = e / D, j = e % D, bj = j / S;
                double acc = qv[k];
#pragma unroll
                for (int l = 0; l < S; ++l) acc += sA[i * D + bj * S + l] * pcol[k][l];
                pp[k] = acc;
                sPp[e] = acc;
            }
        }
        // EK1 observation at the predicted mean (every lane evaluates it)
        Dual<double, d> yd[d], fd[d];
#pragma unroll
        for (int i = 0; i < d; ++i) {
            yd[i].v = cd.T0 * smp[i * S];
#pragma unroll
            for (int j = 0; j < d; ++j) yd[i].g[j] = (i == j) ? 1.0 : 0.0;
        }
        field_eval<d>(field, prm, yd, fd);
        double r[d], hj[d][d];  // hj = -(H/q) F_y
#pragma unroll
        for (int a = 0; a < d; ++a) {
            r[a] = (fd[a].v - cd.T1 * smp[a * S + 1]) * cd.invT1;
#pragma unroll
            for (int b = 0; b < d; ++b) hj[a][b] = -cd.hq * fd[a].g[b];
        }
        // hj[a][b] for lane-dependent a, b, selected among the compile-time
        // entries (dynamic indexing would put the array in scratch memory)
        auto hj_at = [&](int a, int b) {
            double v = 0.0;
#pragma unroll
            for (int x = 0; x < d; ++x)
#pragma unroll
                for (int y = 0; y < d; ++y) v = (x == a && y == b) ? hj[x][y] : v;
            return v;
        };
        wave_sync();
        // U = P- Hbar^T (D x d): U[i][a] = P-[i][a S + 1] + sum_b hj[a][b] P-[i][b S]
        for (int e = lane; e < D * d; e += 64) {
            const int i = e / d, a = e % d;
            double acc = sPp[i * D + a * S + 1];
#pragma unroll
            for (int b = 0; b < d; ++b) acc += hj_at(a, b) * sPp[i * D + b * S];
            sU[e] = acc;
        }
        wave_sync();
        // S = Hbar U (every lane, symmetrised) and its inverse from the
        // adjugate: one FP64 division per step instead of a factorisation's
        // chain of square roots and divisions (d <= 3)
        double Sm[d][d], Si[d][d];
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
            for (int b = 0; b < d; ++b) {
                double acc = sU[(a * S + 1) * d + b];
#pragma unroll
                for (int c = 0; c < d; ++c) acc += hj[a][c] * sU[(c * S) * d + b];
                Sm[a][b] = acc;
            }
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
            for (int b = 0; b < a; ++b) Sm[a][b] = Sm[b][a] = 0.5 * (Sm[a][b] + Sm[b][a]);
        if constexpr (d == 1) {
            Si[0][0] = 1.0 / Sm[0][0];
        } else if constexpr (d == 2) {
            const double id = 1.0 / (Sm[0][0] * Sm[1][1] - Sm[0][1] * Sm[0][1]);
            Si[0][0] = Sm[1][1] * id;
            Si[1][1] = Sm[0][0] * id;
            Si[0][1] = Si[1][0] = -Sm[0][1] * id;
        } else {
            const double c00 = Sm[1][1] * Sm[2][2] - Sm[1][2] * Sm[1][2];
            const double c01 = Sm[1][2] * Sm[0][2] - Sm[0][1] * Sm[2][2];
            const double c02 = Sm[0][1] * Sm[1][2] - Sm[1][1] * Sm[0][2];
            const double id = 1.0 / (Sm[0][0] * c00 + Sm[0][1] * c01 + Sm[0][2] * c02);
            Si[0][0] = c00 * id;
            Si[0][1] = Si[1][0] = c01 * id;
            Si[0][2] = Si[2][0] = c02 * id;
            Si[1][1] = (Sm[0][0] * Sm[2][2] - Sm[0][2] * Sm[0][2]) * id;
            Si[1][2] = Si[2][1] = (Sm[0][2] * Sm[0][1] - Sm[0][0] * Sm[1][2]) * id;
            Si[2][2] = (Sm[0][0] * Sm[1][1] - Sm[0][1] * Sm[0][1]) * id;
        }
        // z = S^-1 r, K = U S^-1
        double z[d];
#pragma unroll
        for (int a = 0; a < d; ++a) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < d; ++c) v += Si[a][c] * r[c];
            z[a] = v;
        }
        // step n: A's columns b S, b S + 1 (rows 0..D-1), then c, after node
        // n's m^f, P
        if (lane < D) {
            double uu[d], kk[d];
#pragma unroll
            for (int a = 0; a < d; ++a) uu[a] = sU[lane * d + a];
#pragma unroll
            for (int a = 0; a < d; ++a) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < d; ++c) v += uu[c] * Si[c][a];
                kk[a] = v;
            }
            double mn = smp[lane];
#pragma unroll
            for (int a = 0; a < d; ++a) {
                sK[lane * d + a] = kk[a];
                mn += kk[a] * r[a];
            }
            sm[lane] = mn;
            bad |= !__builtin_isfinite(mn);
        }
        gdouble *rn = rec + n * REC;
        // c = Hbar^T z: Hbar has 1 at (a, a S + 1) and hj[a][b] at (a, b S)
        if (lane < D) {
            const int b = lane / S, k = lane % S;
            double c0 = 0.0, c1 = 0.0;
#pragma unroll
            for (int a = 0; a < d; ++a) {
                c0 += hj_at(a, b) * z[a];
                c1 = (a == b) ? z[a] : c1;
            }
            rn[D + DD + 2 * d * D + lane] = k == 0 ? c0 : (k == 1 ? c1 : 0.0);
        }
        wave_sync();
        // Joseph form P = A P- A^T, A = I - K Hbar.  A differs from I only in
        // the 2d columns c with c mod S <= 1 (where Hbar has its nonzeros):
        // A[i][b S] = [i == b S] - sum_a K[i][a] hj[a][b],
        // A[i][a S + 1] = [i == a S + 1] - K[i][a].  B = A P- first.
        {
            double bb[EPL];
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const int e = lane + 64 * k;
                bb[k] = 0.0;
                if (e < DD) {
                    const int i = e / D, j = e % D;
                    double ki[d];
#pragma unroll
                    for (int a = 0; a < d; ++a) ki[a] = sK[i * d + a];
                    double acc = (i % S > 1) ? pp[k] : 0.0;
#pragma unroll
                    for (int b = 0; b < d; ++b) {
                        double a0 = (i == b * S) ? 1.0 : 0.0;
#pragma unroll
                        for (int a = 0; a < d; ++a) a0 -= ki[a] * hj[a][b];
                        const double a1 = ((i == b * S + 1) ? 1.0 : 0.0) - ki[b];
                        acc += a0 * sPp[(b * S) * D + j] + a1 * sPp[(b * S + 1) * D + j];
                        if (j == 0) {  // the smoother's record: A[i][b S], A[i][b S + 1]
                            rn[D + DD + (2 * b) * D + i] = a0;
                            rn[D + DD + (2 * b + 1) * D + i] = a1;
                        }
                    }
                    bb[k] = acc;
                }
            }
            // sA is free here (its last reader was the P- stage)
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const int e = lane + 64 * k;
                if (e < DD) sA[e] = bb[k];
            }
            wave_sync();
            // P = B A^T
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const int e = lane + 64 * k;
                if (e < DD) {
                    const int i = e / D, j = e % D;
                    double kj[d];
#pragma unroll
                    for (int a = 0; a < d; ++a) kj[a] = sK[j * d + a];
                    double acc = (j % S > 1) ? bb[k] : 0.0;
#pragma unroll
                    for (int b = 0; b < d; ++b) {
                        double a0 = (j == b * S) ? 1.0 : 0.0;
#pragma unroll
                        for (int a = 0; a < d; ++a) a0 -= kj[a] * hj[a][b];
                        const double a1 = ((j == b * S + 1) ? 1.0 : 0.0) - kj[b];
                        acc += sA[i * D + b * S] * a0 + sA[i * D + b * S + 1] * a1;
                    }
                    sP[e] = acc;
                }
            }
        }
        wave_sync();
    }
    {
        gdouble *rp = rec + cd.M * REC;
        if (lane < D) rp[lane] = sm[lane];
        for (int e = lane; e < DD; e += 64) rp[D + e] = sP[e];
    }
    // smoother.  Each lane's share of a record (its row of P and m^f; for its
    // index i its column of A and c_i) is loaded ahead of its step, so the
    // global-memory latency overlaps the arithmetic of the steps before it.
    // Every lane forms all of t = Phi^T nu from nu in LDS (D (q+1) products:
    // cheaper than a second exchange), so a step is one LDS round trip.
    if (lane < D) snu[lane] = 0.0;
    struct Share {
        double mf, P[D], acol[D], c;
    };
    // Every call issues the same loads, whatever n (0 <= n <= M; record 0's
    // A and c slots are read and left unused): a load taken on one path and
    // skipped on another leaves the compiler no static count of the loads
    // issued after a share, and it then waits for all of them -- the prefetch
    // would not hide anything.  Lanes whose index is not a column of A that
    // differs from I (i mod S > 1) read column 0 and do not use it.
    const int r_own = lane < D ? lane : 0;
    const bool a_col = lane < D && lane % S <= 1;
    const int a_blk = a_col ? 2 * (lane / S) + lane % S : 0;
    auto load_share = [&](int64_t n, Share &sh) {
        const gdouble *rp = rec + n * REC;
        sh.mf = rp[r_own];
#pragma unroll
        for (int l = 0; l < D; ++l) sh.P[l] = rp[D + r_own * D + l];
#pragma unroll
        for (int l = 0; l < D; ++l) sh.acol[l] = rp[D + DD + a_blk * D + l];
        sh.c = rp[D + DD + 2 * d * D + r_own];
    };
    auto at_least0 = [](int64_t k) { return k > 0 ? k : (int64_t)0; };
    // one smoother step on the share of record n
    auto step = [&](int64_t n, const Share &cur) {
        double nu[D], t[D];
#pragma unroll
        for (int j = 0; j < D; ++j) nu[j] = snu[j];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < S; ++l) acc += p1[l][j % S] * nu[(j / S) * S + l];
            t[j] = acc;
        }
        if (lane < D) {
            double acc = cur.mf;
#pragma unroll
            for (int l = 0; l < D; ++l) acc += cur.P[l] * t[l];
            node[n * D + lane] = acc;
            bad |= !__builtin_isfinite(acc);
        }
        if (n >= 1) {
            double v = cur.c, tl = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l) {
                v += cur.acol[l] * t[l];
                tl = (l == lane) ? t[l] : tl;
            }
            if (lane < D) snu[lane] = a_col ? v : tl;
        }
        wave_sync();
    };
    // four buffers taken in turn, loaded three steps ahead: a record comes
    // from L2 in about as long as three steps take.  The loop body holds four
    // steps, so no share is copied (a copy of a share still being loaded
    // would wait for it).
    Share A, B, C, E;
    const int64_t M = cd.M;
    load_share(M, A);
    load_share(at_least0(M - 1), B);
    load_share(at_least0(M - 2), C);
    wave_sync();
    for (int64_t n = M; n >= 0; n -= 4) {
        load_share(at_least0(n - 3), E);
        step(n, A);
        if (n == 0) break;
        load_share(at_least0(n - 4), A);
        step(n - 1, B);
        if (n == 1) break;
        load_share(at_least0(n - 5), B);
        step(n - 2, C);
        if (n == 2) break;
        load_share(at_least0(n - 6), C);
        step(n - 3, E);
    }
    const unsigned long long ballot = __ballot(bad ? 1 : 0);
    if (lane == 0) *cd.status = ballot ? 1 : 0;
}

// Fine row j of request blockIdx.y lies o = j mod s steps after coarse node
// k = j / s; its preconditioned state is, per ODE component, the bridge
// W_o [m_k; m_{k+1}] of the two smoothed coarse means (the prior's mean
// between them; W folds the coordinate changes of H and h).  Row 0 is mu0.
// A request whose coarse smoother produced a non-finite value gets the
// constant start mu0 instead.
static __global__ void k_coarse_bridge(const ReqDev *reqs, const CoarseDev *cds, int d, int q)
{
    const int ri = blockIdx.y;
    const int64_t N = reqs[ri].N;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > N) return;
    const int S = q + 1, D = d * S;
    double *traj = reqs[ri].traj;
    double *row = traj + j * D;
    const double *mu0b = traj + (N + 1) * D + D;  // the resident tail: T, then mu0 / T
    const CoarseDev cd = cds[ri];
    if (j == 0 || *cd.status != 0) {
        for (int k = 0; k < D; ++k) row[k] = mu0b[k];
        return;
    }
    const int64_t k = j / cd.s;
    const int64_t o = j - k * cd.s;
    const double *a = cd.node + k * D;
    const double *b = cd.node + (o ? (k + 1) * D : k * D);
    const double *W = cd.W + o * (int64_t)(2 * S * S);
    for (int i = 0; i < d; ++i)
        for (int r = 0; r < S; ++r) {
            double acc = 0.0;
            for (int c = 0; c < S; ++c) acc += W[r * 2 * S + c] * a[i * S + c] + W[r * 2 * S + S + c] * b[i * S + c];
            row[i * S + r] = acc;
        }
}

// ---------------------------------------------------------------------------
// host-side launch sequences
// ---------------------------------------------------------------------------
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Levels {
    int L;            // number of aggregate levels (>= 1)
    int64_t n[48];    // n[l] aggregates at level l (l = 1..L)
    int64_t off[48];  // record offset of level l
    int64_t total;
};

// forward scan levels: n[1] step-level aggregates, then trees of width W
// until at most W remain (the top tree).  poff[l]: record offset of the tree
// partials of the launch that reduces level l (l = 1..L; level L is the
// single-block top tree).
struct TreeLevels {
    int L;
    int64_t n[48], off[48], poff[48];
    int64_t total, ptotal;
};

static TreeLevels make_tree_levels(int64_t n1, int W)
{
    TreeLevels t{};
    t.L = 1;
    t.n[1] = n1;
    t.off[1] = 0;
    t.poff[1] = 0;
    while (t.n[t.L] > W && t.L < 46) {
        const int64_t nb = (t.n[t.L] + W - 1) / W;
        t.n[t.L + 1] = nb;
        t.off[t.L + 1] = t.off[t.L] + t.n[t.L];
        t.poff[t.L + 1] = t.poff[t.L] + nb * (W - 1);
        ++t.L;
    }
    t.total = t.off[t.L] + t.n[t.L];
    t.ptotal = t.poff[t.L] + (W - 1);
    return t;
}

static Levels make_levels(int64_t n1, int bu, int btop)
{
    Levels lv{};
    lv.L = 1;
    lv.n[1] = n1;
    lv.off[1] = 0;
    while (lv.n[lv.L] > btop && lv.L < 46) {
        lv.n[lv.L + 1] = cdiv(lv.n[lv.L], bu);
        lv.off[lv.L + 1] = lv.off[lv.L] + lv.n[lv.L];
        ++lv.L;
    }
    lv.total = lv.off[lv.L] + lv.n[lv.L];
    return lv;
}

template <class C>
static KArgs<C> make_args(const Pack &pk, const ModelDev &m)
{
    using T = typename C::T;
    KArgs<C> a{};
    a.pk = pk;
    a.Phi = (const T *)m.Phi;
    a.sQ = (const T *)m.sQ;
    a.init = (const T *)m.init;
    return a;
}

template <class C>
static hipError_t fwd_seq(const Pack &pk, const ModelDev &m, const Work &w, hipStream_t s)
{
    using T = typename C::T;
    // the upper levels do not depend on damping (same records, same tree width)
    using CT = Cfg<T, C::d, C::q>;
    if (pk.nf < 1 || pk.nreq < 1 || pk.Lf < 1 || pk.Lf > kMaxLevels) return hipErrorInvalidValue;
    if (C::LM && pk.mode != 0) return hipErrorInvalidValue;
    KArgs<C> a = make_args<C>(pk, m);
    T *agg = (T *)w.fagg, *part = (T *)w.fpart, *pref = (T *)w.fpref;
    auto blocks = [](int64_t groups) { return (unsigned)cdiv(groups, C::GPB); };
    PARAPN_LAUNCH("fwd_reduce1", s, k_fwd_reduce1<C>, dim3(blocks(pk.nf)), dim3(C::NT), 0, s, a, agg);
    for (int l = 1; l < pk.Lf; ++l)
        if (pk.fblocks[l] > 0)
            PARAPN_LAUNCH("fwd_tree_up", s, k_fwd_tree_up<CT>, dim3((unsigned)pk.fblocks[l]), dim3(CT::NT), 0, s, pk,
                          agg, part, l);
    // top trees, one block per request, from the initial state
    PARAPN_LAUNCH("fwd_tree_up", s, k_fwd_tree_up<CT>, dim3((unsigned)pk.nreq), dim3(CT::NT), 0, s, pk, agg, part,
                  0);
    PARAPN_LAUNCH("fwd_tree_down", s, k_fwd_tree_down<CT>, dim3((unsigned)pk.nreq), dim3(CT::NT), 0, s, pk,
                  (const T *)part, pref, (const T *)m.init, 0);
    for (int l = pk.Lf - 1; l >= 1; --l)
        if (pk.fblocks[l] > 0)
            PARAPN_LAUNCH("fwd_tree_down", s, k_fwd_tree_down<CT>, dim3((unsigned)pk.fblocks[l]), dim3(CT::NT), 0, s,
                          pk, (const T *)part, pref, (const T *)m.init, l);
    PARAPN_LAUNCH("fwd_down1", s, k_fwd_down1<C>, dim3(blocks(pk.nf)), dim3(C::NT), 0, s, a, (const T *)pref,
                  (T *)w.se, (T *)w.sL, (T *)w.filt_mf, (T *)w.filt_sPf);
    return hipGetLastError();
}

template <class CF, bool WITH_L>
static hipError_t bwd_seq(const Pack &pk, const ModelDev &m, const Work &w, bool update, void *mout, hipStream_t s)
{
    // the reverse scan works on D rows: groups of next-power-of-two(D) lanes
    using C = Cfg<typename CF::T, CF::d, CF::q, pow2ceil(CF::D)>;
    using T = typename C::T;
    if (pk.ns < 1 || pk.nreq < 1 || pk.Ls < 1 || pk.Ls > kMaxLevels) return hipErrorInvalidValue;
    KArgs<C> a = make_args<C>(pk, m);
    T *agg = (T *)w.sagg, *suf = (T *)w.spref;
    auto blocks = [](int64_t groups) { return (unsigned)cdiv(groups, C::GPB); };
    PARAPN_LAUNCH("bwd_reduce1", s, (k_bwd_reduce1<C, WITH_L>), dim3(blocks(pk.ns)), dim3(C::NT), 0, s, a,
                  (const T *)w.se, (const T *)w.sL, agg);
    for (int l = 1; l < pk.Ls; ++l)
        if (pk.sgroups[l] > 0)
            PARAPN_LAUNCH("bwd_reduce", s, (k_bwd_reduce<C, WITH_L>), dim3(blocks(pk.sgroups[l])), dim3(C::NT), 0, s,
                          pk, agg, l);
    PARAPN_LAUNCH("bwd_top", s, (k_bwd_top<C, WITH_L>), dim3((unsigned)pk.nreq), dim3(C::R), 0, s, pk,
                  (const T *)agg, suf);
    for (int l = pk.Ls - 1; l >= 1; --l)
        if (pk.sgroups[l] > 0)
            PARAPN_LAUNCH("bwd_down", s, (k_bwd_down<C, WITH_L>), dim3(blocks(pk.sgroups[l])), dim3(C::NT), 0, s, pk,
                          (const T *)agg, suf, l);
    if (update)
        PARAPN_LAUNCH("bwd_down1", s, (k_bwd_down1<C, WITH_L, true>), dim3(blocks(pk.ns)), dim3(C::NT), 0, s, a,
                      (const T *)w.se, (const T *)w.sL, (const T *)suf, (T *)nullptr, (T *)w.sPs);
    else
        PARAPN_LAUNCH("bwd_down1", s, (k_bwd_down1<C, WITH_L, false>), dim3(blocks(pk.ns)), dim3(C::NT), 0, s, a,
                      (const T *)w.se, (const T *)w.sL, (const T *)suf, (T *)mout, (T *)w.sPs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename T, typename TS>
__global__ void k_unscale(int D, int64_t N, const double *Td, const TS *src, const T *srcP, T *mo, T *co, double cs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rows = (N + 1) * D;
    if (i >= rows) return;
    const int64_t n = i / D;
    const int r = (int)(i % D);
    const double t = Td ? Td[r] : 1.0;
    if (mo) mo[i] = (T)(t * (double)src[i]);
    if (co) {
        const T *pr = srcP + n * (int64_t)(D * (D + 1) / 2) + r * (r + 1) / 2;
        T *out = co + i * D;
        for (int c = 0; c < D; ++c) out[c] = c <= r ? (T)(cs * t * (double)pr[c]) : T(0);
    }
}

// preconditioned starting trajectory: row 0 is mu0/T; rows n >= 1 are
// init[n] / T (element-wise, may run in place), or mu0/T when init is null.
// Td holds T followed by mu0/T.
template <typename T>
__global__ void k_init_traj(int D, int64_t N, const T *init, const T *Td, T *traj)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (N + 1) * D) return;
    const int k = (int)(i % D);
    traj[i] = (i < D || !init) ? Td[D + k] : init[i] / Td[k];
}

// [N][D][D] -> [N][D][D+1]: one thread per destination entry (the padding
// column is written as zero)
template <typename T>
__global__ void k_pad_rows(int D, int64_t N, const T *src, T *dst)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = N * D * (D + 1);
    if (e >= total) return;
    const int64_t row = e / (D + 1);
    const int c = (int)(e - row * (D + 1));
    dst[e] = c < D ? src[row * D + c] : T(0);
}

// starting trajectories of decoupled chains: one thread per element of
// [B][d][N+1][S]
static __global__ void k_blocks_in(int B, int d, int S, int64_t N, const double *init, const double *Td, const double *mu0b,
                            double *traj)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (N + 1) * S, total = (int64_t)B * d * per;
    if (e >= total) return;
    const int64_t bi = e / per, r = e - bi * per, n = r / S;
    const int k = (int)(r - n * S);
    const int b = (int)(bi / d), i = (int)(bi - (int64_t)b * d);
    const int D = d * S, col = i * S + k;
    traj[e] = (n == 0 || !init) ? mu0b[(int64_t)b * D + col] : init[n * D + col] / Td[k];
}

// one instance's outputs from its decoupled chains: one thread per (n, row)
// of the [N+1][d S] mean; the same thread writes that row of the factor
template <typename T>
__global__ void k_blocks_out(int d, int S, int64_t N, const double *Td, const double *traj, const T *packed,
                             int64_t row0, T *mo, T *co, double cs)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int D = d * S;
    if (e >= (N + 1) * D) return;
    const int64_t n = e / D;
    const int col = (int)(e - n * D), i = col / S, r = col - i * S;
    const double t = Td[r];
    mo[e] = (T)(t * traj[((int64_t)i * (N + 1) + n) * S + r]);
    if (co) {
        const T *pr = packed + (row0 + (int64_t)i * (N + 1) + n) * (S * (S + 1) / 2) + r * (r + 1) / 2;
        T *out = co + e * D;
        for (int c = 0; c < D; ++c) {
            const int j = c / S, cc = c - j * S;
            out[c] = (j == i && cc <= r) ? (T)(cs * t * (double)pr[cc]) : T(0);
        }
    }
}

// Objective value (eq. objective-value) of every request's resident
// trajectory, in the preconditioned coordinates it is kept in, where the
// weighted norm needs no scaling:
//   |eta_n - Phi eta_{n-1}|^2_{Q^-1} = |sqrtQbar^-1 (etabar_n - Phibar etabar_{n-1})|^2,
// halved and summed over n = 1..N into counter word `slot` of the request
// (FP64).  One thread per pack row; a wavefront whose rows all belong to one
// request adds its sum with one atomic.
template <int D>
__global__ __launch_bounds__(256) void k_objective(Pack pk, const double *Phi, const double *sQ, int slot, int rpb)
{
    __shared__ double sPhi[D * D], sL[D * D], sInv[D], wsum[4];
    __shared__ unsigned long long *wdst[4];
    __shared__ int rbase;
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
        sPhi[i] = Phi[i];
        sL[i] = sQ[i];
    }
    if (threadIdx.x < D) sInv[threadIdx.x] = 1.0 / sQ[threadIdx.x * (D + 1)];
    // the block takes rows [r0b, r0b + rpb); the request of its first row by
    // bisection (one thread), then each row walks forward from the previous
    // one (rows are ordered by request)
    const int64_t r0b = (int64_t)blockIdx.x * rpb;
    if (threadIdx.x == 0) {
        int lo = 0, hi = pk.nreq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pk.reqs[mid].row <= r0b)
                lo = mid;
            else
                hi = mid - 1;
        }
        rbase = lo;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int ri = rbase;
    // per wavefront: a running sum for one counter slot, added to memory when
    // the slot changes (requests sharing a slot accumulate together)
    double acc = 0.0;
    unsigned long long *accdst = nullptr;
    for (int64_t base = r0b; base < r0b + rpb; base += blockDim.x) {
        const int64_t r = base + threadIdx.x;
        double v = 0.0;
        unsigned long long *dst = nullptr;
        if (r < pk.rows) {
            while (ri + 1 < pk.nreq && pk.reqs[ri + 1].row <= r) ++ri;
            const ReqDev &q = pk.reqs[ri];
            dst = q.dbits;
            const int64_t n = r - q.row;
            if (n >= 1 && q.traj) {
                const double *a = q.traj + (n - 1) * D, *b = q.traj + n * D;
                double w[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double u = b[i];
#pragma unroll
                    for (int k = 0; k < D; ++k) u -= sPhi[i * D + k] * a[k];
#pragma unroll
                    for (int j = 0; j < i; ++j) u -= sL[i * D + j] * w[j];
                    w[i] = u * sInv[i];
                    v += w[i] * w[i];
                }
                v *= 0.5;
            }
        }
        const unsigned long long *d0 = (const unsigned long long *)__shfl((long long)(uintptr_t)dst, 0);
        if (__all(dst == d0)) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
            if (dst != accdst) {
                if (lane == 0 && accdst) atomicAdd((double *)accdst + slot, acc);
                acc = 0.0;
                accdst = dst;
            }
            acc += v;
        } else if (dst) {
            atomicAdd((double *)dst + slot, v);  // a wavefront across a slot boundary
        }
    }
    if (lane == 0) {
        wsum[wv] = acc;
        wdst[wv] = accdst;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        unsigned long long *cur = nullptr;
        double t = 0.0;
        for (int k = 0; k <= nw; ++k) {
            unsigned long long *dk = k < nw ? wdst[k] : nullptr;
            if (dk != cur) {
                if (cur) atomicAdd((double *)cur + slot, t);
                cur = dk;
                t = 0.0;
            }
            if (dk) t += wsum[k];
        }
    }
}

// zero n 64-bit words (a kernel, so that it may be captured in a graph)
static __global__ void k_zero_u64(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// canonical lower-triangular factor of a D x D square root (one group)
template <class C>
__global__ __launch_bounds__(C::R) void k_tria_square(const typename C::T *full, typename C::T *out)
{
    PARAPN_GROUP_SETUP(C);
    if (grp != 0) return;
    constexpr int D = C::D;
    T v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = lane < D ? full[lane * D + c] : T(0);
    tria_rows_g<T, D, D, C::R, C::SAFE>(v, lane, sh + C::TR);
    if (lane < D)
#pragma unroll
        for (int c = 0; c < D; ++c) out[lane * D + c] = v[c];
}

// ---------------------------------------------------------------------------
// dispatch over the instantiated (d, q) configurations
// ---------------------------------------------------------------------------
template <typename T, class F>
static hipError_t dispatch_t(int d, int q, F &&f)
{
    switch (d * 10 + q) {
    case 11: return f(Cfg<T, 1, 1>{});
    case 12: return f(Cfg<T, 1, 2>{});
    case 13: return f(Cfg<T, 1, 3>{});
    case 14: return f(Cfg<T, 1, 4>{});
    case 21: return f(Cfg<T, 2, 1>{});
    case 22: return f(Cfg<T, 2, 2>{});
    case 23: return f(Cfg<T, 2, 3>{});
    case 24: return f(Cfg<T, 2, 4>{});
    case 31: return f(Cfg<T, 3, 1>{});
    case 32: return f(Cfg<T, 3, 2>{});
    case 33: return f(Cfg<T, 3, 3>{});
    case 34: return f(Cfg<T, 3, 4>{});
    }
    return hipErrorInvalidValue;
}

// damped packs: instantiated in translation units of their own (they build in
// parallel with the rest)
template <typename T>
hipError_t launch_forward_lm_t(int d, int q, const Pack &pk, const ModelDev &m, const Work &w, hipStream_t s)
{
    return dispatch_t<T>(d, q, [&](auto c) {
        using C = decltype(c);
        return fwd_seq<Cfg<T, C::d, C::q, 0, true>>(pk, m, w, s);
    });
}

template <typename T>
hipError_t launch_forward_t(int d, int q, const Pack &pk, const ModelDev &m, const Work &w, hipStream_t s)
{
    if (pk.lm) return launch_forward_lm_t<T>(d, q, pk, m, w, s);
    return dispatch_t<T>(d, q, [&](auto c) { return fwd_seq<decltype(c)>(pk, m, w, s); });
}

template <typename T>
hipError_t launch_smoother_t(int d, int q, const Pack &pk, const ModelDev &m, const Work &w, bool with_cov,
                             bool update, void *mean_out, hipStream_t s)
{
    return dispatch_t<T>(d, q, [&](auto c) {
        using C = decltype(c);
        return with_cov ? bwd_seq<C, true>(pk, m, w, update, mean_out, s)
                        : bwd_seq<C, false>(pk, m, w, update, mean_out, s);
    });
}

template <typename T>
hipError_t launch_filter_combine_t(int d, int q, int64_t count, const void *a, const void *c, void *out,
                                   hipStream_t s)
{
    return dispatch_t<T>(d, q, [&](auto cfg) {
        using C = decltype(cfg);
        hipLaunchKernelGGL(k_filter_combine_batch<C>, dim3((unsigned)cdiv(count, C::GPB)), dim3(C::NT), 0, s,
                           (const T *)a, (const T *)c, (T *)out, count);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_tria_square_t(int d, int q, const void *full, void *out, hipStream_t s)
{
    return dispatch_t<T>(d, q, [&](auto cfg) {
        using C = decltype(cfg);
        hipLaunchKernelGGL(k_tria_square<C>, dim3(1), dim3(C::R), 0, s, (const T *)full, (T *)out);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_coarse_t(int d, int q, const ReqDev *reqs, const CoarseDev *cds, int nreq, int64_t maxN,
                           const void *Phi, const void *Q, hipStream_t s)
{
    if (nreq < 1 || nreq > 65535 || maxN < 1) return hipErrorInvalidValue;
    // the coarse smoother runs in FP64 for either path precision
    hipError_t e = dispatch_t<double>(d, q, [&](auto cfg) {
        using C = decltype(cfg);
        PARAPN_LAUNCH("coarse_eks", s, (k_coarse_eks<C::d, C::q>), dim3((unsigned)nreq), dim3(64), 0, s, reqs, cds,
                      (const double *)Phi, (const double *)Q);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    PARAPN_LAUNCH("coarse_bridge", s, k_coarse_bridge, dim3((unsigned)cdiv(maxN + 1, 256), (unsigned)nreq), dim3(256),
                  0, s, reqs, cds, d, q);
    return hipGetLastError();
}

#ifndef PARAPN_BUILD_FP32
#define PARAPN_BUILD_FP32 1
#endif
#ifndef PARAPN_BUILD_FP64
#define PARAPN_BUILD_FP64 1
#endif
#ifndef PARAPN_BUILD_HELPERS
#define PARAPN_BUILD_HELPERS 1
#endif
// 0: every launcher but the damped forward scan; 1: only the damped one
#ifndef PARAPN_BUILD_LM
#define PARAPN_BUILD_LM 0
#endif

#define PARAPN_INSTANTIATE(T)                                                                                       \
    template hipError_t launch_forward_t<T>(int, int, const Pack &, const ModelDev &, const Work &, hipStream_t);  \
    template hipError_t launch_smoother_t<T>(int, int, const Pack &, const ModelDev &, const Work &, bool, bool,    \
                                             void *, hipStream_t);                                                 \
    template hipError_t launch_filter_combine_t<T>(int, int, int64_t, const void *, const void *, void *,          \
                                                   hipStream_t);                                                   \
    template hipError_t launch_tria_square_t<T>(int, int, const void *, void *, hipStream_t);                     \
    template hipError_t launch_coarse_t<T>(int, int, const ReqDev *, const CoarseDev *, int, int64_t, const void *, \
                                           const void *, hipStream_t);

#define PARAPN_INSTANTIATE_LM(T) \
    template hipError_t launch_forward_lm_t<T>(int, int, const Pack &, const ModelDev &, const Work &, hipStream_t);

#if PARAPN_BUILD_LM
#if PARAPN_BUILD_FP32
PARAPN_INSTANTIATE_LM(float)
#endif
#if PARAPN_BUILD_FP64
PARAPN_INSTANTIATE_LM(double)
#endif
#else
// the damped launchers come from the other translation units
#if PARAPN_BUILD_FP32
extern template hipError_t launch_forward_lm_t<float>(int, int, const Pack &, const ModelDev &, const Work &,
                                                      hipStream_t);
#endif
#if PARAPN_BUILD_FP64
extern template hipError_t launch_forward_lm_t<double>(int, int, const Pack &, const ModelDev &, const Work &,
                                                       hipStream_t);
#endif
#if PARAPN_BUILD_FP32
PARAPN_INSTANTIATE(float)
#endif
#if PARAPN_BUILD_FP64
PARAPN_INSTANTIATE(double)
#endif
#endif

#if PARAPN_BUILD_HELPERS
namespace {
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
struct ProfAcc {
    std::string name;
    double ms;
    int64_t n;
};
bool g_prof_on = false;
std::string g_prof_only;  // empty: every kernel
std::vector<ProfRec> g_prof_pending;
std::vector<ProfAcc> g_prof_acc;
std::vector<hipEvent_t> g_prof_free;  // recorded-and-read events, reused

hipEvent_t prof_event()
{
    if (!g_prof_free.empty()) {
        hipEvent_t e = g_prof_free.back();
        g_prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_resolve()
{
    for (auto &r : g_prof_pending) {
        hipEventSynchronize(r.b);
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        g_prof_free.push_back(r.a);
        g_prof_free.push_back(r.b);
        bool found = false;
        for (auto &a : g_prof_acc)
            if (a.name == r.name) {
                a.ms += ms;
                a.n += 1;
                found = true;
            }
        if (!found) g_prof_acc.push_back({r.name, (double)ms, 1});
    }
    g_prof_pending.clear();
}
}  // namespace

bool prof_on() { return g_prof_on; }

void prof_only(const char *name) { g_prof_only = name ? name : ""; }

void prof_enable(bool on)
{
    g_prof_on = on;
    prof_resolve();
    g_prof_acc.clear();
}

void prof_begin(const char *name, hipStream_t s, hipEvent_t *start)
{
    if (!g_prof_only.empty() && g_prof_only != name) {
        *start = nullptr;
        return;
    }
    *start = prof_event();
    if (*start) hipEventRecord(*start, s);
}

void prof_end(const char *name, hipStream_t s, hipEvent_t start)
{
    if (!start) return;
    hipEvent_t stop = prof_event();
    if (!stop) {
        g_prof_free.push_back(start);
        return;
    }
    hipEventRecord(stop, s);
    g_prof_pending.push_back({name, start, stop});
    // bound the number of events in flight: resolve once many are pending
    if (g_prof_pending.size() >= 4096) prof_resolve();
}

int prof_read(int max, char *names, int name_len, double *total_ms, int64_t *launches)
{
    prof_resolve();
    int k = 0;
    for (auto &a : g_prof_acc) {
        if (k >= max) break;
        std::snprintf(names + (size_t)k * name_len, name_len, "%s", a.name.c_str());
        total_ms[k] = a.ms;
        launches[k] = a.n;
        ++k;
    }
    return (int)g_prof_acc.size();
}

int config_supported(int d, int q) { return (d >= 1 && d <= 3 && q >= 1 && q <= 4) ? 1 : -1; }

int forward_chunk(int64_t N)
{
    // long enough that the step-level aggregates (folded with the cheaper
    // single-element operator) leave little work for the upper levels, short
    // enough that about 8192 groups keep every SIMD busy
    int b1 = 4;
    while (b1 < 32 && N / (2 * b1) >= 8192) b1 *= 2;
    return b1;
}

template <typename T>
static int tree_width_t(int d, int q)
{
    switch (d * 10 + q) {
    case 11: return Cfg<T, 1, 1>::W;
    case 12: return Cfg<T, 1, 2>::W;
    case 13: return Cfg<T, 1, 3>::W;
    case 14: return Cfg<T, 1, 4>::W;
    case 21: return Cfg<T, 2, 1>::W;
    case 22: return Cfg<T, 2, 2>::W;
    case 23: return Cfg<T, 2, 3>::W;
    case 24: return Cfg<T, 2, 4>::W;
    case 31: return Cfg<T, 3, 1>::W;
    case 32: return Cfg<T, 3, 2>::W;
    case 33: return Cfg<T, 3, 3>::W;
    case 34: return Cfg<T, 3, 4>::W;
    }
    return -1;
}

int pack_layout(int fp64, int d, int q, ReqDev *reqs, ScanTab *ftab, ScanTab *stab, int nreq, Pack *pk)
{
    const int W = fp64 ? tree_width_t<double>(d, q) : tree_width_t<float>(d, q);
    constexpr int BS = Cfg<float, 1, 1>::B1;
    if (W < 2 || nreq < 1 || pk->bu < 2 || pk->btop < 1) return -1;
    int64_t f = 0, sm = 0, r = 0, fr = 0, fpr = 0, sr = 0;
    pk->Lf = pk->Ls = 0;
    for (int l = 0; l <= kMaxLevels; ++l) pk->fblocks[l] = pk->sgroups[l] = 0;
    for (int i = 0; i < nreq; ++i) {
        ReqDev &rq = reqs[i];
        if (rq.N < 1) return -1;
        // a caller may preset the chunk length (a function of its own
        // problem only, so results stay independent of the pack)
        if (rq.b1 < 1 || rq.b1 > 32) rq.b1 = forward_chunk(rq.N);
        rq.fchunk = f;
        rq.schunk = sm;
        rq.row = r;
        const int64_t n1f = cdiv(rq.N, rq.b1), n1s = cdiv(rq.N + 1, BS);
        const TreeLevels tl = make_tree_levels(n1f, W);
        const Levels sl = make_levels(n1s, pk->bu, pk->btop);
        if (tl.L > kMaxLevels || sl.L > kMaxLevels) return -1;
        ScanTab &a = ftab[i];
        std::memset(&a, 0, sizeof(a));
        a.L = tl.L;
        a.base = fr;
        a.pbase = fpr;
        for (int l = 1; l <= tl.L; ++l) {
            a.n[l] = (int32_t)tl.n[l];
            a.off[l] = (int32_t)tl.off[l];
            a.poff[l] = (int32_t)tl.poff[l];
        }
        for (int l = 1; l <= kMaxLevels; ++l) {
            a.first[l] = (int32_t)pk->fblocks[l];
            if (l < tl.L) pk->fblocks[l] += tl.n[l + 1];
        }
        ScanTab &b = stab[i];
        std::memset(&b, 0, sizeof(b));
        b.L = sl.L;
        b.base = sr;
        for (int l = 1; l <= sl.L; ++l) {
            b.n[l] = (int32_t)sl.n[l];
            b.off[l] = (int32_t)sl.off[l];
        }
        for (int l = 1; l <= kMaxLevels; ++l) {
            b.first[l] = (int32_t)pk->sgroups[l];
            if (l < sl.L) pk->sgroups[l] += sl.n[l + 1];
        }
        fr += tl.total;
        fpr += tl.ptotal;
        sr += sl.total;
        pk->Lf = std::max(pk->Lf, tl.L);
        pk->Ls = std::max(pk->Ls, sl.L);
        f += n1f;
        sm += n1s;
        r += rq.N + 1;
    }
    pk->nreq = nreq;
    pk->nf = f;
    pk->ns = sm;
    pk->rows = r;
    pk->frecs = fr;
    pk->fprecs = fpr;
    pk->srecs = sr;
    return 0;
}

hipError_t launch_unscale(int fp64, int D, int64_t N, const double *Tdiag_dev, const void *src_mean,
                          const void *src_packed, void *mean_out, void *cov_out, hipStream_t s, bool src_fp64,
                          double cov_scale)
{
    const int64_t rows = (N + 1) * D;
    const unsigned blocks = (unsigned)cdiv(rows, 256);
    if (fp64)
        hipLaunchKernelGGL((k_unscale<double, double>), dim3(blocks), dim3(256), 0, s, D, N, Tdiag_dev,
                           (const double *)src_mean, (const double *)src_packed, (double *)mean_out,
                           (double *)cov_out, cov_scale);
    else if (src_fp64)
        hipLaunchKernelGGL((k_unscale<float, double>), dim3(blocks), dim3(256), 0, s, D, N, Tdiag_dev,
                           (const double *)src_mean, (const float *)src_packed, (float *)mean_out, (float *)cov_out, cov_scale);
    else
        hipLaunchKernelGGL((k_unscale<float, float>), dim3(blocks), dim3(256), 0, s, D, N, Tdiag_dev,
                           (const float *)src_mean, (const float *)src_packed, (float *)mean_out, (float *)cov_out, cov_scale);
    return hipGetLastError();
}

hipError_t launch_objective(int d, int q, const Pack &pk, const double *Phi, const double *sQ, int slot, hipStream_t s)
{
    if (pk.rows < 1) return hipSuccess;
    return dispatch_t<double>(d, q, [&](auto cfg) {
        using C = decltype(cfg);
        // about 2048 blocks, each a whole number of 256-row passes
        const int64_t rpb = 256 * cdiv(cdiv(pk.rows, 2048), 256);
        PARAPN_LAUNCH("objective", s, k_objective<C::D>, dim3((unsigned)cdiv(pk.rows, rpb)), dim3(256), 0, s, pk, Phi,
                      sQ, slot, (int)rpb);
        return hipGetLastError();
    });
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_pad_rows(int fp64, int D, int64_t N, const void *src, void *dst, hipStream_t s)
{
    const unsigned blocks = (unsigned)cdiv(N * D * (D + 1), 256);
    if (fp64)
        hipLaunchKernelGGL(k_pad_rows<double>, dim3(blocks), dim3(256), 0, s, D, N, (const double *)src,
                           (double *)dst);
    else
        hipLaunchKernelGGL(k_pad_rows<float>, dim3(blocks), dim3(256), 0, s, D, N, (const float *)src, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_blocks_in(int B, int d, int S, int64_t N, const double *init, const double *Td, const double *mu0b,
                            double *traj, hipStream_t s)
{
    const int64_t total = (int64_t)B * d * (N + 1) * S;
    hipLaunchKernelGGL(k_blocks_in, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, B, d, S, N, init, Td, mu0b,
                       traj);
    return hipGetLastError();
}

hipError_t launch_blocks_out(int fp64, int d, int S, int64_t N, const double *Td, const double *traj,
                             const void *packed, int64_t row0, void *mean_out, void *cov_out, double cov_scale,
                             hipStream_t s)
{
    const unsigned blocks = (unsigned)cdiv((N + 1) * d * S, 256);
    if (fp64)
        hipLaunchKernelGGL(k_blocks_out<double>, dim3(blocks), dim3(256), 0, s, d, S, N, Td, traj,
                           (const double *)packed, row0, (double *)mean_out, (double *)cov_out, cov_scale);
    else
        hipLaunchKernelGGL(k_blocks_out<float>, dim3(blocks), dim3(256), 0, s, d, S, N, Td, traj,
                           (const float *)packed, row0, (float *)mean_out, (float *)cov_out, cov_scale);
    return hipGetLastError();
}

hipError_t launch_init_traj(int D, int64_t N, const double *init, const double *Td, double *traj, hipStream_t s)
{
    const unsigned blocks = (unsigned)cdiv((N + 1) * D, 256);
    hipLaunchKernelGGL(k_init_traj<double>, dim3(blocks), dim3(256), 0, s, D, N, init, Td, traj);
    return hipGetLastError();
}
#endif

}  // namespace parapn
