// C ABI of the parallel-in-time probabilistic ODE solver (include/parapn.h):
// argument checking, the FP64 host part of the prior (Sec. 2.1, Sec. 2.4)
// and of the exact initialisation (eq. mu0), workspace management, and the
// iteration loop of Alg. 2 around the device scans.
#include "parapn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dense.h"
#include "fields.h"
#include "parapn_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PARAPN_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define PARAPN_HIP(call, what)                     \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ---------------------------------------------------------------------------
// truncated Taylor series (degree <= 4) for Taylor-mode initialisation
// ---------------------------------------------------------------------------
struct Ser {
    double c[5];
};
Ser ser_const(double v)
{
    Ser s{};
    s.c[0] = v;
    return s;
}
Ser operator+(const Ser &a, const Ser &b)
{
    Ser r;
    for (int i = 0; i < 5; ++i) r.c[i] = a.c[i] + b.c[i];
    return r;
}
Ser operator-(const Ser &a, const Ser &b)
{
    Ser r;
    for (int i = 0; i < 5; ++i) r.c[i] = a.c[i] - b.c[i];
    return r;
}
Ser operator*(const Ser &a, const Ser &b)
{
    Ser r{};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; i + j < 5; ++j) r.c[i + j] += a.c[i] * b.c[j];
    return r;
}
Ser operator+(const Ser &a, double s) { return a + ser_const(s); }
Ser operator+(double s, const Ser &a) { return a + ser_const(s); }
Ser operator-(const Ser &a, double s) { return a - ser_const(s); }
Ser operator-(double s, const Ser &a) { return ser_const(s) - a; }
Ser operator*(const Ser &a, double s)
{
    Ser r;
    for (int i = 0; i < 5; ++i) r.c[i] = a.c[i] * s;
    return r;
}
Ser operator*(double s, const Ser &a) { return a * s; }

template <int d>
bool taylor_mu0_d(int field, const double *p, const double *y0, int q, double *mu0)
{
    Ser y[d], f[d];
    for (int i = 0; i < d; ++i) y[i] = ser_const(y0[i]);
    // coefficient k of f(y(t)) depends on the coefficients 0..k of y only
    for (int k = 0; k < q; ++k) {
        if (!parapn::field_eval<d>(field, p, y, f)) return false;
        for (int i = 0; i < d; ++i) y[i].c[k + 1] = f[i].c[k] / (k + 1);
    }
    for (int i = 0; i < d; ++i) {
        double fact = 1.0;
        for (int j = 0; j <= q; ++j) {
            if (j > 0) fact *= j;
            mu0[i * (q + 1) + j] = fact * y[i].c[j];
        }
    }
    return true;
}

// the method-of-lines field (any d >= 3): periodic second differences with
// dx = 1/d plus the logistic reaction, on truncated series
bool taylor_mu0_mol(int d, const double *p, const double *y0, int q, double *mu0)
{
    std::vector<Ser> y(d), f(d);
    const double k = p[0] * (double)d * (double)d;
    for (int i = 0; i < d; ++i) y[i] = ser_const(y0[i]);
    for (int kk = 0; kk < q; ++kk) {
        for (int i = 0; i < d; ++i)
            f[i] = k * (y[(i + d - 1) % d] - 2.0 * y[i] + y[(i + 1) % d]) + y[i] * (1.0 - y[i]);
        for (int i = 0; i < d; ++i) y[i].c[kk + 1] = f[i].c[kk] / (kk + 1);
    }
    for (int i = 0; i < d; ++i) {
        double fact = 1.0;
        for (int j = 0; j <= q; ++j) {
            if (j > 0) fact *= j;
            mu0[i * (q + 1) + j] = fact * y[i].c[j];
        }
    }
    return true;
}

bool taylor_mu0(int field, int d, const double *p, const double *y0, int q, double *mu0)
{
    if (field == parapn::F_MOL) return d >= 3 && taylor_mu0_mol(d, p, y0, q, mu0);
    switch (d) {
    case 1: return taylor_mu0_d<1>(field, p, y0, q, mu0);
    case 2: return taylor_mu0_d<2>(field, p, y0, q, mu0);
    case 3: return taylor_mu0_d<3>(field, p, y0, q, mu0);
    }
    return false;
}

// ---------------------------------------------------------------------------
// preconditioned IWP(q) prior: with T = sqrt(h) diag(h^{q-i}/(q-i)!) the
// transition T^{-1} Phi(h) T has entries binom(q-i, j-i) (j >= i) and the
// process noise T^{-1} Q(h) T^{-T} has entries 1/(2q+1-i-j); neither depends
// on h.  Full-state matrices are I_d (x) block.
// ---------------------------------------------------------------------------
double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

void prior_blocks(int d, int q, std::vector<double> &Phi, std::vector<double> &sQ)
{
    const int S = q + 1, D = d * S;
    std::vector<double> Qb(S * S), Lb(S * S, 0.0);
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) Qb[i * S + j] = 1.0 / (2 * q + 1 - i - j);
    // Cholesky of the (flipped) Hilbert block
    for (int j = 0; j < S; ++j) {
        double s = Qb[j * S + j];
        for (int k = 0; k < j; ++k) s -= Lb[j * S + k] * Lb[j * S + k];
        Lb[j * S + j] = std::sqrt(s);
        for (int i = j + 1; i < S; ++i) {
            double t = Qb[i * S + j];
            for (int k = 0; k < j; ++k) t -= Lb[i * S + k] * Lb[j * S + k];
            Lb[i * S + j] = t / Lb[j * S + j];
        }
    }
    Phi.assign(D * D, 0.0);
    sQ.assign(D * D, 0.0);
    for (int b = 0; b < d; ++b)
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) {
                Phi[(b * S + i) * D + b * S + j] = j >= i ? binom(q - i, j - i) : 0.0;
                sQ[(b * S + i) * D + b * S + j] = Lb[i * S + j];
            }
}

void precond_diag(int d, int q, double h, std::vector<double> &T)
{
    const int S = q + 1;
    T.resize(d * S);
    for (int b = 0; b < d; ++b)
        for (int i = 0; i < S; ++i) T[b * S + i] = std::sqrt(h) * std::pow(h, q - i) / fact(q - i);
}

// exp(A) for small n: scaling and squaring of the Taylor series
void expm_small(int n, const std::vector<double> &A, std::vector<double> &E)
{
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += std::fabs(A[i * n + j]);
        nrm = std::max(nrm, r);
    }
    int sq = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = std::ldexp(1.0, -sq);
    std::vector<double> term(n * n, 0.0), nxt(n * n);
    E.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) E[i * n + i] = term[i * n + i] = 1.0;
    for (int k = 1; k <= 24; ++k) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int l = 0; l < n; ++l) t += term[i * n + l] * A[l * n + j];
                nxt[i * n + j] = t * sc / k;
            }
        term.swap(nxt);
        for (int i = 0; i < n * n; ++i) E[i] += term[i];
    }
    for (int r = 0; r < sq; ++r) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int l = 0; l < n; ++l) t += E[i * n + l] * E[l * n + j];
                nxt[i * n + j] = t;
            }
        E.swap(nxt);
    }
}

// Preconditioned blocks of a prior whose q-th derivative has the drift
// dX_q = sum_k c_k X_k dt + dW (the alternative Gauss-Markov priors of
// Sec. 2.1; c = 0 is the integrated Wiener process).  With T as above the
// drift becomes h T^{-1} F T = Fb, Fb[i][i+1] = q - i and last row
// cb[k] = Fb[q][k] = c_k h^{q+1-k} / (q-k)!, and the noise enters as
// e_q e_q^T over unit time, so Van Loan's block exponential
// exp([[-Fb, e_q e_q^T], [0, Fb^T]]) = [[., E12], [0, E22]] gives
// Phibar = E22^T and Qbar = Phibar E12 without cancellation.
void prior_blocks_lti(int d, int q, const double *cb, std::vector<double> &Phi, std::vector<double> &sQ)
{
    const int S = q + 1, D = d * S, M = 2 * S;
    std::vector<double> C(M * M, 0.0), E;
    for (int i = 0; i < q; ++i) {
        C[i * M + i + 1] = -(double)(q - i);
        C[(S + i + 1) * M + S + i] = (double)(q - i);
    }
    for (int k = 0; k <= q; ++k) {
        C[q * M + k] -= cb[k];
        C[(S + k) * M + S + q] += cb[k];
    }
    C[q * M + S + q] = 1.0;
    expm_small(M, C, E);
    std::vector<double> Pb(S * S), Qb(S * S, 0.0), Lb(S * S, 0.0);
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) Pb[i * S + j] = E[(S + j) * M + S + i];
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) {
            double t = 0.0;
            for (int l = 0; l < S; ++l) t += Pb[i * S + l] * E[l * M + S + j];
            Qb[i * S + j] = t;
        }
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < i; ++j) Qb[i * S + j] = Qb[j * S + i] = 0.5 * (Qb[i * S + j] + Qb[j * S + i]);
    for (int j = 0; j < S; ++j) {
        double v = Qb[j * S + j];
        for (int k = 0; k < j; ++k) v -= Lb[j * S + k] * Lb[j * S + k];
        Lb[j * S + j] = std::sqrt(v);
        for (int i = j + 1; i < S; ++i) {
            double t = Qb[i * S + j];
            for (int k = 0; k < j; ++k) t -= Lb[i * S + k] * Lb[j * S + k];
            Lb[i * S + j] = t / Lb[j * S + j];
        }
    }
    Phi.assign(D * D, 0.0);
    sQ.assign(D * D, 0.0);
    for (int b = 0; b < d; ++b)
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) {
                Phi[(b * S + i) * D + b * S + j] = Pb[i * S + j];
                sQ[(b * S + i) * D + b * S + j] = Lb[i * S + j];
            }
}

// IOUP(q, theta): dX_q = -theta X_q dt + dW
void prior_blocks_ioup(int d, int q, double h, double theta, std::vector<double> &Phi, std::vector<double> &sQ)
{
    double cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    cb[q] = -theta * h;
    prior_blocks_lti(d, q, cb, Phi, sQ);
}

// Matern(nu = q + 1/2, length scale ell): drift polynomial (s + lambda)^(q+1),
// lambda = sqrt(2 nu) / ell, so c_k = -binom(q+1, k) lambda^(q+1-k); unit
// diffusion.  In preconditioned form cb[k] = c_k h^{q+1-k} / (q-k)! =
// -binom(q+1, k) (lambda h)^{q+1-k} / (q-k)!.
void prior_blocks_matern(int d, int q, double h, double ell, std::vector<double> &Phi, std::vector<double> &sQ)
{
    const double lh = std::sqrt(2.0 * q + 1.0) / ell * h;
    double cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k <= q; ++k) cb[k] = -binom(q + 1, k) * std::pow(lh, q + 1 - k) / fact(q - k);
    prior_blocks_lti(d, q, cb, Phi, sQ);
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// coarse-grid starting trajectory (remark on other initial state
// trajectories, Sec. 3.2.2): grid rule, bridge weights, device layout
// ---------------------------------------------------------------------------
// default coarse-grid size: max(1024, 64 ceil(log2 N)), at most N
int64_t default_coarse_points(int64_t N)
{
    int lg = 1;
    while ((int64_t(1) << lg) < N) ++lg;
    return std::min<int64_t>(N, std::max<int64_t>(1024, 64 * (int64_t)lg));
}

// s = ceil(N / target) fine steps per coarse step, M = ceil(N / s) coarse steps
void coarse_grid(int64_t N, int64_t target, int64_t &s, int64_t &M)
{
    if (target < 1) target = 1;
    s = std::max<int64_t>(1, (N + target - 1) / target);
    M = (N + s - 1) / s;
}

// Bridge weights.  Given the full states (q derivatives) at both ends of a
// coarse step, the IWP(q) prior's mean in between is the Hermite interpolant
// of degree 2q+1 (it minimises the integral of the squared (q+1)-th
// derivative).  With tau = o/s in [0, 1] and the Hermite basis b_beta on
// [0, 1] for the data p^(j)(0) (beta = j) and p^(j)(1) (beta = S + j):
//   x^(r)(t_k + tau H) = H^-r sum_beta b_beta^(r)(tau) H^j x^(j)_node(beta).
// In preconditioned coordinates (coarse T_c of H on the nodes, fine T_f of
// h on the row) the weight of beta = (node, j) for derivative r is
//   W[o][r][beta] = sqrt(s) s^(q-r) (q-r)!/(q-j)! b_beta^(r)(o/s),
// independent of h.  Layout W[o][r][2S] for o = 0..s-1.
void bridge_weights(int q, int64_t s, std::vector<double> &W)
{
    const int S = q + 1, n = 2 * S;
    // V[beta][a] = d^j/dtau^j tau^a at the node of beta; basis coefficients = V^-1
    std::vector<double> V(n * n, 0.0), X(n * n, 0.0);
    for (int j = 0; j < S; ++j)
        for (int a = 0; a < n; ++a) {
            if (a == j) V[j * n + a] = fact(j);
            if (a >= j) V[(S + j) * n + a] = fact(a) / fact(a - j);
        }
    for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
    // Gauss-Jordan with partial pivoting: V X = I
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(V[r * n + c]) > std::fabs(V[piv * n + c])) piv = r;
        for (int k = 0; k < n; ++k) {
            std::swap(V[c * n + k], V[piv * n + k]);
            std::swap(X[c * n + k], X[piv * n + k]);
        }
        const double dv = V[c * n + c];
        for (int k = 0; k < n; ++k) {
            V[c * n + k] /= dv;
            X[c * n + k] /= dv;
        }
        for (int r = 0; r < n; ++r)
            if (r != c) {
                const double f = V[r * n + c];
                if (f == 0.0) continue;
                for (int k = 0; k < n; ++k) {
                    V[r * n + k] -= f * V[c * n + k];
                    X[r * n + k] -= f * X[c * n + k];
                }
            }
    }
    // X[a][beta]: coefficient of tau^a in b_beta
    W.assign((size_t)s * S * n, 0.0);
    for (int64_t o = 0; o < s; ++o) {
        double *Wo = W.data() + (size_t)o * S * n;
        const double tau = (double)o / (double)s;
        for (int r = 0; r < S; ++r) {
            const double sc_r = std::sqrt((double)s) * std::pow((double)s, q - r) * fact(q - r);
            if (o == 0) {  // the coarse node itself
                Wo[r * n + r] = sc_r / fact(q - r);
                continue;
            }
            for (int beta = 0; beta < n; ++beta) {
                const int j = beta % S;
                double bv = 0.0;
                for (int a = n - 1; a >= r; --a) bv = bv * tau + X[a * n + beta] * fact(a) / fact(a - r);
                Wo[r * n + beta] = sc_r / fact(q - j) * bv;
            }
        }
    }
}


// Byte offsets of one pack's scratch inside the context workspace.
struct PackLayout {
    size_t se, sL, sPs, mf, sPf, fagg, fpart, fpref, sagg, spref, consts, consts64, reqs, ftab, stab, dbits, extra,
        total;
};

PackLayout pack_scratch_layout(int D, int esz, const parapn::Pack &pk, int nreq, bool cov, size_t extra_bytes)
{
    const size_t DP = (size_t)D * (D + 1) / 2;
    const size_t FEF = (size_t)3 * D * D + 2 * D + 1, FS = (size_t)D + D * D, SAF = (size_t)2 * D * D + D + 1;
    PackLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    L.se = take((size_t)pk.rows * (D * D + 2 * D + 1) * esz);
    L.sL = take((size_t)pk.rows * DP * esz);
    L.sPs = cov ? take((size_t)pk.rows * DP * esz) : 0;
    L.mf = take((size_t)pk.rows * D * esz);
    L.sPf = take((size_t)pk.rows * DP * esz);
    L.fagg = take((size_t)pk.frecs * FEF * esz);
    L.fpart = take((size_t)pk.fprecs * FEF * esz);
    L.fpref = take((size_t)pk.frecs * FS * esz);
    L.sagg = take((size_t)pk.srecs * SAF * esz);
    L.spref = take((size_t)pk.srecs * FS * esz);
    L.consts = take((size_t)(3 * D * D + D) * esz);
    L.consts64 = take((size_t)2 * D * D * 8);  // FP64 Phi, sqrtQ (the objective value)
    L.reqs = take((size_t)nreq * sizeof(parapn::ReqDev));
    L.ftab = take((size_t)nreq * sizeof(parapn::ScanTab));
    L.stab = take((size_t)nreq * sizeof(parapn::ScanTab));
    L.dbits = take((size_t)nreq * parapn::kCounters * sizeof(unsigned long long));
    L.extra = take(extra_bytes);
    L.total = o;
    return L;
}

// One pack ready to run: device-table images (in the byte layout of the
// workspace region from L.reqs to L.dbits), pack totals and scratch layout.
struct PackPlan {
    std::vector<parapn::ReqDev> reqs;
    std::vector<parapn::ScanTab> ftab, stab;
    std::vector<unsigned char> image;
    parapn::Pack pk;
    PackLayout L;
};

// reqs: N, field, scales and trajectory of each request
int plan_pack(int fp64, int d, int q, const std::vector<parapn::ReqDev> &reqs, bool cov, size_t extra,
              PackPlan &pl, bool lm = false)
{
    const int nreq = (int)reqs.size();
    const int D = d * (q + 1), esz = fp64 ? 8 : 4;
    pl.reqs = reqs;
    pl.ftab.assign(nreq, parapn::ScanTab{});
    pl.stab.assign(nreq, parapn::ScanTab{});
    pl.pk = parapn::Pack{};
    pl.pk.bu = 8;
    pl.pk.btop = 16;
    pl.pk.lm = lm ? 1 : 0;
    if (parapn::pack_layout(fp64, d, q, pl.reqs.data(), pl.ftab.data(), pl.stab.data(), nreq, &pl.pk) != 0)
        return fail(PARAPN_EINVAL, "problem too long for the scan levels of this build");
    pl.L = pack_scratch_layout(D, esz, pl.pk, nreq, cov, extra);
    return PARAPN_OK;
}

// Fill the device pointers of the plan for a workspace at ws and build the
// image of its tables.
// group > 1: requests i share the counter slot i / group.
void bind_plan(PackPlan &pl, char *ws, int group = 1)
{
    const int nreq = (int)pl.reqs.size();
    unsigned long long *dbits = (unsigned long long *)(ws + pl.L.dbits);
    for (int i = 0; i < nreq; ++i) pl.reqs[i].dbits = dbits + parapn::kCounters * (i / group);
    pl.pk.reqs = (const parapn::ReqDev *)(ws + pl.L.reqs);
    pl.pk.ftab = (const parapn::ScanTab *)(ws + pl.L.ftab);
    pl.pk.stab = (const parapn::ScanTab *)(ws + pl.L.stab);
    pl.image.assign(pl.L.dbits - pl.L.reqs, 0);
    std::memcpy(pl.image.data(), pl.reqs.data(), nreq * sizeof(parapn::ReqDev));
    std::memcpy(pl.image.data() + (pl.L.ftab - pl.L.reqs), pl.ftab.data(), nreq * sizeof(parapn::ScanTab));
    std::memcpy(pl.image.data() + (pl.L.stab - pl.L.reqs), pl.stab.data(), nreq * sizeof(parapn::ScanTab));
}

// Host-side description of one IVP being solved (Alg. 2).
struct Solve {
    int field, d, q, D, precision;
    int64_t N;
    double t0, t1, h, tol;
    double lm_sigma, lm_s;  // damping (0: none) and its preconditioned per-step std
    int prior;              // PARAPN_PRIOR_*
    double theta;           // IOUP rate or Matern length scale
    int max_iter, fixed_iters;
    int init_mode;          // PARAPN_INIT_*
    int64_t coarse_target;  // coarse-grid size target (init_mode COARSE)
    int start = PARAPN_START_CONSTANT;
    int stop_rule;          // bit 0 trajectory change, bit 1 objective change
    double obj_atol, obj_rtol;
    int calibrate;
    int lin;                // PARAPN_LIN_*
    double params[PARAPN_MAX_PARAMS];
    std::vector<double> Td, mu0, mu0b;  // preconditioner, mu0, mu0 / T
    // iteration state
    int iter = 0;
    int status = PARAPN_MAXITER;
    bool done = false, converged = false;
    double delta = 0.0, tol_used = 0.0;
    std::vector<double> deltas;
    double sigma2 = NAN;     // quasi-MLE diffusion of the last undamped filter pass
    double objective = NAN;  // V of the current trajectory
    double obj_prev = NAN;   // V before the last pass (the objective rule)
    std::vector<double> objectives;
};

int prepare(const parapn_problem *p, Solve &sv)
{
    sv.field = p->field;
    sv.d = p->d;
    sv.q = p->q;
    sv.D = p->d * (p->q + 1);
    sv.precision = p->precision;
    sv.N = p->N;
    sv.t0 = p->t0;
    sv.t1 = p->t1;
    sv.h = (p->t1 - p->t0) / (double)p->N;
    sv.tol = p->tol;
    sv.max_iter = p->max_iter;
    sv.fixed_iters = p->fixed_iters;
    sv.lm_sigma = p->lm_sigma;
    sv.prior = p->prior;
    sv.theta = p->prior_theta;
    sv.init_mode = p->init_mode;
    sv.coarse_target = p->coarse_points > 0 ? p->coarse_points : default_coarse_points(p->N);
    sv.stop_rule = p->stop_rule == 0 ? 1 : p->stop_rule;
    sv.obj_atol = p->obj_atol;
    sv.obj_rtol = p->obj_rtol;
    sv.calibrate = p->calibrate;
    sv.lin = p->linearization;
    for (int i = 0; i < PARAPN_MAX_PARAMS; ++i) sv.params[i] = i < p->n_params ? p->params[i] : 0.0;
    precond_diag(sv.d, sv.q, sv.h, sv.Td);
    sv.mu0.assign(sv.D, 0.0);
    if (!taylor_mu0(sv.field, sv.d, sv.params, p->y0, sv.q, sv.mu0.data()))
        return fail(PARAPN_EINVAL, "field not available for d");
    sv.lm_s = sv.lm_sigma > 0.0 ? sv.lm_sigma / (std::sqrt(sv.h) * sv.Td[0]) : 0.0;
    sv.mu0b.resize(sv.D);
    for (int k = 0; k < sv.D; ++k) {
        if (!std::isfinite(sv.mu0[k])) return fail(PARAPN_EINVAL, "non-finite initial derivatives");
        sv.mu0b[k] = sv.mu0[k] / sv.Td[k];
    }
    return PARAPN_OK;
}

// the solve's preconditioned prior blocks for d components
void prior_blocks_of(const Solve &sv, int d, std::vector<double> &Phi, std::vector<double> &sQ)
{
    if (sv.prior == PARAPN_PRIOR_IOUP)
        prior_blocks_ioup(d, sv.q, sv.h, sv.theta, Phi, sQ);
    else if (sv.prior == PARAPN_PRIOR_MATERN)
        prior_blocks_matern(d, sv.q, sv.h, sv.theta, Phi, sQ);
    else
        prior_blocks(d, sv.q, Phi, sQ);
}

void fill_reqdev(const Solve &sv, double *traj, unsigned long long *dbits, parapn::ReqDev &r)
{
    std::memset(&r, 0, sizeof(r));
    r.field = sv.field;
    r.lin = sv.lin;
    for (int i = 0; i < PARAPN_MAX_PARAMS; ++i) r.p[i] = sv.params[i];
    r.T0 = sv.Td[0];
    r.T1 = sv.Td[1];
    r.invT1 = 1.0 / sv.Td[1];
    r.hq = sv.h / sv.q;
    r.lm_s = sv.lm_s;
    r.traj = traj;
    r.dbits = dbits;
    r.N = sv.N;
}

// Upload the (precision, d, q) constants: Phi | sqrtQ | initial increment
// state (0, 0) -- the scans run on the increment over a trajectory whose
// row 0 is mu0 itself.
int upload_consts(const Solve &sv, bool fp64, char *dst, char *dst64, hipStream_t s)
{
    const int D = sv.d * (sv.q + 1);
    std::vector<double> Phi, sQ;
    prior_blocks_of(sv, sv.d, Phi, sQ);
    std::vector<double> c64(2 * D * D);
    for (int i = 0; i < D * D; ++i) {
        c64[i] = Phi[i];
        c64[D * D + i] = sQ[i];
    }
    PARAPN_HIP(hipMemcpyAsync(dst64, c64.data(), c64.size() * 8, hipMemcpyHostToDevice, s), "copy FP64 constants");
    std::vector<double> cst(3 * D * D + D, 0.0);
    for (int i = 0; i < D * D; ++i) {
        cst[i] = Phi[i];
        cst[D * D + i] = sQ[i];
    }
    if (fp64) {
        PARAPN_HIP(hipMemcpyAsync(dst, cst.data(), cst.size() * 8, hipMemcpyHostToDevice, s), "copy constants");
    } else {
        std::vector<float> cf(cst.begin(), cst.end());
        PARAPN_HIP(hipMemcpyAsync(dst, cf.data(), cf.size() * 4, hipMemcpyHostToDevice, s), "copy constants");
    }
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    return PARAPN_OK;
}

parapn::ModelDev model_from(char *cdev, int D, int esz)
{
    parapn::ModelDev m;
    m.Phi = cdev;
    m.sQ = cdev + (size_t)D * D * esz;
    m.init = cdev + (size_t)2 * D * D * esz;
    return m;
}

parapn::Work work_from(char *ws, const PackLayout &L, bool cov)
{
    parapn::Work w{};
    w.se = ws + L.se;
    w.sL = ws + L.sL;
    w.sPs = cov ? ws + L.sPs : nullptr;
    w.mf = ws + L.mf;
    w.sPf = ws + L.sPf;
    w.fagg = ws + L.fagg;
    w.fpart = ws + L.fpart;
    w.fpref = ws + L.fpref;
    w.sagg = ws + L.sagg;
    w.spref = ws + L.spref;
    return w;
}

// Device scratch of one request's coarse-grid start (byte offsets from its
// base): smoothed coarse nodes, RTS gains, bridge weights, mu0 in coarse
// coordinates, the status word, the request's tables and the IWP constants.
struct CoarseLayout {
    int64_t s, M;
    size_t node, gain, W, mu0c, status, cd, req, consts, total;
};

CoarseLayout coarse_layout(const Solve &sv)
{
    CoarseLayout c{};
    coarse_grid(sv.N, sv.coarse_target, c.s, c.M);
    const size_t D = sv.D, S = sv.q + 1;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = align_up(o + b);
        return r;
    };
    const size_t d = sv.d;
    c.node = take((size_t)(c.M + 1) * D * 8);
    c.gain = take((size_t)(c.M + 1) * parapn::coarse_record_doubles((int)d, sv.q) * 8);
    c.W = take((size_t)c.s * S * 2 * S * 8);
    c.mu0c = take(D * 8);
    c.status = take(sizeof(int));
    c.cd = take(sizeof(parapn::CoarseDev));
    c.req = take(sizeof(parapn::ReqDev));
    c.consts = take(2 * D * D * 8);
    c.total = o;
    return c;
}

// Run the coarse-grid start of one solve into its resident trajectory (whose
// tail already holds T and mu0/T) and record which start the solve uses.
// Waits for the stream (the host tables are locals; the verdict is read back).
int coarse_start(Solve &sv, bool fp64, char *base, const CoarseLayout &cl, double *traj, hipStream_t s)
{
    const int D = sv.D, S = sv.q + 1;
    std::vector<double> Tc, W, Phi, sQ;
    precond_diag(sv.d, sv.q, (double)cl.s * sv.h, Tc);
    bridge_weights(sv.q, cl.s, W);
    prior_blocks(sv.d, sv.q, Phi, sQ);  // the IWP prior, whatever the solve's prior
    // [Phi | Q]: the preconditioned process-noise covariance has the entries
    // 1/(2q+1-i-j) per component block
    std::vector<double> cst((size_t)2 * D * D, 0.0);
    for (int i = 0; i < D * D; ++i) cst[i] = Phi[i];
    for (int b = 0; b < sv.d; ++b)
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) cst[D * D + (b * S + i) * D + b * S + j] = 1.0 / (2 * sv.q + 1 - i - j);
    std::vector<double> mu0c(D);
    for (int k = 0; k < D; ++k) mu0c[k] = sv.mu0[k] / Tc[k];
    parapn::CoarseDev cd{};
    cd.M = cl.M;
    cd.s = cl.s;
    cd.T0 = Tc[0];
    cd.T1 = Tc[1];
    cd.invT1 = 1.0 / Tc[1];
    cd.hq = (double)cl.s * sv.h / sv.q;
    cd.node = (double *)(base + cl.node);
    cd.gain = base + cl.gain;
    cd.W = (const double *)(base + cl.W);
    cd.mu0c = (const double *)(base + cl.mu0c);
    cd.status = (int *)(base + cl.status);
    parapn::ReqDev rq;
    fill_reqdev(sv, traj, nullptr, rq);
    PARAPN_HIP(hipMemcpyAsync(base + cl.W, W.data(), W.size() * 8, hipMemcpyHostToDevice, s), "copy bridge weights");
    PARAPN_HIP(hipMemcpyAsync(base + cl.mu0c, mu0c.data(), D * 8, hipMemcpyHostToDevice, s), "copy mu0");
    PARAPN_HIP(hipMemcpyAsync(base + cl.cd, &cd, sizeof(cd), hipMemcpyHostToDevice, s), "copy coarse table");
    PARAPN_HIP(hipMemcpyAsync(base + cl.req, &rq, sizeof(rq), hipMemcpyHostToDevice, s), "copy request table");
    PARAPN_HIP(hipMemcpyAsync(base + cl.consts, cst.data(), cst.size() * 8, hipMemcpyHostToDevice, s),
               "copy constants");
    PARAPN_HIP(parapn::launch_coarse(fp64, sv.d, sv.q, (const parapn::ReqDev *)(base + cl.req),
                                     (const parapn::CoarseDev *)(base + cl.cd), 1, sv.N, base + cl.consts,
                                     base + cl.consts + (size_t)D * D * 8, s),
               "coarse start");
    int status = 0;
    PARAPN_HIP(hipMemcpyAsync(&status, base + cl.status, sizeof(int), hipMemcpyDeviceToHost, s), "read status");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    sv.start = status == 0 ? PARAPN_START_COARSE : PARAPN_START_COARSE_FAILED;
    return PARAPN_OK;
}

}  // namespace

struct parapn_ctx {
    int device;
    size_t budget;
    void *ws;
    size_t ws_bytes;
    unsigned long long *host_bits;  // pinned
    size_t host_bits_n;
    // what the workspace already holds: constants and request table of the
    // last pack (skip re-uploading them on the next iteration of that pack)
    const void *consts_at;
    int consts_key;
    const void *reqs_at;
    std::vector<unsigned char> reqs_key;  // bytes of the table last copied
};

static int ensure_ws(parapn_ctx *ctx, size_t bytes)
{
    if (ctx->budget && bytes > ctx->budget)
        return fail(PARAPN_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the context budget");
    if (bytes <= ctx->ws_bytes) return PARAPN_OK;
    if (ctx->ws) {
        PARAPN_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        PARAPN_HIP(hipFree(ctx->ws), "hipFree");
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    ctx->consts_at = nullptr;
    ctx->reqs_at = nullptr;
    hipError_t e = hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return fail(PARAPN_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
    }
    ctx->ws_bytes = bytes;
    return PARAPN_OK;
}

static int ensure_host_bits(parapn_ctx *ctx, size_t n)
{
    if (n <= ctx->host_bits_n) return PARAPN_OK;
    if (ctx->host_bits) hipHostFree(ctx->host_bits);
    ctx->host_bits = nullptr;
    ctx->host_bits_n = 0;
    PARAPN_HIP(hipHostMalloc((void **)&ctx->host_bits, n * sizeof(unsigned long long), hipHostMallocDefault),
               "hipHostMalloc");
    ctx->host_bits_n = n;
    return PARAPN_OK;
}

static int check_problem(const parapn_problem *p, int *q_out, int *D_out)
{
    if (!p) return fail(PARAPN_EINVAL, "problem is NULL");
    int np;
    if (p->field == parapn::F_MOL) {
        // the dense engine
        if (p->q < 1 || p->q > 4) return fail(PARAPN_EINVAL, "q must be in 1..4");
        if (p->d < 3 || p->d * (p->q + 1) > parapn::kDenseMaxD)
            return fail(PARAPN_EINVAL, "the method-of-lines field needs d >= 3 and d(q+1) <= " +
                                           std::to_string(parapn::kDenseMaxD));
        if (p->lm_sigma != 0.0) return fail(PARAPN_EINVAL, "damping (lm_sigma > 0) is not available for this field");
        np = 1;
        if (p->n_params >= 1 && p->params && !(std::isfinite(p->params[0]) && p->params[0] >= 0.0))
            return fail(PARAPN_EINVAL, "nu must be finite and >= 0");
    } else {
        const int fd = parapn::field_fixed_dim(p->field);
        if (fd < 0) return fail(PARAPN_EINVAL, "unknown field id " + std::to_string(p->field));
        if (fd > 0 && p->d != fd) return fail(PARAPN_EINVAL, "field requires d = " + std::to_string(fd));
        if (p->d < 1 || p->d > 3) return fail(PARAPN_EINVAL, "d must be in 1..3 in this build");
        if (p->q < 1 || p->q > 4) return fail(PARAPN_EINVAL, "q must be in 1..4");
        if (parapn::config_supported(p->d, p->q) < 0) return fail(PARAPN_EINVAL, "unsupported (d, q)");
        np = parapn::field_n_params(p->field, p->d);
    }
    if (p->n_params < np || p->n_params > PARAPN_MAX_PARAMS)
        return fail(PARAPN_EINVAL, "field needs " + std::to_string(np) + " parameters");
    if (np > 0 && !p->params) return fail(PARAPN_EINVAL, "params is NULL");
    if (!p->y0) return fail(PARAPN_EINVAL, "y0 is NULL");
    if (p->N < 1) return fail(PARAPN_EINVAL, "N must be >= 1");
    if (!(p->t1 > p->t0) || !std::isfinite(p->t0) || !std::isfinite(p->t1))
        return fail(PARAPN_EINVAL, "need finite t1 > t0");
    if (p->max_iter < 1 && p->fixed_iters < 1) return fail(PARAPN_EINVAL, "max_iter must be >= 1");
    if (p->precision != PARAPN_FP64 && p->precision != PARAPN_FP32_SQRT)
        return fail(PARAPN_EINVAL, "unknown precision");
    if (p->init_on_device != 0 && p->init_on_device != 1) return fail(PARAPN_EINVAL, "init_on_device must be 0 or 1");
    if (!(p->lm_sigma >= 0.0) || !std::isfinite(p->lm_sigma)) return fail(PARAPN_EINVAL, "lm_sigma must be finite and >= 0");
    if (p->prior != PARAPN_PRIOR_IWP && p->prior != PARAPN_PRIOR_IOUP && p->prior != PARAPN_PRIOR_MATERN)
        return fail(PARAPN_EINVAL, "unknown prior");
    if (p->init_mode != PARAPN_INIT_CONSTANT && p->init_mode != PARAPN_INIT_COARSE)
        return fail(PARAPN_EINVAL, "unknown init_mode");
    if (p->coarse_points < 0) return fail(PARAPN_EINVAL, "coarse_points must be >= 0");
    if (p->stop_rule < 0 || p->stop_rule > 3) return fail(PARAPN_EINVAL, "stop_rule must be 0..3");
    if (!(p->obj_atol >= 0.0) || !(p->obj_rtol >= 0.0)) return fail(PARAPN_EINVAL, "objective tolerances must be >= 0");
    if (p->linearization < PARAPN_LIN_EK1 || p->linearization > PARAPN_LIN_DIAG_EK1)
        return fail(PARAPN_EINVAL, "unknown linearization");
    if (p->calibrate != 0 && p->calibrate != 1) return fail(PARAPN_EINVAL, "calibrate must be 0 or 1");
    if (p->field == parapn::F_MOL && p->linearization == PARAPN_LIN_EK1 && p->calibrate)
        return fail(PARAPN_EINVAL, "sigma-hat (calibrate) is formed for the method-of-lines field under EK0 or "
                                   "DiagonalEK1 only");
    if (p->field == parapn::F_MOL && p->init_mode == PARAPN_INIT_COARSE && !p->init_traj)
        return fail(PARAPN_EINVAL, "the coarse-grid start is available for the fixed-size fields");
    if (p->prior == PARAPN_PRIOR_IOUP && !(std::isfinite(p->prior_theta) && p->prior_theta >= 0.0))
        return fail(PARAPN_EINVAL, "prior_theta must be finite and >= 0");
    if (p->prior == PARAPN_PRIOR_MATERN && !(std::isfinite(p->prior_theta) && p->prior_theta > 0.0))
        return fail(PARAPN_EINVAL, "the Matern length scale (prior_theta) must be finite and > 0");
    for (int i = 0; i < p->d; ++i)
        if (!std::isfinite(p->y0[i])) return fail(PARAPN_EINVAL, "y0 is not finite");
    *q_out = p->q;
    *D_out = p->d * (p->q + 1);
    return PARAPN_OK;
}

// One IEKS iteration (linearise, both scans, trajectory update) for a pack
// of solves sharing (precision, d, q), enqueued on s.  trajs[i] are their
// resident FP64 trajectories.  The pack's delta counters are copied
// (asynchronously) to ctx->host_bits[slot .. slot + 2 nreq), which the
// caller has sized.  fixed: a plan the caller already sized the workspace
// for (else the pack is planned here and the workspace grown to fit it).
static int pack_enqueue(parapn_ctx *ctx, std::vector<Solve *> &sv, std::vector<double *> &trajs, hipStream_t s,
                        PackPlan *fixed, size_t slot, bool obj_start = false)
{
    const int nreq = (int)sv.size();
    const Solve &s0 = *sv[0];
    const bool fp64 = s0.precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4, D = s0.D;
    PackPlan local;
    PackPlan *pl = fixed;
    int rc;
    if (!pl) {
        std::vector<parapn::ReqDev> reqs(nreq);
        for (int i = 0; i < nreq; ++i) fill_reqdev(*sv[i], trajs[i], nullptr, reqs[i]);
        rc = plan_pack(fp64, s0.d, s0.q, reqs, false, 0, local, s0.lm_sigma > 0.0);
        if (rc) return rc;
        rc = ensure_ws(ctx, local.L.total);
        if (rc) return rc;
        pl = &local;
    }
    if (slot + parapn::kCounters * (size_t)nreq > ctx->host_bits_n) return fail(PARAPN_EINVAL, "internal: delta slots");
    char *ws = (char *)ctx->ws;
    bind_plan(*pl, ws);
    const PackLayout &L = pl->L;
    // IWP constants depend on (d, q, precision) only and are cached; IOUP
    // ones also on h and theta and are uploaded every time
    const int ckey = (s0.d * 8 + s0.q) * 2 + (fp64 ? 1 : 0);
    const bool cacheable = s0.prior == PARAPN_PRIOR_IWP;
    if (!cacheable || ctx->consts_at != ws + L.consts || ctx->consts_key != ckey) {
        rc = upload_consts(s0, fp64, ws + L.consts, ws + L.consts64, s);
        if (rc) return rc;
        ctx->consts_at = cacheable ? ws + L.consts : nullptr;
        ctx->consts_key = ckey;
    }
    if (ctx->reqs_at != ws + L.reqs || ctx->reqs_key != pl->image) {
        PARAPN_HIP(hipMemcpyAsync(ws + L.reqs, pl->image.data(), pl->image.size(), hipMemcpyHostToDevice, s),
                   "copy request tables");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        ctx->reqs_at = ws + L.reqs;
        ctx->reqs_key = pl->image;
    }
    unsigned long long *dbits = (unsigned long long *)(ws + L.dbits);
    PARAPN_HIP(parapn::launch_zero_u64(dbits, parapn::kCounters * (int64_t)nreq, s), "reset delta slots");
    parapn::Pack pk = pl->pk;
    pk.mode = 0;
    pk.lm = s0.lm_sigma > 0.0 ? 1 : 0;
    const parapn::ModelDev m = model_from(ws + L.consts, D, esz);
    const parapn::Work w = work_from(ws, L, false);
    const double *c64 = (const double *)(ws + L.consts64);
    if (obj_start)
        PARAPN_HIP(parapn::launch_objective(s0.d, s0.q, pk, c64, c64 + D * D, 4, s), "objective of the start");
    PARAPN_HIP(parapn::launch_forward(fp64, s0.d, s0.q, pk, m, w, s), "forward scan");
    PARAPN_HIP(parapn::launch_smoother(fp64, s0.d, s0.q, pk, m, w, false, true, nullptr, s), "reverse scan");
    PARAPN_HIP(parapn::launch_objective(s0.d, s0.q, pk, c64, c64 + D * D, 3, s), "objective");
    PARAPN_HIP(hipMemcpyAsync(ctx->host_bits + slot, dbits, parapn::kCounters * nreq * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s),
               "read delta");
    return PARAPN_OK;
}

// Advance each solve's state from its iteration's counters (stride words per
// request: delta and max |E0 trajectory| as bit patterns; with the row
// engine's kCounters also the innovations' quadratic-form sum, the objective
// after and before the pass, as doubles).  The stopping rule of Sec. 3.2.2:
// the trajectory change below tol, or the objective change below
// obj_atol + obj_rtol |V|, as the solve's stop_rule selects.
static void pack_finish(std::vector<Solve *> &sv, const unsigned long long *bits, int stride = parapn::kCounters)
{
    for (size_t i = 0; i < sv.size(); ++i) {
        Solve &v = *sv[i];
        if (v.done) continue;
        double delta, mmax, qf = NAN, Vend = NAN, Vstart = NAN;
        std::memcpy(&delta, bits + stride * i, 8);
        std::memcpy(&mmax, bits + stride * i + 1, 8);
        if (stride >= 5) {
            std::memcpy(&qf, bits + stride * i + 2, 8);
            std::memcpy(&Vend, bits + stride * i + 3, 8);
            std::memcpy(&Vstart, bits + stride * i + 4, 8);
        }
        if (v.iter == 0) v.obj_prev = Vstart;
        v.iter += 1;
        v.delta = delta;
        v.deltas.push_back(delta);
        // the FP32 filter's quadratic forms are not reported (see the FP64 pass)
        v.sigma2 = (v.lm_sigma > 0.0 || v.precision != PARAPN_FP64) ? NAN : qf / ((double)v.N * v.d);
        v.objective = Vend;
        v.objectives.push_back(Vend);
        const bool obj_stop = (v.stop_rule & 2) && std::fabs(Vend - v.obj_prev) <= v.obj_atol + v.obj_rtol * std::fabs(Vend);
        v.obj_prev = Vend;
        const int limit = v.fixed_iters > 0 ? v.fixed_iters : v.max_iter;
        if (!std::isfinite(delta)) {
            v.status = PARAPN_ENONFINITE;
            v.done = true;
            continue;
        }
        v.tol_used = v.precision == PARAPN_FP64 ? v.tol : std::fmax(v.tol, std::ldexp(mmax, -20));
        if (v.fixed_iters > 0) {
            if (v.iter >= limit) {
                v.status = PARAPN_OK;
                v.done = true;
            }
        } else if (((v.stop_rule & 1) && delta < v.tol_used) || obj_stop) {
            v.status = PARAPN_OK;
            v.converged = true;
            v.done = true;
        } else if (v.iter >= limit) {
            v.status = PARAPN_MAXITER;
            v.done = true;
        }
    }
}

// One iteration with its read-back: every solve's state is current after it.
static int pack_iteration(parapn_ctx *ctx, std::vector<Solve *> &sv, std::vector<double *> &trajs, hipStream_t s,
                          PackPlan *fixed = nullptr)
{
    int rc = ensure_host_bits(ctx, parapn::kCounters * sv.size());
    if (rc) return rc;
    bool obj_start = false;
    for (Solve *v : sv) obj_start |= v->iter == 0 && (v->stop_rule & 2);
    rc = pack_enqueue(ctx, sv, trajs, s, fixed, 0, obj_start);
    if (rc) return rc;
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    pack_finish(sv, ctx->host_bits);
    return PARAPN_OK;
}

// resident per-solve device buffer: trajectory [N+1][D], then T and mu0/T
static size_t resident_bytes(const Solve &sv) { return align_up(((size_t)(sv.N + 1) * sv.D + 2 * sv.D) * 8); }

static int init_resident(const Solve &sv, double *buf, const double *init_traj, bool on_device, hipStream_t s)
{
    const int D = sv.D;
    double *traj = buf, *tail = buf + (size_t)(sv.N + 1) * D;
    std::vector<double> Tmu(2 * D);
    for (int k = 0; k < D; ++k) {
        Tmu[k] = sv.Td[k];
        Tmu[D + k] = sv.mu0b[k];
    }
    PARAPN_HIP(hipMemcpyAsync(tail, Tmu.data(), 2 * D * sizeof(double), hipMemcpyHostToDevice, s), "copy T");
    const double *init = nullptr;
    if (init_traj && on_device) {
        init = init_traj;
    } else if (init_traj) {
        // the caller's host trajectory, preconditioned in place on the device
        PARAPN_HIP(hipMemcpyAsync(traj, init_traj, (size_t)(sv.N + 1) * D * sizeof(double), hipMemcpyHostToDevice, s),
                   "copy traj");
        init = traj;
    }
    // row 0 is always mu0 (only its E0 part enters the convergence test)
    PARAPN_HIP(parapn::launch_init_traj(D, sv.N, init, tail, traj, s), "initial trajectory");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");  // Tmu is a local
    return PARAPN_OK;
}

// ---------------------------------------------------------------------------
// dense engine (method-of-lines field): B instances of one problem
// ---------------------------------------------------------------------------

static int64_t dense_traj_stride(int D, int64_t N) { return ((N + 1) * D + 2 * D + 31) & ~int64_t(31); }

struct DenseLayout {
    size_t traj, dbits, active, A, b, C, e, J, E, g, L, scratch, total;
};

static DenseLayout dense_layout(bool fp64, int D, int64_t N, int B, bool cov)
{
    DenseLayout L{};
    size_t off = 0;
    const size_t esz = fp64 ? 8 : 4, el = (size_t)B * N, DD = (size_t)D * D;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.traj = take((size_t)B * dense_traj_stride(D, N) * 8);
    L.dbits = take((size_t)4 * B * 8);  // delta and max |E0 mu| per instance, then V after and before the pass
    L.active = take((size_t)B * 4);
    L.A = take(el * DD * esz);
    L.C = take(el * DD * esz);
    L.J = take(el * DD * esz);
    L.E = take(el * DD * esz);
    L.b = take(el * D * esz);
    L.e = take(el * D * esz);
    L.g = take(el * D * esz);
    L.L = cov ? take(el * DD * esz) : 0;
    L.scratch = take((size_t)parapn::dense_workgroups(fp64) * parapn::dense_scratch_elems(D) * esz);
    L.total = off;
    return L;
}

// Alg. 2 for instances b = 0..B-1 of problem p with initial values
// y0s + b d.  All instances iterate together; one that has converged (or
// turned non-finite) is frozen: its kernels skip it from then on, so its
// result is the one it would get alone.
static int dense_solve(parapn_ctx *ctx, const parapn_problem *p, int B, const double *y0s, void *mean_out,
                       void *cov_out, parapn_info *info, hipStream_t s)
{
    const bool fp64 = p->precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4;
    std::vector<Solve> sv(B);
    for (int b = 0; b < B; ++b) {
        parapn_problem pb = *p;
        pb.y0 = y0s + (size_t)b * p->d;
        for (int i = 0; i < p->d; ++i)
            if (!std::isfinite(pb.y0[i])) return fail(PARAPN_EINVAL, "y0 is not finite");
        const int rc = prepare(&pb, sv[b]);
        if (rc) return rc;
    }
    const int D = sv[0].D;
    const int64_t N = sv[0].N;
    const DenseLayout L = dense_layout(fp64, D, N, B, cov_out != nullptr);
    int rc = ensure_ws(ctx, L.total);
    if (rc) return rc;
    rc = ensure_host_bits(ctx, 4 * (size_t)B);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    // the dense layout overwrites what the row-per-lane packs cached there
    ctx->consts_at = nullptr;
    ctx->reqs_at = nullptr;
    const int64_t ts = dense_traj_stride(D, N);
    double *traj = (double *)(ws + L.traj);
    for (int b = 0; b < B; ++b) {
        rc = init_resident(sv[b], traj + (size_t)b * ts, p->init_traj, p->init_on_device != 0, s);
        if (rc) return rc;
    }
    parapn::DenseModel md{};
    md.field = p->field;
    md.d = p->d;
    md.q = p->q;
    md.D = D;
    md.B = B;
    md.N = N;
    md.hq = sv[0].h / p->q;
    md.T0 = sv[0].Td[0];
    md.T1 = sv[0].Td[1];
    for (int i = 0; i < parapn::kMaxParams; ++i) md.p[i] = sv[0].params[i];
    {
        std::vector<double> Phi, sQ;
        prior_blocks_of(sv[0], 1, Phi, sQ);
        const int S = p->q + 1;
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) {
                md.phib[i * 5 + j] = Phi[i * S + j];
                md.sqb[i * 5 + j] = sQ[i * S + j];
            }
    }
    parapn::DenseWork w{};
    w.A = ws + L.A;
    w.b = ws + L.b;
    w.C = ws + L.C;
    w.e = ws + L.e;
    w.J = ws + L.J;
    w.E = ws + L.E;
    w.g = ws + L.g;
    w.L = cov_out ? ws + L.L : nullptr;
    w.scratch = ws + L.scratch;
    w.traj = traj;
    w.traj_stride = ts;
    w.dbits = (unsigned long long *)(ws + L.dbits);
    int *active_dev = (int *)(ws + L.active);
    w.active = active_dev;
    w.nwg = parapn::dense_workgroups(fp64);
    std::vector<Solve *> ptr(B);
    for (int b = 0; b < B; ++b) ptr[b] = &sv[b];
    std::vector<int> active(B, 1);
    double *obj = (double *)(w.dbits + 2 * B);
    // counters in pack_finish's layout: delta, max |E0 mu|, no quadratic-form
    // sum (sigma-hat is not formed here), V after and before the pass
    std::vector<unsigned long long> counters((size_t)parapn::kCounters * B);
    const double nan = NAN;
    unsigned long long nan_bits;
    std::memcpy(&nan_bits, &nan, 8);
    while (true) {
        bool obj_start = false;
        for (int b = 0; b < B; ++b) obj_start |= !sv[b].done && sv[b].iter == 0 && (sv[b].stop_rule & 2);
        PARAPN_HIP(hipMemcpyAsync(active_dev, active.data(), (size_t)B * sizeof(int), hipMemcpyHostToDevice, s),
                   "copy flags");
        PARAPN_HIP(parapn::launch_zero_u64(w.dbits, 4 * (int64_t)B, s), "reset counters");
        if (obj_start) PARAPN_HIP(parapn::dense_objective(md, w, obj, 1, s), "objective of the start");
        PARAPN_HIP(parapn::dense_iteration(fp64, md, w, s), "dense iteration");
        PARAPN_HIP(parapn::dense_objective(md, w, obj, 0, s), "objective");
        PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, w.dbits, (size_t)4 * B * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s),
                   "read counters");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        for (int b = 0; b < B; ++b) {
            unsigned long long *c = counters.data() + (size_t)parapn::kCounters * b;
            c[0] = ctx->host_bits[2 * b];
            c[1] = ctx->host_bits[2 * b + 1];
            c[2] = nan_bits;
            c[3] = ctx->host_bits[2 * B + 2 * b];
            c[4] = obj_start ? ctx->host_bits[2 * B + 2 * b + 1] : nan_bits;
        }
        pack_finish(ptr, counters.data(), parapn::kCounters);
        bool all = true;
        for (int b = 0; b < B; ++b) {
            active[b] = sv[b].done ? 0 : 1;
            all = all && sv[b].done;
        }
        if (all) break;
    }
    for (int b = 0; b < B; ++b) {
        const double *tb = traj + (size_t)b * ts;
        PARAPN_HIP(parapn::launch_unscale(fp64, D, N, tb + (size_t)(N + 1) * D, tb, nullptr,
                                          (char *)mean_out + (size_t)b * (N + 1) * D * esz, nullptr, s, true),
                   "unscale");
    }
    if (cov_out) {
        // factors at each instance's last linearisation (its filtering
        // marginals are still in place)
        w.active = nullptr;
        PARAPN_HIP(parapn::dense_covariance(fp64, md, w, cov_out, s), "covariance pass");
    }
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    int status = PARAPN_OK;
    for (int b = 0; b < B; ++b) {
        const Solve &v = sv[b];
        if (info) {
            parapn_info &f = info[b];
            f.iterations = v.iter;
            f.converged = v.converged ? 1 : 0;
            f.final_delta = v.delta;
            f.tol_used = v.tol_used;
            f.start = p->init_traj ? PARAPN_START_GIVEN : PARAPN_START_CONSTANT;
            f.sigma_hat = NAN;  // not computed by the dense engine
            f.objective = v.objective;
            const int cap = std::max(v.max_iter, v.fixed_iters);
            if (f.delta_history)
                for (int k = 0; k < (int)v.deltas.size() && k < cap; ++k) f.delta_history[k] = v.deltas[k];
            if (f.objective_history)
                for (int k = 0; k < (int)v.objectives.size() && k < cap; ++k) f.objective_history[k] = v.objectives[k];
        }
        if (v.status == PARAPN_ENONFINITE)
            status = PARAPN_ENONFINITE;
        else if (v.status == PARAPN_MAXITER && status == PARAPN_OK)
            status = PARAPN_MAXITER;
    }
    if (status == PARAPN_ENONFINITE) g_err = "non-finite values in the iterate";
    return status;
}

// Workspace of the decoupled chains (below): trajectories [B][d][N+1][S],
// T (S values), mu0/T ([B][D]), a staging copy of a host init_traj, the pack
// scratch for all instances and (calibrated FP32 with factors) an FP64
// pack's.
struct DecoupledLayout {
    size_t T, mu, stage, pack, pack64, total;
};

static int decoupled_layout(const parapn_problem *p, int B, bool want_cov, DecoupledLayout &DL)
{
    const bool fp64 = p->precision == PARAPN_FP64;
    const int d = p->d, S = p->q + 1, D = d * S;
    const int64_t N = p->N;
    DL.T = align_up((size_t)B * d * (N + 1) * S * 8);
    DL.mu = DL.T + align_up((size_t)S * 8);
    DL.stage = DL.mu + align_up((size_t)B * D * 8);
    DL.pack = DL.stage + (p->init_traj && !p->init_on_device ? align_up((size_t)(N + 1) * D * 8) : 0);
    std::vector<parapn::ReqDev> r((size_t)B * d, parapn::ReqDev{});
    for (auto &x : r) {
        x.N = N;
        x.b1 = parapn::forward_chunk(N * d);
    }
    PackPlan pl;
    int rc = plan_pack(fp64, 1, p->q, r, want_cov, 0, pl);
    if (rc) return rc;
    DL.pack64 = DL.pack + pl.L.total;
    DL.total = DL.pack64;
    if (!fp64 && want_cov && p->calibrate) {
        rc = plan_pack(true, 1, p->q, r, false, 0, pl);
        if (rc) return rc;
        DL.total += pl.L.total;
    }
    return PARAPN_OK;
}

// ---------------------------------------------------------------------------
// method-of-lines field under an approximate Jacobian: decoupled chains
// ---------------------------------------------------------------------------
// With F_y ~ 0 or diag(F_y) (remark on approximate Jacobians, Sec. 3.2.1),
// Sigma0 = 0 and the prior I_d (x) (one-dimensional prior), every matrix of
// the linearised state-space model is block diagonal over the d grid points:
// the filter and smoother factor into d independent problems of state size
// S = q+1 with one scalar observation per step.  They run as d = 1 requests
// of the row-per-lane engine (field F_MOL_COMPONENT, whose linearisation
// reads the neighbours' trajectories).  Instance b's grid point i keeps its
// preconditioned trajectory at traj + (b d + i)(N+1) S; the d requests of an
// instance share one counter slot, so delta and max |E0| are maxima over the
// chain and the quadratic forms and objective values its sums.  An instance
// that stops leaves the pack with its outputs written (its factors from the
// covariance pass over the last linearisation), so its result is the one it
// gets alone.
static int decoupled_solve(parapn_ctx *ctx, const parapn_problem *p, int B, const double *y0s, void *mean_out,
                           void *cov_out, parapn_info *info, hipStream_t s)
{
    const bool fp64 = p->precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4, d = p->d, q = p->q, S = q + 1, D = d * S;
    const int64_t N = p->N, ts = (N + 1) * S;
    std::vector<Solve> sv(B);
    for (int b = 0; b < B; ++b) {
        parapn_problem pb = *p;
        pb.y0 = y0s + (size_t)b * d;
        for (int i = 0; i < d; ++i)
            if (!std::isfinite(pb.y0[i])) return fail(PARAPN_EINVAL, "y0 is not finite");
        const int rc = prepare(&pb, sv[b]);
        if (rc) return rc;
        sv[b].start = p->init_traj ? PARAPN_START_GIVEN : PARAPN_START_CONSTANT;
    }
    const bool want_cov = cov_out != nullptr;
    const bool pass64 = !fp64 && want_cov && p->calibrate;
    const double k = (p->n_params >= 1 ? p->params[0] : 0.0) * (double)d * (double)d;
    double *trajs = nullptr;  // set once the workspace is in place
    auto requests = [&](const std::vector<int> &act) {
        std::vector<parapn::ReqDev> reqs(act.size() * d);
        for (size_t a = 0; a < act.size(); ++a)
            for (int i = 0; i < d; ++i) {
                parapn::ReqDev &r = reqs[a * d + i];
                fill_reqdev(sv[act[a]], trajs ? trajs + ((size_t)act[a] * d + i) * ts : nullptr, nullptr, r);
                r.field = parapn::F_MOL_COMPONENT;
                // the chunk length of a solve with the chain's total steps: each
                // chain alone is short, and short chunks would leave most of
                // the work to the upper scan levels
                r.b1 = parapn::forward_chunk(N * d);
                std::memset(r.p, 0, sizeof(r.p));
                r.p[0] = k;
                r.p[1] = (double)((((i + d - 1) % d) - i) * ts);
                r.p[2] = (double)((((i + 1) % d) - i) * ts);
            }
        return reqs;
    };
    std::vector<int> act(B);
    for (int b = 0; b < B; ++b) act[b] = b;
    const bool stage = p->init_traj && !p->init_on_device;
    DecoupledLayout DL;
    int rc = decoupled_layout(p, B, want_cov, DL);
    if (rc) return rc;
    const size_t o_T = DL.T, o_mu = DL.mu, o_stage = DL.stage, o_pack = DL.pack, o_64 = DL.pack64;
    PackPlan pl, pl64;
    rc = ensure_ws(ctx, DL.total);
    if (rc) return rc;
    rc = ensure_host_bits(ctx, parapn::kCounters * (size_t)B);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    ctx->consts_at = nullptr;  // this layout overwrites what the packs cached
    ctx->reqs_at = nullptr;
    trajs = (double *)ws;
    double *Tdev = (double *)(ws + o_T), *mudev = (double *)(ws + o_mu);
    {
        std::vector<double> host((size_t)S + (size_t)B * D);
        for (int j = 0; j < S; ++j) host[j] = sv[0].Td[j];
        for (int b = 0; b < B; ++b)
            for (int j = 0; j < D; ++j) host[S + (size_t)b * D + j] = sv[b].mu0b[j];
        PARAPN_HIP(hipMemcpyAsync(Tdev, host.data(), S * 8, hipMemcpyHostToDevice, s), "copy T");
        PARAPN_HIP(hipMemcpyAsync(mudev, host.data() + S, (size_t)B * D * 8, hipMemcpyHostToDevice, s), "copy mu0");
        const double *init = p->init_traj;
        if (stage) {
            PARAPN_HIP(hipMemcpyAsync(ws + o_stage, p->init_traj, (size_t)(N + 1) * D * 8, hipMemcpyHostToDevice, s),
                       "copy traj");
            init = (const double *)(ws + o_stage);
        }
        PARAPN_HIP(parapn::launch_blocks_in(B, d, S, N, init, Tdev, mudev, trajs, s), "starting trajectories");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");  // host is a local
    }
    Solve one = sv[0];  // the constants of one grid point
    one.d = 1;
    one.D = S;
    char *wp = ws + o_pack;
    const double *c64 = nullptr;
    parapn::ModelDev m{};
    bool need_plan = true;
    while (!act.empty()) {
        if (need_plan) {
            // the constants sit after the per-row arrays, so they move with the plan
            rc = plan_pack(fp64, 1, q, requests(act), want_cov, 0, pl);
            if (rc) return rc;
            bind_plan(pl, wp, d);
            rc = upload_consts(one, fp64, wp + pl.L.consts, wp + pl.L.consts64, s);
            if (rc) return rc;
            c64 = (const double *)(wp + pl.L.consts64);
            m = model_from(wp + pl.L.consts, S, esz);
            PARAPN_HIP(hipMemcpyAsync(wp + pl.L.reqs, pl.image.data(), pl.image.size(), hipMemcpyHostToDevice, s),
                       "copy request tables");
            PARAPN_HIP(hipStreamSynchronize(s), "sync");  // the image is host memory of the plan
            need_plan = false;
        }
        const int na = (int)act.size();
        std::vector<Solve *> ptr(na);
        bool obj_start = false;
        for (int a = 0; a < na; ++a) {
            ptr[a] = &sv[act[a]];
            obj_start |= ptr[a]->iter == 0 && (ptr[a]->stop_rule & 2);
        }
        unsigned long long *dbits = (unsigned long long *)(wp + pl.L.dbits);
        parapn::Pack pk = pl.pk;
        pk.mode = 0;
        pk.lm = 0;
        const parapn::Work w = work_from(wp, pl.L, false);
        PARAPN_HIP(parapn::launch_zero_u64(dbits, parapn::kCounters * (int64_t)na, s), "reset counters");
        if (obj_start) PARAPN_HIP(parapn::launch_objective(1, q, pk, c64, c64 + S * S, 4, s), "objective of the start");
        PARAPN_HIP(parapn::launch_forward(fp64, 1, q, pk, m, w, s), "forward scan");
        PARAPN_HIP(parapn::launch_smoother(fp64, 1, q, pk, m, w, false, true, nullptr, s), "reverse scan");
        PARAPN_HIP(parapn::launch_objective(1, q, pk, c64, c64 + S * S, 3, s), "objective");
        PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, dbits, parapn::kCounters * na * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s),
                   "read counters");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        pack_finish(ptr, ctx->host_bits);
        std::vector<int> fin;  // positions in act of the instances that stopped
        for (int a = 0; a < na; ++a)
            if (ptr[a]->done) fin.push_back(a);
        if (fin.empty()) continue;
        if (pass64) {
            // sigma-hat of each stopping instance from one FP64 linearise-and-
            // filter pass at its final iterate (see parapn_solve)
            std::vector<int> sub;
            for (int a : fin)
                if (ptr[a]->status != PARAPN_ENONFINITE) sub.push_back(act[a]);
            if (!sub.empty()) {
                char *w64 = ws + o_64;
                rc = plan_pack(true, 1, q, requests(sub), false, 0, pl64);
                if (rc) return rc;
                bind_plan(pl64, w64, d);
                rc = upload_consts(one, true, w64 + pl64.L.consts, w64 + pl64.L.consts64, s);
                if (rc) return rc;
                PARAPN_HIP(hipMemcpyAsync(w64 + pl64.L.reqs, pl64.image.data(), pl64.image.size(),
                                          hipMemcpyHostToDevice, s),
                           "copy request tables");
                unsigned long long *db = (unsigned long long *)(w64 + pl64.L.dbits);
                PARAPN_HIP(parapn::launch_zero_u64(db, parapn::kCounters * (int64_t)sub.size(), s), "reset counters");
                parapn::Pack p64 = pl64.pk;
                p64.mode = 0;
                p64.lm = 0;
                PARAPN_HIP(parapn::launch_forward(1, 1, q, p64, model_from(w64 + pl64.L.consts, S, 8),
                                                  work_from(w64, pl64.L, false), s),
                           "FP64 forward scan");
                PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, db, parapn::kCounters * sub.size() * 8,
                                          hipMemcpyDeviceToHost, s),
                           "read counters");
                PARAPN_HIP(hipStreamSynchronize(s), "sync");
                for (size_t j = 0; j < sub.size(); ++j) {
                    double qf;
                    std::memcpy(&qf, ctx->host_bits + parapn::kCounters * j + 2, 8);
                    sv[sub[j]].sigma2 = qf / ((double)N * d);
                }
            }
        }
        parapn::Work wc = work_from(wp, pl.L, want_cov);
        if (want_cov)
            PARAPN_HIP(parapn::launch_smoother(fp64, 1, q, pk, m, wc, true, false, wc.mf, s), "covariance pass");
        for (int a : fin) {
            const int b = act[a];
            const double cs = p->calibrate ? std::sqrt(sv[b].sigma2) : 1.0;
            PARAPN_HIP(parapn::launch_blocks_out(fp64, d, S, N, Tdev, trajs + (size_t)b * d * ts, wc.sPs,
                                                 (int64_t)a * d * (N + 1),
                                                 (char *)mean_out + (size_t)b * (N + 1) * D * esz,
                                                 want_cov ? (char *)cov_out + (size_t)b * (N + 1) * D * D * esz
                                                          : nullptr,
                                                 cs, s),
                       "outputs");
        }
        std::vector<int> keep;
        for (int a = 0; a < na; ++a)
            if (!ptr[a]->done) keep.push_back(act[a]);
        act.swap(keep);
        need_plan = true;
    }
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    int status = PARAPN_OK;
    for (int b = 0; b < B; ++b) {
        const Solve &v = sv[b];
        if (info) {
            parapn_info &f = info[b];
            f.iterations = v.iter;
            f.converged = v.converged ? 1 : 0;
            f.final_delta = v.delta;
            f.tol_used = v.tol_used;
            f.start = v.start;
            f.sigma_hat = std::sqrt(v.sigma2);
            f.objective = v.objective;
            const int cap = std::max(v.max_iter, v.fixed_iters);
            if (f.delta_history)
                for (int j = 0; j < (int)v.deltas.size() && j < cap; ++j) f.delta_history[j] = v.deltas[j];
            if (f.objective_history)
                for (int j = 0; j < (int)v.objectives.size() && j < cap; ++j) f.objective_history[j] = v.objectives[j];
        }
        if (v.status == PARAPN_ENONFINITE)
            status = PARAPN_ENONFINITE;
        else if (v.status == PARAPN_MAXITER && status == PARAPN_OK)
            status = PARAPN_MAXITER;
    }
    if (status == PARAPN_ENONFINITE) g_err = "non-finite values in the iterate";
    return status;
}

namespace {
int scratch_address(int device, void **out);
}  // namespace

extern "C" {

const char *parapn_last_error(void) { return g_err.c_str(); }

int parapn_create(parapn_ctx **out, int device, size_t budget)
{
    if (!out) return fail(PARAPN_EINVAL, "ctx pointer is NULL");
    int n = 0;
    PARAPN_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(PARAPN_EINVAL, "no such device");
    PARAPN_HIP(hipSetDevice(device), "hipSetDevice");
    void *scr = nullptr;  // the allocation-free entry point's scratch on this device
    int src = scratch_address(device, &scr);
    if (src) return src;
    parapn_ctx *c = new parapn_ctx{};
    c->device = device;
    c->budget = budget;
    int rc = ensure_host_bits(c, 64);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return PARAPN_OK;
}

void parapn_destroy(parapn_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->ws) {
        hipDeviceSynchronize();
        hipFree(c->ws);
    }
    if (c->host_bits) hipHostFree(c->host_bits);
    delete c;
}

int parapn_workspace_size(const parapn_problem *p, size_t *bytes)
{
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (!bytes) return fail(PARAPN_EINVAL, "bytes is NULL");
    if (p->field == parapn::F_MOL && p->linearization != PARAPN_LIN_EK1) {
        DecoupledLayout DL;
        rc = decoupled_layout(p, 1, true, DL);
        if (rc) return rc;
        *bytes = DL.total;
        return PARAPN_OK;
    }
    if (p->field == parapn::F_MOL) {
        *bytes = dense_layout(p->precision == PARAPN_FP64, D, p->N, 1, true).total;
        return PARAPN_OK;
    }
    std::vector<parapn::ReqDev> r(1, parapn::ReqDev{});
    r[0].N = p->N;
    size_t resident = align_up(((size_t)(p->N + 1) * D + 2 * D) * 8);
    if (!p->init_traj && p->init_mode == PARAPN_INIT_COARSE) {
        Solve sv;
        rc = prepare(p, sv);
        if (rc) return rc;
        resident += coarse_layout(sv).total;
    }
    PackPlan pl;
    rc = plan_pack(p->precision == PARAPN_FP64, p->d, q, r, true, resident, pl);
    if (rc) return rc;
    *bytes = pl.L.total;
    return PARAPN_OK;
}

int parapn_solve(parapn_ctx *ctx, const parapn_problem *p, void *mean_out, void *sqrtcov_out, parapn_info *info,
                 void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (!mean_out) return fail(PARAPN_EINVAL, "mean_out is NULL");
    const bool fp64 = p->precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4;
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if (p->field == parapn::F_MOL && p->linearization != PARAPN_LIN_EK1)
        return decoupled_solve(ctx, p, 1, p->y0, mean_out, sqrtcov_out, info, s);
    if (p->field == parapn::F_MOL) return dense_solve(ctx, p, 1, p->y0, mean_out, sqrtcov_out, info, s);
    Solve sv;
    rc = prepare(p, sv);
    if (rc) return rc;
    const bool want_cov = sqrtcov_out != nullptr;

    // the workspace holds the pack scratch (sized with the covariance pass)
    // and, in its extra region, the resident trajectory
    PackPlan pl;
    std::vector<parapn::ReqDev> r(1);
    fill_reqdev(sv, nullptr, nullptr, r[0]);
    const bool coarse = !p->init_traj && sv.init_mode == PARAPN_INIT_COARSE;
    const CoarseLayout cl = coarse ? coarse_layout(sv) : CoarseLayout{};
    // a calibrated FP32 solve takes sigma-hat from one FP64 filter pass at the
    // final iterate (in FP32 the innovations' quadratic forms cancel: each is
    // tiny against the terms it is formed from at a converged iterate)
    const bool pass64 = !fp64 && sv.calibrate;
    PackPlan pl64;
    if (pass64) {
        rc = plan_pack(true, sv.d, sv.q, r, false, 0, pl64, false);
        if (rc) return rc;
    }
    const size_t extra64 = pass64 ? pl64.L.total : 0;
    rc = plan_pack(fp64, sv.d, sv.q, r, true, resident_bytes(sv) + cl.total + extra64, pl, sv.lm_sigma > 0.0);
    if (rc) return rc;
    const PackLayout &L = pl.L;
    rc = ensure_ws(ctx, L.total);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    double *traj = (double *)(ws + L.extra);
    pl.reqs[0].traj = traj;
    rc = init_resident(sv, traj, p->init_traj, p->init_on_device != 0, s);
    if (rc) return rc;
    sv.start = p->init_traj ? PARAPN_START_GIVEN : PARAPN_START_CONSTANT;
    if (coarse) {
        rc = coarse_start(sv, fp64, ws + L.extra + resident_bytes(sv), cl, traj, s);
        if (rc) return rc;
    }

    std::vector<Solve *> one{&sv};
    std::vector<double *> trajs{traj};
    if (sv.fixed_iters > 0) {
        // the iteration count is known: queue every iteration, each copying
        // its counters to its own slot, and read them all after one wait
        // (iterations after a non-finite one change nothing that is returned)
        rc = ensure_host_bits(ctx, parapn::kCounters * (size_t)sv.fixed_iters);
        if (rc) return rc;
        for (int it = 0; it < sv.fixed_iters; ++it) {
            rc = pack_enqueue(ctx, one, trajs, s, &pl, parapn::kCounters * (size_t)it);
            if (rc) return rc;
        }
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        for (int it = 0; it < sv.fixed_iters && !sv.done; ++it)
            pack_finish(one, ctx->host_bits + parapn::kCounters * it);
    }
    while (!sv.done) {
        rc = pack_iteration(ctx, one, trajs, s, &pl);
        if (rc) return rc;
    }
    const double *Tdev = traj + (size_t)(sv.N + 1) * D;
    if (want_cov) {
        // smoothed factors of the last linearisation: the reverse scan with
        // factors over the smoothing elements still in the workspace (the
        // means go to scratch; the trajectory already holds them).  The
        // constants and request tables are in place from the iterations.
        parapn::Pack pk = pl.pk;
        const parapn::ModelDev m = model_from(ws + L.consts, D, esz);
        const parapn::Work w = work_from(ws, L, true);
        if (pk.lm && sv.status != PARAPN_ENONFINITE) {
            // damped iterations: the factors (and the quasi-MLE diffusion)
            // come from an undamped linearise-and-filter pass at the final
            // iterate
            pk.lm = 0;
            unsigned long long *db = (unsigned long long *)(ws + L.dbits);
            PARAPN_HIP(parapn::launch_zero_u64(db, parapn::kCounters, s), "reset counters");
            PARAPN_HIP(parapn::launch_forward(fp64, sv.d, sv.q, pk, m, w, s), "undamped forward scan");
            PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, db, parapn::kCounters * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost, s),
                       "read counters");
            PARAPN_HIP(hipStreamSynchronize(s), "sync");
            double qf;
            std::memcpy(&qf, ctx->host_bits + 2, 8);
            if (fp64) sv.sigma2 = qf / ((double)sv.N * sv.d);
        }
        if (pass64 && sv.status != PARAPN_ENONFINITE) {
            // FP64 linearise-and-filter pass at the final iterate for sigma-hat
            char *w64 = ws + L.extra + resident_bytes(sv) + cl.total;
            pl64.reqs[0].traj = traj;
            bind_plan(pl64, w64);
            const PackLayout &L64 = pl64.L;
            rc = upload_consts(sv, true, w64 + L64.consts, w64 + L64.consts64, s);  // waits for the stream
            if (rc) return rc;
            PARAPN_HIP(hipMemcpyAsync(w64 + L64.reqs, pl64.image.data(), pl64.image.size(), hipMemcpyHostToDevice, s),
                       "copy request tables");
            unsigned long long *db = (unsigned long long *)(w64 + L64.dbits);
            PARAPN_HIP(parapn::launch_zero_u64(db, parapn::kCounters, s), "reset counters");
            parapn::Pack p64 = pl64.pk;
            p64.mode = 0;
            p64.lm = 0;
            PARAPN_HIP(parapn::launch_forward(1, sv.d, sv.q, p64, model_from(w64 + L64.consts, D, 8),
                                              work_from(w64, L64, false), s),
                       "FP64 forward scan");
            PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, db, parapn::kCounters * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost, s),
                       "read counters");
            PARAPN_HIP(hipStreamSynchronize(s), "sync");
            double qf;
            std::memcpy(&qf, ctx->host_bits + 2, 8);
            sv.sigma2 = qf / ((double)sv.N * sv.d);
        }
        // calibrate: Sigma scales with the diffusion, so the factors with sigma-hat
        const double cs = sv.calibrate ? std::sqrt(sv.sigma2) : 1.0;
        PARAPN_HIP(parapn::launch_smoother(fp64, sv.d, sv.q, pk, m, w, true, false, w.mf, s), "covariance pass");
        PARAPN_HIP(parapn::launch_unscale(fp64, D, sv.N, Tdev, traj, w.sPs, mean_out, sqrtcov_out, s, true, cs),
                   "unscale");
    } else {
        PARAPN_HIP(parapn::launch_unscale(fp64, D, sv.N, Tdev, traj, nullptr, mean_out, nullptr, s, true),
                   "unscale");
    }
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    if (info) {
        info->iterations = sv.iter;
        info->converged = sv.converged ? 1 : 0;
        info->final_delta = sv.delta;
        info->tol_used = sv.tol_used;
        info->start = sv.start;
        info->sigma_hat = std::sqrt(sv.sigma2);
        info->objective = sv.objective;
        const int cap = std::max(sv.max_iter, sv.fixed_iters);
        if (info->delta_history)
            for (int k = 0; k < (int)sv.deltas.size() && k < cap; ++k) info->delta_history[k] = sv.deltas[k];
        if (info->objective_history)
            for (int k = 0; k < (int)sv.objectives.size() && k < cap; ++k) info->objective_history[k] = sv.objectives[k];
    }
    if (sv.status == PARAPN_ENONFINITE) g_err = "non-finite values in the iterate";
    return sv.status;
}

int parapn_start_trajectory(parapn_ctx *ctx, const parapn_problem *p, double *traj_out, int32_t *start,
                            void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (!traj_out) return fail(PARAPN_EINVAL, "traj_out is NULL");
    if (p->field == parapn::F_MOL) return fail(PARAPN_EINVAL, "the start is reported for the fixed-size fields");
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    Solve sv;
    rc = prepare(p, sv);
    if (rc) return rc;
    const bool coarse = !p->init_traj && sv.init_mode == PARAPN_INIT_COARSE;
    const CoarseLayout cl = coarse ? coarse_layout(sv) : CoarseLayout{};
    rc = ensure_ws(ctx, resident_bytes(sv) + cl.total);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    double *traj = (double *)ws;
    rc = init_resident(sv, traj, p->init_traj, p->init_on_device != 0, s);
    if (rc) return rc;
    sv.start = p->init_traj ? PARAPN_START_GIVEN : PARAPN_START_CONSTANT;
    if (coarse) {
        rc = coarse_start(sv, p->precision == PARAPN_FP64, ws + resident_bytes(sv), cl, traj, s);
        if (rc) return rc;
    }
    PARAPN_HIP(parapn::launch_unscale(1, D, sv.N, traj + (size_t)(sv.N + 1) * D, traj, nullptr, traj_out, nullptr,
                                      s, true),
               "unscale");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    if (start) *start = sv.start;
    return PARAPN_OK;
}

int parapn_solve_batch(parapn_ctx *ctx, const parapn_problem *p, int32_t batch, const double *y0s, void *mean_out,
                       void *sqrtcov_out, parapn_info *info, void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (batch < 1) return fail(PARAPN_EINVAL, "batch must be >= 1");
    if (!y0s) return fail(PARAPN_EINVAL, "y0s is NULL");
    if (!mean_out) return fail(PARAPN_EINVAL, "mean_out is NULL");
    for (size_t i = 0; i < (size_t)batch * p->d; ++i)
        if (!std::isfinite(y0s[i])) return fail(PARAPN_EINVAL, "y0s is not finite");
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if (p->field == parapn::F_MOL && p->linearization != PARAPN_LIN_EK1)
        return decoupled_solve(ctx, p, batch, y0s, mean_out, sqrtcov_out, info, s);
    if (p->field == parapn::F_MOL) return dense_solve(ctx, p, batch, y0s, mean_out, sqrtcov_out, info, s);
    // row-per-lane fields: one solve after another
    const size_t esz = p->precision == PARAPN_FP64 ? 8 : 4;
    const size_t mstride = (size_t)(p->N + 1) * D * esz, cstride = mstride * D;
    int status = PARAPN_OK;
    for (int b = 0; b < batch; ++b) {
        parapn_problem pb = *p;
        pb.y0 = y0s + (size_t)b * p->d;
        rc = parapn_solve(ctx, &pb, (char *)mean_out + b * mstride,
                          sqrtcov_out ? (char *)sqrtcov_out + b * cstride : nullptr, info ? info + b : nullptr, stream);
        if (rc < 0 && rc != PARAPN_ENONFINITE) return rc;
        if (rc == PARAPN_ENONFINITE)
            status = PARAPN_ENONFINITE;
        else if (rc == PARAPN_MAXITER && status == PARAPN_OK)
            status = PARAPN_MAXITER;
    }
    if (status == PARAPN_ENONFINITE) g_err = "non-finite values in the iterate";
    return status;
}

}  // extern "C"

namespace {

// Argument checks of ParaRTS (shared by both entry points); q_out = D/dobs - 1.
int pararts_check(int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0, const void *sqrt_sigma0,
                  const void *Phi, const void *sqrtQ, const void *H, const void *dvec, const void *mean_out, int *q_out)
{
    if (precision != PARAPN_FP64 && precision != PARAPN_FP32_SQRT) return fail(PARAPN_EINVAL, "unknown precision");
    if (dobs < 1 || D <= dobs || D > PARAPN_MAX_D || D % dobs != 0)
        return fail(PARAPN_EINVAL, "this build needs D = dobs*(q+1) with 1 <= q <= 4 and D <= 15");
    const int q = D / dobs - 1;
    if (parapn::config_supported(dobs, q) < 0) return fail(PARAPN_EINVAL, "unsupported (D, dobs)");
    if (N < 1) return fail(PARAPN_EINVAL, "N must be >= 1");
    if (!mu0 || !sqrt_sigma0 || !Phi || !sqrtQ || !H || !dvec || !mean_out)
        return fail(PARAPN_EINVAL, "NULL input or mean_out");
    *q_out = q;
    return PARAPN_OK;
}

// ParaRTS on a planned pack whose scratch starts at ws (device memory of at
// least pl.L.total bytes).  Allocates nothing; waits for the stream.
// phin, sqn: a time-varying model's per-step Phi_n, sqrtQ_n in the kernels'
// padded layout [N][D][D+1] (device), or null for the constant Phi, sqrtQ.
int pararts_run(char *ws, PackPlan &pl, int32_t D, int32_t dobs, int q, int64_t N, bool fp64, const void *mu0,
                const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out, hipStream_t s,
                const void *phin = nullptr, const void *sqn = nullptr)
{
    const int d = dobs, esz = fp64 ? 8 : 4;
    const PackLayout &L = pl.L;
    bind_plan(pl, ws);
    // initial-state record: mu0 followed by the canonical lower factor of Sigma0
    char *init = ws + L.consts;
    PARAPN_HIP(hipMemcpyAsync(init, mu0, (size_t)D * esz, hipMemcpyDeviceToDevice, s), "copy mu0");
    PARAPN_HIP(parapn::launch_tria_square(fp64, d, q, sqrt_sigma0, init + (size_t)D * esz, s),
               "canonicalise sqrt_sigma0");
    PARAPN_HIP(hipMemcpyAsync(ws + L.reqs, pl.image.data(), pl.image.size(), hipMemcpyHostToDevice, s),
               "copy request tables");
    parapn::ModelDev m;
    m.Phi = Phi;
    m.sQ = sqrtQ;
    m.init = init;
    parapn::Work w = work_from(ws, L, true);
    w.filt_mf = (filt_mean_out || filt_sqrtcov_out) ? w.mf : nullptr;
    w.filt_sPf = (filt_mean_out || filt_sqrtcov_out) ? w.sPf : nullptr;
    parapn::Pack pk = pl.pk;
    pk.mode = 1;
    pk.H = H;
    pk.dv = dvec;
    pk.phin = phin;
    pk.sqn = sqn;
    PARAPN_HIP(parapn::launch_forward(fp64, d, q, pk, m, w, s), "forward scan");
    if (filt_mean_out || filt_sqrtcov_out)
        PARAPN_HIP(parapn::launch_unscale(fp64, D, N, nullptr, w.mf, w.sPf, filt_mean_out, filt_sqrtcov_out, s),
                   "filtered outputs");
    PARAPN_HIP(parapn::launch_smoother(fp64, d, q, pk, m, w, true, false, mean_out, s), "reverse scan");
    if (sqrtcov_out)
        PARAPN_HIP(parapn::launch_unscale(fp64, D, N, nullptr, nullptr, w.sPs, nullptr, sqrtcov_out, s),
                   "smoothed factors");
    // the host table image must outlive its copy
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    return PARAPN_OK;
}

// Scratch of the allocation-free ParaRTS entry point: one array per device,
// in the library's own device data, held until the process ends.  Host code
// never passes `scratch` itself to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (resolved once per
// device, with that device current).
int scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(PARAPN_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return PARAPN_OK;
}

}  // namespace

extern "C" {

int parapn_pararts(parapn_ctx *ctx, int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                   const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                   void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out, void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    int q;
    int rc = pararts_check(D, dobs, N, precision, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out, &q);
    if (rc) return rc;
    const bool fp64 = precision == PARAPN_FP64;
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PackPlan pl;
    std::vector<parapn::ReqDev> r(1, parapn::ReqDev{});
    r[0].N = N;
    rc = plan_pack(fp64, dobs, q, r, true, 0, pl);
    if (rc) return rc;
    rc = ensure_ws(ctx, pl.L.total);
    if (rc) return rc;
    ctx->consts_at = nullptr;  // both regions are overwritten
    ctx->reqs_at = nullptr;
    return pararts_run((char *)ctx->ws, pl, D, dobs, q, N, fp64, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out,
                       sqrtcov_out, filt_mean_out, filt_sqrtcov_out, s);
}

int parapn_pararts_tv(parapn_ctx *ctx, int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                      const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                      void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out, void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    int q;
    int rc = pararts_check(D, dobs, N, precision, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out, &q);
    if (rc) return rc;
    const bool fp64 = precision == PARAPN_FP64;
    const size_t esz = fp64 ? 8 : 4, padded = align_up((size_t)N * D * (D + 1) * esz);
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PackPlan pl;
    std::vector<parapn::ReqDev> r(1, parapn::ReqDev{});
    r[0].N = N;
    rc = plan_pack(fp64, dobs, q, r, true, 2 * padded, pl);
    if (rc) return rc;
    rc = ensure_ws(ctx, pl.L.total);
    if (rc) return rc;
    ctx->consts_at = nullptr;  // every region is overwritten
    ctx->reqs_at = nullptr;
    char *ws = (char *)ctx->ws, *phin = ws + pl.L.extra, *sqn = phin + padded;
    PARAPN_HIP(parapn::launch_pad_rows(fp64, D, N, Phi, phin, s), "per-step transitions");
    PARAPN_HIP(parapn::launch_pad_rows(fp64, D, N, sqrtQ, sqn, s), "per-step noise factors");
    return pararts_run(ws, pl, D, dobs, q, N, fp64, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out, sqrtcov_out,
                       filt_mean_out, filt_sqrtcov_out, s, phin, sqn);
}

int parapn_pararts_noalloc(int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                           const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H,
                           const void *dvec, void *mean_out, void *sqrtcov_out, void *filt_mean_out,
                           void *filt_sqrtcov_out, void *stream)
{
    int q;
    int rc = pararts_check(D, dobs, N, precision, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out, &q);
    if (rc) return rc;
    const bool fp64 = precision == PARAPN_FP64;
    hipStream_t s = (hipStream_t)stream;
    PackPlan pl;
    std::vector<parapn::ReqDev> r(1, parapn::ReqDev{});
    r[0].N = N;
    rc = plan_pack(fp64, dobs, q, r, true, 0, pl);
    if (rc) return rc;
    if (pl.L.total > kNoAllocScratchBytes)
        return fail(PARAPN_ENOMEM, "parapn_pararts_noalloc: this problem needs " + std::to_string(pl.L.total) +
                                       " bytes of scratch; the static scratch holds " +
                                       std::to_string(kNoAllocScratchBytes) + " (use parapn_pararts)");
    int device = 0;
    PARAPN_HIP(hipGetDevice(&device), "hipGetDevice");
    void *ws = nullptr;
    rc = scratch_address(device, &ws);
    if (rc) return rc;
    return pararts_run((char *)ws, pl, D, dobs, q, N, fp64, mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, mean_out,
                       sqrtcov_out, filt_mean_out, filt_sqrtcov_out, s);
}

int parapn_filter_combine(parapn_ctx *ctx, int32_t D, int64_t count, int32_t precision, const void *a, const void *c,
                          void *out, void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    if (precision != PARAPN_FP64 && precision != PARAPN_FP32_SQRT) return fail(PARAPN_EINVAL, "unknown precision");
    if (count < 0 || !a || !c || !out) return fail(PARAPN_EINVAL, "bad arguments");
    int d = 0, q = 0;
    for (int dd = 1; dd <= 3 && !d; ++dd)
        for (int qq = 1; qq <= 4; ++qq)
            if (dd * (qq + 1) == D) {
                d = dd;
                q = qq;
                break;
            }
    if (!d) return fail(PARAPN_EINVAL, "no configuration with this D");
    if (count == 0) return PARAPN_OK;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(parapn::launch_filter_combine(precision == PARAPN_FP64, d, q, count, a, c, out, s), "combine");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    return PARAPN_OK;
}

int parapn_profile_enable(int on)
{
    parapn::prof_enable(on != 0);
    return PARAPN_OK;
}

int parapn_profile_only(const char *kernel)
{
    parapn::prof_only(kernel);
    return PARAPN_OK;
}

int parapn_profile_read(int32_t max, char *names, int32_t name_len, double *total_ms, int64_t *launches,
                        int32_t *n_out)
{
    if (max < 0 || name_len < 1 || (max > 0 && (!names || !total_ms || !launches)))
        return fail(PARAPN_EINVAL, "bad arguments");
    int n = parapn::prof_read(max, names, name_len, total_ms, launches);
    if (n_out) *n_out = n;
    return PARAPN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// continuous-batching server
// ---------------------------------------------------------------------------
namespace {

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device chunks (hipMalloc'd when the pool first needs them) carved first-fit
// for resident trajectories and returned with coalescing; chunks live until
// the server is destroyed, so a stream whose working set has been reached
// allocates nothing.
struct Pool {
    struct Chunk {
        char *base;
        size_t size;
        std::map<size_t, size_t> free;  // offset -> length
    };
    std::vector<Chunk> chunks;

    int alloc(size_t bytes, char **out)
    {
        bytes = align_up(bytes);
        for (auto &c : chunks)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= bytes) {
                    const size_t off = it->first, len = it->second;
                    c.free.erase(it);
                    if (len > bytes) c.free[off + bytes] = len - bytes;
                    *out = c.base + off;
                    return PARAPN_OK;
                }
        const size_t sz = std::max(bytes, size_t(256) << 20);
        char *p = nullptr;
        if (hipMalloc((void **)&p, sz) != hipSuccess) return fail(PARAPN_ENOMEM, "server pool: hipMalloc failed");
        Chunk c{p, sz, {}};
        if (sz > bytes) c.free[bytes] = sz - bytes;
        chunks.push_back(std::move(c));
        *out = p;
        return PARAPN_OK;
    }
    void release(char *p, size_t bytes)
    {
        bytes = align_up(bytes);
        for (auto &c : chunks)
            if (p >= c.base && p < c.base + c.size) {
                auto it = c.free.emplace((size_t)(p - c.base), bytes).first;
                auto nx = std::next(it);
                if (nx != c.free.end() && it->first + it->second == nx->first) {
                    it->second += nx->second;
                    c.free.erase(nx);
                }
                if (it != c.free.begin()) {
                    auto pv = std::prev(it);
                    if (pv->first + pv->second == it->first) {
                        pv->second += it->second;
                        c.free.erase(it);
                    }
                }
                return;
            }
    }
    void destroy()
    {
        for (auto &c : chunks) hipFree(c.base);
        chunks.clear();
    }
};

// Device buffer that only grows (call between steps: nothing may be in flight).
struct DevBuf {
    char *p = nullptr;
    size_t cap = 0;
    int ensure(size_t n, bool *moved = nullptr)
    {
        if (n <= cap) return PARAPN_OK;
        // doubling from 64 MiB: a stream's packs reach their size in few steps
        size_t want = std::max<size_t>(size_t(64) << 20, 2 * cap);
        while (want < n) want *= 2;
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
        if (hipMalloc((void **)&p, want) != hipSuccess) return fail(PARAPN_ENOMEM, "server scratch: hipMalloc failed");
        cap = want;
        if (moved) *moved = true;
        return PARAPN_OK;
    }
    void destroy()
    {
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Pinned host buffer that only grows.
struct HostBuf {
    unsigned char *p = nullptr;
    size_t cap = 0;
    int ensure(size_t n)
    {
        if (n <= cap) return PARAPN_OK;
        if (p) hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = size_t(1) << 20;
        while (want < n) want *= 2;
        if (hipHostMalloc((void **)&p, want, hipHostMallocDefault) != hipSuccess)
            return fail(PARAPN_ENOMEM, "server staging: hipHostMalloc failed");
        cap = want;
        return PARAPN_OK;
    }
    void destroy()
    {
        if (p) hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct ServedReq {
    uint64_t id;
    Solve sv;
    void *mean_out, *cov_out;
    char *resident;
    size_t res_bytes, bytes;  // resident trajectory; admitted footprint
    double t_submit, t_start;
    int adm_slot;             // this step's coarse-start status word, or -1
};

// One pack per (precision, d, q, damped): its own scratch (tables, elements,
// scan levels, delta slots), pinned staging, and the graph of one iteration
// of its current composition.  The tables are rebuilt only when the
// composition changes; a graph is captured once a composition has lasted one
// step and replayed while it lasts.
struct PackState {
    DevBuf dev;
    HostBuf img, bits;
    std::vector<const ServedReq *> sig;
    bool cov = false;
    bool obj_start = false;  // the objective of the start is wanted (a member at its first iteration)
    PackPlan plan;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int stable = 0;
    std::vector<ServedReq *> members;
    std::vector<Solve *> solves;

    void drop_graph()
    {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

// scratch of a request's coarse-grid start (transient: its admission step)
size_t coarse_bytes(const Solve &sv) { return sv.init_mode == PARAPN_INIT_COARSE ? coarse_layout(sv).total : 0; }

// admitted footprint of a request: its resident trajectory, its scan scratch
// (in a pack, the same region it would use alone) and its coarse start
size_t footprint(const Solve &sv, bool cov)
{
    std::vector<parapn::ReqDev> r(1);
    fill_reqdev(sv, nullptr, nullptr, r[0]);
    PackPlan pl;
    if (plan_pack(sv.precision == PARAPN_FP64, sv.d, sv.q, r, cov, 0, pl, sv.lm_sigma > 0.0) != PARAPN_OK)
        return SIZE_MAX;
    return resident_bytes(sv) + pl.L.total + coarse_bytes(sv);
}

int pack_key(const Solve &v) { return (((v.precision == PARAPN_FP64 ? 1 : 0) * 4 + v.d) * 8 + v.q) * 2 + (v.lm_sigma > 0.0); }

}  // namespace

struct parapn_server {
    parapn_ctx *ctx;
    hipStream_t stream;
    int max_slots;
    size_t budget, used, peak;
    int64_t admitted, completed;
    std::deque<ServedReq *> queue;
    std::vector<ServedReq *> active;
    std::deque<parapn_completion> done;
    Pool pool;
    std::map<int, PackState> packs;
    DevBuf adm_dev;  // coarse starts of one step's admissions
    HostBuf stage;   // pinned staging of one step's admissions
};

namespace {

// Queue one iteration of a pack (delta slots reset, forward scan, reverse
// scan with the trajectory update, delta read-back into the pack's pinned
// bits).  Only launches and a device-to-host copy: capturable.
int pack_iteration_enqueue(PackState &pk, bool fp64, int d, int q, hipStream_t s)
{
    const int nreq = (int)pk.members.size();
    const int D = d * (q + 1), esz = fp64 ? 8 : 4;
    const PackLayout &L = pk.plan.L;
    char *ws = pk.dev.p;
    unsigned long long *dbits = (unsigned long long *)(ws + L.dbits);
    PARAPN_HIP(parapn::launch_zero_u64(dbits, parapn::kCounters * (int64_t)nreq, s), "reset delta slots");
    parapn::Pack p = pk.plan.pk;
    p.mode = 0;
    const parapn::ModelDev m = model_from(ws + L.consts, D, esz);
    const parapn::Work w = work_from(ws, L, false);
    const double *c64 = (const double *)(ws + L.consts64);
    if (pk.obj_start)
        PARAPN_HIP(parapn::launch_objective(d, q, p, c64, c64 + D * D, 4, s), "objective of the start");
    PARAPN_HIP(parapn::launch_forward(fp64, d, q, p, m, w, s), "forward scan");
    PARAPN_HIP(parapn::launch_smoother(fp64, d, q, p, m, w, false, true, nullptr, s), "reverse scan");
    PARAPN_HIP(parapn::launch_objective(d, q, p, c64, c64 + D * D, 3, s), "objective");
    PARAPN_HIP(hipMemcpyAsync(pk.bits.p, dbits, parapn::kCounters * (size_t)nreq * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s),
               "read delta");
    return PARAPN_OK;
}

// (Re)build a pack's tables for its members, upload them and its constants.
int pack_replan(PackState &pk, bool fp64, int d, int q, bool lm, hipStream_t s)
{
    const int nreq = (int)pk.members.size();
    const int D = d * (q + 1);
    std::vector<parapn::ReqDev> reqs(nreq);
    for (int i = 0; i < nreq; ++i) fill_reqdev(pk.members[i]->sv, (double *)pk.members[i]->resident, nullptr, reqs[i]);
    int rc = plan_pack(fp64, d, q, reqs, pk.cov, 0, pk.plan, lm);
    if (rc) return rc;
    bool moved = false;
    rc = pk.dev.ensure(pk.plan.L.total, &moved);
    if (rc) return rc;
    if (moved) pk.drop_graph();
    bind_plan(pk.plan, pk.dev.p);
    // staging: constants [Phi | sqrtQ | initial increment state (0, 0)], then the table image
    std::vector<double> Phi, sQ;
    prior_blocks(d, q, Phi, sQ);
    const size_t cbytes = (size_t)(3 * D * D + D) * (fp64 ? 8 : 4);
    rc = pk.img.ensure(cbytes + pk.plan.image.size());
    if (rc) return rc;
    std::memset(pk.img.p, 0, cbytes);
    for (int i = 0; i < D * D; ++i) {
        if (fp64) {
            ((double *)pk.img.p)[i] = Phi[i];
            ((double *)pk.img.p)[D * D + i] = sQ[i];
        } else {
            ((float *)pk.img.p)[i] = (float)Phi[i];
            ((float *)pk.img.p)[D * D + i] = (float)sQ[i];
        }
    }
    std::memcpy(pk.img.p + cbytes, pk.plan.image.data(), pk.plan.image.size());
    PARAPN_HIP(hipMemcpyAsync(pk.dev.p + pk.plan.L.consts, pk.img.p, cbytes, hipMemcpyHostToDevice, s),
               "copy constants");
    // FP64 Phi, sqrtQ for the objective value, after the table image
    const size_t c64off = align_up(cbytes + pk.plan.image.size());
    rc = pk.img.ensure(c64off + (size_t)2 * D * D * 8);
    if (rc) return rc;
    double *c64 = (double *)(pk.img.p + c64off);
    for (int i = 0; i < D * D; ++i) {
        c64[i] = Phi[i];
        c64[D * D + i] = sQ[i];
    }
    PARAPN_HIP(hipMemcpyAsync(pk.dev.p + pk.plan.L.consts64, c64, (size_t)2 * D * D * 8, hipMemcpyHostToDevice, s),
               "copy FP64 constants");
    PARAPN_HIP(hipMemcpyAsync(pk.dev.p + pk.plan.L.reqs, pk.img.p + cbytes, pk.plan.image.size(),
                              hipMemcpyHostToDevice, s),
               "copy request tables");
    rc = pk.bits.ensure(parapn::kCounters * (size_t)nreq * sizeof(unsigned long long));
    return rc;
}

// Admission work of one step on the stream: every admitted request's resident
// tail (T, mu0/T) and constant trajectory, then the coarse-grid starts of
// those that asked for one, one launch per (d, q).  Host tables are staged
// in pinned memory that stays untouched until the step's wait.
int admit_enqueue(parapn_server *srv, std::vector<ServedReq *> &adm, hipStream_t s)
{
    if (adm.empty()) return PARAPN_OK;
    // staging layout: tails, then per coarse group [reqs | cds | consts], then per
    // coarse request [W | mu0c], then the status words (read back)
    struct Item {
        ServedReq *r;
        CoarseLayout cl;
        size_t w_off, mu_off;  // in the upload region
        size_t node_off, gain_off;  // in the scratch region
    };
    std::map<int, std::vector<Item>> groups;  // by d * 8 + q
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t r = off;
        off = align_up(off + b);
        return r;
    };
    std::vector<size_t> tail_off(adm.size());
    for (size_t i = 0; i < adm.size(); ++i) tail_off[i] = take((size_t)2 * adm[i]->sv.D * 8);
    for (ServedReq *r : adm)
        if (r->sv.init_mode == PARAPN_INIT_COARSE) groups[r->sv.d * 8 + r->sv.q].push_back(Item{r, coarse_layout(r->sv)});
    struct Group {
        int d, q;
        size_t reqs_off, cds_off, consts_off;
        std::vector<Item> *items;
    };
    std::vector<Group> gl;
    int nstat = 0;
    for (auto &kv : groups) {
        Group g;
        g.d = kv.first / 8;
        g.q = kv.first % 8;
        g.items = &kv.second;
        const int n = (int)kv.second.size();
        g.reqs_off = take((size_t)n * sizeof(parapn::ReqDev));
        g.cds_off = take((size_t)n * sizeof(parapn::CoarseDev));
        const int D = g.d * (g.q + 1);
        g.consts_off = take((size_t)2 * D * D * 8);
        for (Item &it : kv.second) {
            it.w_off = take((size_t)it.cl.s * (g.q + 1) * 2 * (g.q + 1) * 8);
            it.mu_off = take((size_t)D * 8);
            it.r->adm_slot = nstat++;
        }
        gl.push_back(g);
    }
    const size_t status_off = take((size_t)std::max(nstat, 1) * sizeof(int));
    const size_t upload = off;
    // device scratch of the coarse smoothers after the upload region
    for (auto &kv : groups)
        for (Item &it : kv.second) {
            it.node_off = take((size_t)(it.cl.M + 1) * it.r->sv.D * 8);
            it.gain_off = take((size_t)(it.cl.M + 1) * parapn::coarse_record_doubles(it.r->sv.d, it.r->sv.q) * 8);
        }
    int rc = srv->stage.ensure(upload);
    if (rc) return rc;
    rc = srv->adm_dev.ensure(off);
    if (rc) return rc;
    unsigned char *h = srv->stage.p;
    char *dv = srv->adm_dev.p;
    // resident tails and the constant start
    for (size_t i = 0; i < adm.size(); ++i) {
        const Solve &v = adm[i]->sv;
        double *t = (double *)(h + tail_off[i]);
        for (int k = 0; k < v.D; ++k) {
            t[k] = v.Td[k];
            t[v.D + k] = v.mu0b[k];
        }
        double *traj = (double *)adm[i]->resident;
        double *tail = traj + (size_t)(v.N + 1) * v.D;
        PARAPN_HIP(hipMemcpyAsync(tail, t, (size_t)2 * v.D * 8, hipMemcpyHostToDevice, s), "copy T");
        PARAPN_HIP(parapn::launch_init_traj(v.D, v.N, nullptr, tail, traj, s), "initial trajectory");
    }
    if (gl.empty()) return PARAPN_OK;
    for (Group &g : gl) {
        const int D = g.d * (g.q + 1), S = g.q + 1;
        std::vector<double> Phi, sQ;
        prior_blocks(g.d, g.q, Phi, sQ);
        double *cst = (double *)(h + g.consts_off);
        for (int i = 0; i < 2 * D * D; ++i) cst[i] = 0.0;
        for (int i = 0; i < D * D; ++i) cst[i] = Phi[i];
        for (int b = 0; b < g.d; ++b)
            for (int i = 0; i < S; ++i)
                for (int j = 0; j < S; ++j) cst[D * D + (b * S + i) * D + b * S + j] = 1.0 / (2 * g.q + 1 - i - j);
        parapn::ReqDev *rq = (parapn::ReqDev *)(h + g.reqs_off);
        parapn::CoarseDev *cd = (parapn::CoarseDev *)(h + g.cds_off);
        int64_t maxN = 1;
        for (size_t k = 0; k < g.items->size(); ++k) {
            Item &it = (*g.items)[k];
            Solve &v = it.r->sv;
            std::vector<double> Tc, W;
            precond_diag(v.d, v.q, (double)it.cl.s * v.h, Tc);
            bridge_weights(v.q, it.cl.s, W);
            std::memcpy(h + it.w_off, W.data(), W.size() * 8);
            double *mu = (double *)(h + it.mu_off);
            for (int j = 0; j < D; ++j) mu[j] = v.mu0[j] / Tc[j];
            fill_reqdev(v, (double *)it.r->resident, nullptr, rq[k]);
            parapn::CoarseDev c{};
            c.M = it.cl.M;
            c.s = it.cl.s;
            c.T0 = Tc[0];
            c.T1 = Tc[1];
            c.invT1 = 1.0 / Tc[1];
            c.hq = (double)it.cl.s * v.h / v.q;
            c.node = (double *)(dv + it.node_off);
            c.gain = dv + it.gain_off;
            c.W = (const double *)(dv + it.w_off);
            c.mu0c = (const double *)(dv + it.mu_off);
            c.status = (int *)(dv + status_off) + it.r->adm_slot;
            cd[k] = c;
            maxN = std::max<int64_t>(maxN, v.N);
        }
        (void)maxN;
    }
    PARAPN_HIP(hipMemcpyAsync(dv, h, status_off, hipMemcpyHostToDevice, s), "copy coarse tables");
    for (Group &g : gl) {
        int64_t maxN = 1;
        for (Item &it : *g.items) maxN = std::max<int64_t>(maxN, it.r->sv.N);
        const int D = g.d * (g.q + 1);
        PARAPN_HIP(parapn::launch_coarse(1, g.d, g.q, (const parapn::ReqDev *)(dv + g.reqs_off),
                                         (const parapn::CoarseDev *)(dv + g.cds_off), (int)g.items->size(), maxN,
                                         dv + g.consts_off, dv + g.consts_off + (size_t)D * D * 8, s),
                   "coarse start");
    }
    PARAPN_HIP(hipMemcpyAsync(h + status_off, dv + status_off, (size_t)nstat * sizeof(int), hipMemcpyDeviceToHost, s),
               "read coarse status");
    // after the step's wait, each coarse request reads its word from here
    for (auto &kv : groups)
        for (Item &it : kv.second) it.r->adm_slot = (int)(status_off / sizeof(int)) + it.r->adm_slot;
    return PARAPN_OK;
}

}  // namespace

extern "C" {

int parapn_server_create(parapn_server **out, parapn_ctx *ctx, int32_t max_slots, size_t hbm_budget_bytes,
                         void *stream)
{
    if (!out || !ctx) return fail(PARAPN_EINVAL, "NULL argument");
    if (max_slots < 1) return fail(PARAPN_EINVAL, "max_slots must be >= 1");
    parapn_server *sv = new parapn_server{};
    sv->ctx = ctx;
    sv->stream = (hipStream_t)stream;
    sv->max_slots = max_slots;
    sv->budget = hbm_budget_bytes;
    sv->used = 0;
    *out = sv;
    return PARAPN_OK;
}

void parapn_server_destroy(parapn_server *srv)
{
    if (!srv) return;
    hipSetDevice(srv->ctx->device);
    hipStreamSynchronize(srv->stream);
    for (ServedReq *r : srv->active) delete r;
    for (ServedReq *r : srv->queue) delete r;
    for (auto &kv : srv->packs) {
        kv.second.drop_graph();
        kv.second.dev.destroy();
        kv.second.img.destroy();
        kv.second.bits.destroy();
    }
    srv->adm_dev.destroy();
    srv->stage.destroy();
    srv->pool.destroy();
    delete srv;
}

double parapn_server_clock(void) { return now_seconds(); }

int parapn_server_footprint(const parapn_problem *p, size_t *bytes)
{
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (!bytes) return fail(PARAPN_EINVAL, "bytes is NULL");
    if (p->field == parapn::F_MOL) return fail(PARAPN_EINVAL, "the server does not batch the method-of-lines field");
    if (p->prior != PARAPN_PRIOR_IWP) return fail(PARAPN_EINVAL, "served requests use the IWP prior");
    Solve sv;
    rc = prepare(p, sv);
    if (rc) return rc;
    *bytes = footprint(sv, false);
    return *bytes == SIZE_MAX ? PARAPN_EINVAL : PARAPN_OK;
}

int parapn_server_stats(parapn_server *srv, size_t *used_bytes, size_t *peak_bytes, int64_t *admitted,
                        int64_t *completed)
{
    if (!srv) return fail(PARAPN_EINVAL, "server is NULL");
    if (used_bytes) *used_bytes = srv->used;
    if (peak_bytes) *peak_bytes = srv->peak;
    if (admitted) *admitted = srv->admitted;
    if (completed) *completed = srv->completed;
    return PARAPN_OK;
}

int parapn_server_submit(parapn_server *srv, const parapn_problem *p, uint64_t req_id, void *mean_out,
                         void *sqrtcov_out)
{
    if (!srv) return fail(PARAPN_EINVAL, "server is NULL");
    int q, D;
    int rc = check_problem(p, &q, &D);
    if (rc) return rc;
    if (!mean_out) return fail(PARAPN_EINVAL, "mean_out is NULL");
    if (p->init_traj) return fail(PARAPN_EINVAL, "served requests start from mu0 or their coarse-grid start");
    if (p->field == parapn::F_MOL) return fail(PARAPN_EINVAL, "the server does not batch the method-of-lines field");
    if (p->prior != PARAPN_PRIOR_IWP) return fail(PARAPN_EINVAL, "served requests use the IWP prior");
    ServedReq *r = new ServedReq{};
    r->id = req_id;
    rc = prepare(p, r->sv);
    if (rc) {
        delete r;
        return rc;
    }
    r->mean_out = mean_out;
    r->cov_out = sqrtcov_out;
    r->res_bytes = resident_bytes(r->sv);
    r->bytes = footprint(r->sv, sqrtcov_out != nullptr);
    r->adm_slot = -1;
    if (r->bytes == SIZE_MAX) {  // the reason is already recorded
        delete r;
        return PARAPN_EINVAL;
    }
    if (srv->budget && r->bytes > srv->budget) {
        delete r;
        return fail(PARAPN_ENOMEM, "request footprint exceeds the server budget");
    }
    r->t_submit = now_seconds();
    srv->queue.push_back(r);
    return PARAPN_OK;
}

int parapn_server_step(parapn_server *srv, int32_t *n_active, int32_t *n_queued)
{
    if (!srv) return fail(PARAPN_EINVAL, "server is NULL");
    hipStream_t s = srv->stream;
    PARAPN_HIP(hipSetDevice(srv->ctx->device), "hipSetDevice");
    // 1. admission in arrival order, by slots and HBM footprint
    std::vector<ServedReq *> adm;
    while (!srv->queue.empty() && (int)srv->active.size() < srv->max_slots) {
        ServedReq *r = srv->queue.front();
        if (srv->budget && srv->used + r->bytes > srv->budget) break;
        if (srv->pool.alloc(r->res_bytes, &r->resident) != PARAPN_OK) break;  // wait for memory to free up
        r->t_start = now_seconds();
        r->adm_slot = -1;
        r->sv.start = PARAPN_START_CONSTANT;
        srv->used += r->bytes;
        srv->peak = std::max(srv->peak, srv->used);
        srv->admitted += 1;
        srv->queue.pop_front();
        srv->active.push_back(r);
        adm.push_back(r);
    }
    int rc = admit_enqueue(srv, adm, s);
    if (rc) return rc;
    // 2. one IEKS iteration for every active request: the packs are queued
    // back to back and their work overlaps on the device; one wait
    for (auto &kv : srv->packs) {
        kv.second.members.clear();
        kv.second.solves.clear();
    }
    for (ServedReq *r : srv->active) {
        PackState &pk = srv->packs[pack_key(r->sv)];
        pk.members.push_back(r);
        pk.solves.push_back(&r->sv);
    }
    // graphs need a stream that can be captured (not the legacy default
    // stream) and no per-launch timing events
    const bool graphs = s != nullptr && !parapn::prof_on();
    for (auto &kv : srv->packs) {
        PackState &pk = kv.second;
        if (pk.members.empty()) {
            pk.sig.clear();
            pk.drop_graph();
            continue;
        }
        const Solve &v0 = *pk.solves[0];
        const bool fp64 = v0.precision == PARAPN_FP64, lm = v0.lm_sigma > 0.0;
        bool cov = false, obj_start = false;
        for (ServedReq *r : pk.members) {
            cov |= r->cov_out != nullptr;
            obj_start |= r->sv.iter == 0 && (r->sv.stop_rule & 2);
        }
        if (obj_start != pk.obj_start) pk.drop_graph();  // another launch sequence
        pk.obj_start = obj_start;
        std::vector<const ServedReq *> sig(pk.members.begin(), pk.members.end());
        if (sig != pk.sig || cov != pk.cov) {
            pk.drop_graph();
            pk.sig = sig;
            pk.cov = cov;
            pk.stable = 0;
            rc = pack_replan(pk, fp64, v0.d, v0.q, lm, s);
            if (rc) return rc;
        } else {
            pk.stable += 1;
        }
        if (graphs && pk.stable >= 1) {
            if (!pk.exec) {
                PARAPN_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
                rc = pack_iteration_enqueue(pk, fp64, v0.d, v0.q, s);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(s, &g);
                if (rc) {
                    if (g) hipGraphDestroy(g);
                    return rc;
                }
                PARAPN_HIP(e, "end capture");
                pk.graph = g;
                PARAPN_HIP(hipGraphInstantiate(&pk.exec, pk.graph, nullptr, nullptr, 0), "graph instantiate");
            }
            PARAPN_HIP(hipGraphLaunch(pk.exec, s), "graph launch");
        } else {
            rc = pack_iteration_enqueue(pk, fp64, v0.d, v0.q, s);
            if (rc) return rc;
        }
    }
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    for (ServedReq *r : adm)
        if (r->adm_slot >= 0)
            r->sv.start = ((const int *)srv->stage.p)[r->adm_slot] == 0 ? PARAPN_START_COARSE
                                                                       : PARAPN_START_COARSE_FAILED;
    for (auto &kv : srv->packs)
        if (!kv.second.members.empty())
            pack_finish(kv.second.solves, (const unsigned long long *)kv.second.bits.p);
    // 3. retire the finished requests: their means (and factors) in original
    // coordinates, then their memory back to the pool
    bool any = false;
    for (auto &kv : srv->packs) {
        PackState &pk = kv.second;
        if (pk.members.empty()) continue;
        bool cov_done = false;
        for (ServedReq *r : pk.members) cov_done |= r->sv.done && r->cov_out && r->sv.status != PARAPN_ENONFINITE;
        const Solve &v0 = *pk.solves[0];
        const bool fp64 = v0.precision == PARAPN_FP64;
        const int D = v0.D, esz = fp64 ? 8 : 4;
        const PackLayout &L = pk.plan.L;
        if (cov_done) {
            // smoothed factors of the last linearisation: the reverse scan with
            // factors over the pack's smoothing elements (means to scratch)
            parapn::Pack p = pk.plan.pk;
            p.mode = 0;
            const parapn::ModelDev m = model_from(pk.dev.p + L.consts, D, esz);
            const parapn::Work w = work_from(pk.dev.p, L, true);
            if (p.lm) {
                p.lm = 0;
                PARAPN_HIP(parapn::launch_forward(fp64, v0.d, v0.q, p, m, w, s), "undamped forward scan");
            }
            PARAPN_HIP(parapn::launch_smoother(fp64, v0.d, v0.q, p, m, w, true, false, w.mf, s), "covariance pass");
        }
        for (size_t i = 0; i < pk.members.size(); ++i) {
            ServedReq *r = pk.members[i];
            if (!r->sv.done) continue;
            any = true;
            const Solve &v = r->sv;
            const double *traj = (const double *)r->resident;
            const double *Tdev = traj + (size_t)(v.N + 1) * v.D;
            const bool want = r->cov_out && v.status != PARAPN_ENONFINITE;
            const char *sPs = want ? pk.dev.p + L.sPs + (size_t)pk.plan.reqs[i].row * (D * (D + 1) / 2) * esz : nullptr;
            const double cs = v.calibrate ? std::sqrt(v.sigma2) : 1.0;
            PARAPN_HIP(parapn::launch_unscale(fp64, v.D, v.N, Tdev, traj, sPs, r->mean_out, want ? r->cov_out : nullptr,
                                              s, true, cs),
                       "unscale");
        }
    }
    if (any) {
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        std::vector<ServedReq *> still;
        for (ServedReq *r : srv->active) {
            if (!r->sv.done) {
                still.push_back(r);
                continue;
            }
            srv->pool.release(r->resident, r->res_bytes);
            srv->used -= r->bytes;
            const Solve &v = r->sv;
            parapn_completion c{};
            c.req_id = r->id;
            c.status = v.status;
            c.iterations = v.iter;
            c.final_delta = v.delta;
            c.t_submit = r->t_submit;
            c.t_start = r->t_start;
            c.t_done = now_seconds();
            c.start = v.start;
            c.sigma_hat = std::sqrt(v.sigma2);
            c.objective = v.objective;
            srv->done.push_back(c);
            srv->completed += 1;
            delete r;
        }
        srv->active.swap(still);
    }
    if (n_active) *n_active = (int32_t)srv->active.size();
    if (n_queued) *n_queued = (int32_t)srv->queue.size();
    return PARAPN_OK;
}

int parapn_server_poll(parapn_server *srv, parapn_completion *out, int32_t max, int32_t *n_out)
{
    if (!srv || (max > 0 && !out)) return fail(PARAPN_EINVAL, "bad arguments");
    int k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    if (n_out) *n_out = k;
    return PARAPN_OK;
}

}  // extern "C"
