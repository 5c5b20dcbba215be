// C ABI of the parallel-in-time probabilistic ODE solver (include/parapn.h):
// argument checking, the FP64 host part of the prior (Sec. 2.1, Sec. 2.4)
// and of the exact initialisation (eq. mu0), workspace management, and the
// iteration loop of Alg. 2 around the device scans.
#include "parapn.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

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

bool taylor_mu0(int field, int d, const double *p, const double *y0, int q, double *mu0)
{
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

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t off_traj, off_mf, off_sPf, off_se, off_sL, off_sPs, off_fagg, off_fpref, off_sagg, off_spref;
    size_t off_consts, off_T, off_dbits, total;
};

// Forward chunk: long enough that the step-level aggregates (folded with the
// cheaper single-element operator) leave little work for the upper tree levels,
// short enough that about 8192 groups keep every SIMD busy.
parapn::ScanPlan default_plan(int64_t N)
{
    parapn::ScanPlan p;
    p.N = N;
    int b1 = 4;
    while (b1 < 32 && N / (2 * b1) >= 8192) b1 *= 2;
    p.b1 = b1;
    p.bs1 = 8;
    p.bu = 8;
    p.btop = 16;
    return p;
}

Layout make_layout(int D, int64_t N, int esz, bool cov, const parapn::ScanPlan &plan)
{
    const size_t DP = (size_t)D * (D + 1) / 2;
    const size_t rows = (size_t)N + 1;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t elems) {
        size_t r = o;
        o = align_up(o + elems * esz);
        return r;
    };
    L.off_traj = align_up(o);  // FP64 trajectory in both precisions
    o = align_up(o + rows * D * sizeof(double));
    L.off_mf = take(rows * D);
    L.off_sPf = take(rows * DP);
    L.off_se = take(rows * (D * D + D));
    L.off_sL = take(rows * DP);
    L.off_sPs = cov ? take(rows * DP) : 0;
    const size_t fagg = parapn::work_elems_fagg(D, plan);
    L.off_fagg = take(fagg);
    L.off_fpref = take(parapn::work_records_fpref(plan) * (D + D * D));
    const size_t sagg = parapn::work_elems_sagg(D, plan);
    const size_t srec = sagg / (2 * D * D + D);
    L.off_sagg = take(sagg);
    L.off_spref = take(srec * (D + D * D));
    L.off_consts = take(3 * D * D + D);
    o = align_up(o);
    L.off_T = o;
    o = align_up(o + 2 * D * sizeof(double));  // T, then mu0bar in double
    L.off_dbits = o;
    o = align_up(o + 2 * sizeof(unsigned long long));
    L.total = o;
    return L;
}

}  // namespace

struct parapn_ctx {
    int device;
    size_t budget;
    void *ws;
    size_t ws_bytes;
    unsigned long long *host_bits;  // pinned, 2 entries
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
    hipError_t e = hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return fail(PARAPN_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
    }
    ctx->ws_bytes = bytes;
    return PARAPN_OK;
}

static int check_problem(const parapn_problem *p, int *q_out, int *D_out)
{
    if (!p) return fail(PARAPN_EINVAL, "problem is NULL");
    const int fd = parapn::field_fixed_dim(p->field);
    if (fd < 0) return fail(PARAPN_EINVAL, "unknown field id " + std::to_string(p->field));
    if (fd > 0 && p->d != fd) return fail(PARAPN_EINVAL, "field requires d = " + std::to_string(fd));
    if (p->d < 1 || p->d > 3) return fail(PARAPN_EINVAL, "d must be in 1..3 in this build");
    if (p->q < 1 || p->q > 4) return fail(PARAPN_EINVAL, "q must be in 1..4");
    if (parapn::config_supported(p->d, p->q) < 0) return fail(PARAPN_EINVAL, "unsupported (d, q)");
    const int np = parapn::field_n_params(p->field, p->d);
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
    for (int i = 0; i < p->d; ++i)
        if (!std::isfinite(p->y0[i])) return fail(PARAPN_EINVAL, "y0 is not finite");
    *q_out = p->q;
    *D_out = p->d * (p->q + 1);
    return PARAPN_OK;
}

extern "C" {

const char *parapn_last_error(void) { return g_err.c_str(); }

int parapn_create(parapn_ctx **out, int device, size_t budget)
{
    if (!out) return fail(PARAPN_EINVAL, "ctx pointer is NULL");
    int n = 0;
    PARAPN_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(PARAPN_EINVAL, "no such device");
    PARAPN_HIP(hipSetDevice(device), "hipSetDevice");
    parapn_ctx *c = new parapn_ctx{};
    c->device = device;
    c->budget = budget;
    hipError_t e = hipHostMalloc((void **)&c->host_bits, 2 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipHostMalloc");
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
    const int esz = p->precision == PARAPN_FP64 ? 8 : 4;
    *bytes = make_layout(D, p->N, esz, true, default_plan(p->N)).total;
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
    const int d = p->d, S = q + 1;
    const bool fp64 = p->precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4;
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");

    const parapn::ScanPlan plan = default_plan(p->N);
    const bool want_cov = sqrtcov_out != nullptr;
    const Layout L = make_layout(D, p->N, esz, want_cov, plan);
    rc = ensure_ws(ctx, L.total);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;

    // FP64 host constants
    const double h = (p->t1 - p->t0) / (double)p->N;
    std::vector<double> Phi, sQ, Td, mu0(D);
    prior_blocks(d, q, Phi, sQ);
    precond_diag(d, q, h, Td);
    double prm[PARAPN_MAX_PARAMS] = {0};
    for (int i = 0; i < p->n_params && i < PARAPN_MAX_PARAMS; ++i) prm[i] = p->params[i];
    if (!taylor_mu0(p->field, d, prm, p->y0, q, mu0.data())) return fail(PARAPN_EINVAL, "field not available for d");
    for (int k = 0; k < D; ++k)
        if (!std::isfinite(mu0[k])) return fail(PARAPN_EINVAL, "non-finite initial derivatives");
    // Phi | sQ | m0 (= 0) | S0 (= 0): the scans run on the increment over the
    // trajectory, whose row 0 is mu0 itself, so the initial increment is 0;
    // (m0, S0) is one contiguous initial-state record
    std::vector<double> cst(3 * D * D + D, 0.0);
    for (int i = 0; i < D * D; ++i) {
        cst[i] = Phi[i];
        cst[D * D + i] = sQ[i];
    }
    std::vector<double> Tmu(2 * D);
    for (int k = 0; k < D; ++k) {
        Tmu[k] = Td[k];
        Tmu[D + k] = mu0[k] / Td[k];
    }
    char *cdev = ws + L.off_consts;
    if (fp64) {
        PARAPN_HIP(hipMemcpyAsync(cdev, cst.data(), cst.size() * 8, hipMemcpyHostToDevice, s), "copy constants");
    } else {
        std::vector<float> cf(cst.begin(), cst.end());
        PARAPN_HIP(hipMemcpyAsync(cdev, cf.data(), cf.size() * 4, hipMemcpyHostToDevice, s), "copy constants");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");  // cf is a local
    }
    PARAPN_HIP(hipMemcpyAsync(ws + L.off_T, Tmu.data(), 2 * D * sizeof(double), hipMemcpyHostToDevice, s),
               "copy T");

    parapn::ModelDev m;
    m.Phi = cdev;
    m.sQ = cdev + (size_t)D * D * esz;
    m.m0 = cdev + (size_t)2 * D * D * esz;
    m.S0 = cdev + (size_t)(2 * D * D + D) * esz;
    m.init = m.m0;

    parapn::Work w{};
    w.traj = ws + L.off_traj;
    w.mf = ws + L.off_mf;
    w.sPf = ws + L.off_sPf;
    w.se = ws + L.off_se;
    w.sL = ws + L.off_sL;
    w.sPs = want_cov ? ws + L.off_sPs : nullptr;
    w.fagg = ws + L.off_fagg;
    w.fpref = ws + L.off_fpref;
    w.sagg = ws + L.off_sagg;
    w.spref = ws + L.off_spref;
    w.dbits = (unsigned long long *)(ws + L.off_dbits);

    // initial trajectory (Alg. 2): constant mu0, or the caller's; preconditioned,
    // FP64, row 0 always mu0 (only E0 of row 0 enters the convergence test)
    if (p->init_traj) {
        const size_t rows = (size_t)p->N + 1;
        std::vector<double> tr(rows * D);
        for (int k = 0; k < D; ++k) tr[k] = mu0[k] / Td[k];
        for (size_t n = 1; n < rows; ++n)
            for (int k = 0; k < D; ++k) tr[n * D + k] = p->init_traj[n * D + k] / Td[k];
        PARAPN_HIP(hipMemcpyAsync(w.traj, tr.data(), tr.size() * 8, hipMemcpyHostToDevice, s), "copy traj");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
    } else {
        PARAPN_HIP(parapn::launch_fill_traj(1, D, p->N, ws + L.off_T + D * sizeof(double), w.traj, s),
                   "fill trajectory");
    }

    parapn::ObsSpec obs{};
    obs.mode = 0;
    obs.traj = w.traj;
    obs.field = p->field;
    for (int i = 0; i < PARAPN_MAX_PARAMS; ++i) obs.p[i] = prm[i];
    obs.T0 = Td[0];
    obs.T1 = Td[1];
    obs.invT1 = 1.0 / Td[1];
    obs.hq = h / q;

    const int limit = p->fixed_iters > 0 ? p->fixed_iters : p->max_iter;
    int status = PARAPN_MAXITER, k = 0;
    double delta = 0.0, tol_used = p->tol;
    for (k = 1; k <= limit; ++k) {
        PARAPN_HIP(hipMemsetAsync(w.dbits, 0, 2 * sizeof(unsigned long long), s), "memset");
        PARAPN_HIP(parapn::launch_forward(fp64, d, q, plan, m, obs, w, s), "forward scan");
        PARAPN_HIP(parapn::launch_smoother(fp64, d, q, plan, m, w, false, true, nullptr, Td[0], s), "reverse scan");
        PARAPN_HIP(hipMemcpyAsync(ctx->host_bits, w.dbits, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                   "read delta");
        PARAPN_HIP(hipStreamSynchronize(s), "sync");
        unsigned long long b0 = ctx->host_bits[0], b1 = ctx->host_bits[1];
        double mmax;
        std::memcpy(&delta, &b0, 8);
        std::memcpy(&mmax, &b1, 8);
        if (info && info->delta_history && k <= (p->max_iter > limit ? p->max_iter : limit))
            info->delta_history[k - 1] = delta;
        if (!std::isfinite(delta)) {
            status = PARAPN_ENONFINITE;
            break;
        }
        tol_used = fp64 ? p->tol : std::fmax(p->tol, std::ldexp(mmax, -20));
        if (p->fixed_iters > 0) {
            if (k == limit) {
                status = PARAPN_OK;
                break;
            }
            continue;
        }
        if (delta < tol_used) {
            status = PARAPN_OK;
            break;
        }
        if (k == limit) {
            status = PARAPN_MAXITER;
            break;
        }
    }
    if (k > limit) k = limit;
    if (want_cov) {
        // the smoothing factors of the last linearisation, from the filtering
        // marginals still in the workspace (the means are not needed again)
        PARAPN_HIP(parapn::launch_smoother(fp64, d, q, plan, m, w, true, false, w.mf, Td[0], s), "covariance pass");
    }
    PARAPN_HIP(parapn::launch_unscale(fp64, D, p->N, (const double *)(ws + L.off_T), w.traj, w.sPs, mean_out,
                                      sqrtcov_out, s, true),
               "unscale");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    if (info) {
        info->iterations = k;
        info->converged = status == PARAPN_OK && p->fixed_iters <= 0;
        info->final_delta = delta;
        info->tol_used = tol_used;
    }
    if (status == PARAPN_ENONFINITE) g_err = "non-finite values in the iterate";
    (void)S;
    return status;
}

int parapn_pararts(parapn_ctx *ctx, int32_t D, int32_t dobs, int64_t N, int32_t precision, const void *mu0,
                   const void *sqrt_sigma0, const void *Phi, const void *sqrtQ, const void *H, const void *dvec,
                   void *mean_out, void *sqrtcov_out, void *filt_mean_out, void *filt_sqrtcov_out, void *stream)
{
    if (!ctx) return fail(PARAPN_EINVAL, "ctx is NULL");
    if (precision != PARAPN_FP64 && precision != PARAPN_FP32_SQRT) return fail(PARAPN_EINVAL, "unknown precision");
    if (dobs < 1 || D <= dobs || D > PARAPN_MAX_D || D % dobs != 0)
        return fail(PARAPN_EINVAL, "this build needs D = dobs*(q+1) with 1 <= q <= 4 and D <= 15");
    const int d = dobs, q = D / dobs - 1;
    if (parapn::config_supported(d, q) < 0) return fail(PARAPN_EINVAL, "unsupported (D, dobs)");
    if (N < 1) return fail(PARAPN_EINVAL, "N must be >= 1");
    if (!mu0 || !sqrt_sigma0 || !Phi || !sqrtQ || !H || !dvec || !mean_out)
        return fail(PARAPN_EINVAL, "NULL input or mean_out");
    const bool fp64 = precision == PARAPN_FP64;
    const int esz = fp64 ? 8 : 4;
    hipStream_t s = (hipStream_t)stream;
    PARAPN_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    const parapn::ScanPlan plan = default_plan(N);
    const Layout L = make_layout(D, N, esz, true, plan);
    int rc = ensure_ws(ctx, L.total);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    // initial-state record: mu0 followed by the canonical lower factor of Sigma0
    char *init = ws + L.off_consts;
    char *S0c = init + (size_t)D * esz;
    PARAPN_HIP(hipMemcpyAsync(init, mu0, (size_t)D * esz, hipMemcpyDeviceToDevice, s), "copy mu0");
    PARAPN_HIP(parapn::launch_tria_square(fp64, d, q, sqrt_sigma0, S0c, s), "canonicalise sqrt_sigma0");
    parapn::ModelDev m;
    m.Phi = Phi;
    m.sQ = sqrtQ;
    m.m0 = init;
    m.S0 = S0c;
    m.init = init;
    parapn::Work w{};
    w.traj = ws + L.off_traj;
    w.mf = ws + L.off_mf;
    w.sPf = ws + L.off_sPf;
    w.se = ws + L.off_se;
    w.sL = ws + L.off_sL;
    w.sPs = ws + L.off_sPs;
    w.filt_mf = (filt_mean_out || filt_sqrtcov_out) ? w.mf : nullptr;
    w.filt_sPf = (filt_mean_out || filt_sqrtcov_out) ? w.sPf : nullptr;
    w.fagg = ws + L.off_fagg;
    w.fpref = ws + L.off_fpref;
    w.sagg = ws + L.off_sagg;
    w.spref = ws + L.off_spref;
    w.dbits = (unsigned long long *)(ws + L.off_dbits);
    w.traj = nullptr;  // a given linear model: no trajectory, no prior offsets
    parapn::ObsSpec obs{};
    obs.mode = 1;
    obs.H = H;
    obs.dv = dvec;
    PARAPN_HIP(parapn::launch_forward(fp64, d, q, plan, m, obs, w, s), "forward scan");
    if (filt_mean_out || filt_sqrtcov_out)
        PARAPN_HIP(parapn::launch_unscale(fp64, D, N, nullptr, w.mf, w.sPf, filt_mean_out, filt_sqrtcov_out, s),
                   "filtered outputs");
    PARAPN_HIP(parapn::launch_smoother(fp64, d, q, plan, m, w, true, false, mean_out, 1.0, s), "reverse scan");
    if (sqrtcov_out)
        PARAPN_HIP(parapn::launch_unscale(fp64, D, N, nullptr, nullptr, w.sPs, nullptr, sqrtcov_out, s),
                   "smoothed factors");
    PARAPN_HIP(hipStreamSynchronize(s), "sync");
    return PARAPN_OK;
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
