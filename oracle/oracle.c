/*
 * Sequential FP64 reference for the parallel-in-time probabilistic ODE solver
 * (Bosch, Corenflos, Yaghoobi, Tronarp, Hennig, Saerkkae: "Parallel-in-Time
 * Probabilistic Numerical ODE Solvers", JMLR 25, 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, helper or constant
 * table with the HIP implementation.
 *
 * What it computes, and where the paper defines it:
 *   - IWP(q) transition Phi(h) and process noise Q(h) in closed form
 *     (Sec. 2.1, the display after the prior SDE).  The printed formula for
 *     Phi is garbled (an indicator 1_{i=j} with h^{i-j}); we use the standard
 *     reading [Phi]_ij = h^{j-i}/(j-i)! for j >= i (upper triangular).
 *   - The coordinate-change preconditioner named in Sec. 2.4 ("Preconditioned
 *     state transitions"): T = sqrt(h) diag(h^{q-i}/(q-i)!); all filtering is
 *     done on Ybar = T^{-1} Y.  The Dirac observation rows are divided by the
 *     scale of the first-derivative coordinate (exact: the data are noiseless).
 *   - Exact initialisation mu0 = [y0, y', ..., y^(q)] (eq. mu0) by truncated
 *     Taylor-series arithmetic, Sigma0 = 0.
 *   - EK1 linearisation H = E1 - F_y E0, d = f - F_y E0 eta (Sec. 3.2.1).
 *   - The smoother: what ParaRTS (Alg. 1) reaches exactly is the ordinary
 *     Kalman filter / Rauch-Tung-Striebel smoother; the oracle is that plain
 *     definition, run sequentially in square-root form with the tria operator
 *     of Sec. 3.1.2 (Householder LQ of the stacked factors).
 *   - The IEKS outer loop of Alg. 2: constant initial trajectory eta_n = mu0,
 *     linearise at every step, smooth, take the smoothed mean as the next
 *     trajectory, stop on the trajectory change.
 *   - For pins only: the square-root filtering elements (eq.
 *     sqrt-filtering-elements), the filtering operator (eq.
 *     sqrt-associative-filtering), the smoothing elements (eq.
 *     sqrt-smoothing-elements) and the smoothing operator (eq.
 *     sqrt-associative-smoothing), written from the paper's formulas.
 *
 * Conventions: row-major dense matrices; state index k = i*(q+1) + j for ODE
 * component i and derivative order j (the Kronecker ordering I_d (x) (q+1) of
 * Sec. 2.1); square-root factors are lower-triangular with a non-negative
 * diagonal.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small dense linear algebra                                                */
/* ------------------------------------------------------------------------ */

static double *dalloc(long n)
{
    double *p = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    return p;
}

/* C (n x m) = op(A) * op(B); op = transpose when the flag is set.
 * A is stored (ta ? k x n : n x k), B is stored (tb ? m x k : k x m). */
static void mm(int n, int m, int k, const double *A, int ta, const double *B, int tb, double *C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) {
                double a = ta ? A[l * n + i] : A[i * k + l];
                double b = tb ? B[j * k + l] : B[l * m + j];
                s += a * b;
            }
            C[i * m + j] = s;
        }
}

static void mv(int n, int k, const double *A, int ta, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int l = 0; l < k; ++l) s += (ta ? A[l * n + i] : A[i * k + l]) * x[l];
        y[i] = s;
    }
}

/* tria(M): for M (n x m) return lower-triangular L (n x n) with L L^T = M M^T.
 * Householder reflections act on the rows of M from the right (a QR of M^T),
 * then column signs are flipped so that diag(L) >= 0.  Columns of L beyond
 * min(n, m) are zero. */
void orc_tria(int n, int m, const double *M, double *L)
{
    int w = m > n ? m : n;
    double *W = dalloc((long)n * w);
    double *v = dalloc(w);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) W[r * w + c] = M[r * m + c];
    int kmax = n < m ? n : m;
    for (int k = 0; k < kmax; ++k) {
        double nrm2 = 0.0;
        for (int c = k; c < m; ++c) nrm2 += W[k * w + c] * W[k * w + c];
        double nrm = sqrt(nrm2);
        if (nrm == 0.0) continue;
        double x0 = W[k * w + k];
        double alpha = x0 >= 0.0 ? -nrm : nrm;
        for (int c = k; c < m; ++c) v[c] = W[k * w + c];
        v[k] -= alpha;
        double vv = 0.0;
        for (int c = k; c < m; ++c) vv += v[c] * v[c];
        if (vv == 0.0) continue;
        for (int r = k; r < n; ++r) {
            double s = 0.0;
            for (int c = k; c < m; ++c) s += W[r * w + c] * v[c];
            s = 2.0 * s / vv;
            for (int c = k; c < m; ++c) W[r * w + c] -= s * v[c];
        }
        W[k * w + k] = alpha;
        for (int c = k + 1; c < m; ++c) W[k * w + c] = 0.0;
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) L[r * n + c] = (c <= r && c < m) ? W[r * w + c] : 0.0;
    for (int c = 0; c < n; ++c)
        if (L[c * n + c] < 0.0)
            for (int r = c; r < n; ++r) L[r * n + c] = -L[r * n + c];
    free(W);
    free(v);
}

/* plain Cholesky of a symmetric positive-definite A (n x n) */
int orc_chol(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return -1;
        L[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    return 0;
}

/* X (r x n) = B (r x n) * L^{-1}, L lower-triangular n x n (solve X L = B) */
static void right_solve_lower(int r, int n, const double *L, const double *B, double *X)
{
    for (int i = 0; i < r; ++i)
        for (int j = n - 1; j >= 0; --j) {
            double s = B[i * n + j];
            for (int k = j + 1; k < n; ++k) s -= X[i * n + k] * L[k * n + j];
            X[i * n + j] = s / L[j * n + j];
        }
}

/* X (r x n) = B (r x n) * L^{-T}, L lower-triangular (solve X L^T = B) */
static void right_solve_lower_t(int r, int n, const double *L, const double *B, double *X)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < n; ++j) {
            double s = B[i * n + j];
            for (int k = 0; k < j; ++k) s -= X[i * n + k] * L[j * n + k];
            X[i * n + j] = s / L[j * n + j];
        }
}

/* x = L^{-1} b, L lower-triangular n x n */
static void lower_solve_vec(int n, const double *L, const double *b, double *x)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
        x[i] = s / L[i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* vector-field registry (oracle copy)                                      */
/* ------------------------------------------------------------------------ */

enum {
    ORC_LOGISTIC = 0,
    ORC_FHN = 1,
    ORC_LORENZ = 2,
    ORC_LV = 3,
    ORC_MOL = 4,
    ORC_AFFINE = 5,
    ORC_RIGID = 6,
    ORC_VDP = 7
};

/* number of ODE components, or -1 when the parameters do not fit */
int orc_field_dim(int field, int d_requested, int nparams)
{
    switch (field) {
    case ORC_LOGISTIC: return 1;
    case ORC_FHN: return nparams >= 3 ? 2 : -1;
    case ORC_LORENZ: return nparams >= 3 ? 3 : -1;
    case ORC_LV: return nparams >= 4 ? 2 : -1;
    case ORC_MOL: return (d_requested >= 3 && nparams >= 1) ? d_requested : -1;
    case ORC_AFFINE: return (d_requested >= 1 && nparams >= d_requested * d_requested + d_requested) ? d_requested : -1;
    case ORC_RIGID: return 3;
    case ORC_VDP: return nparams >= 1 ? 2 : -1;
    }
    return -1;
}

void orc_field_f(int field, const double *p, int d, const double *y, double *f)
{
    switch (field) {
    case ORC_LOGISTIC: f[0] = y[0] * (1.0 - y[0]); break;
    case ORC_FHN: {
        double a = p[0], b = p[1], c = p[2], V = y[0], R = y[1];
        f[0] = c * (V - V * V * V / 3.0 + R);
        f[1] = -(V - a + b * R) / c;
    } break;
    case ORC_LORENZ: {
        double s = p[0], r = p[1], be = p[2];
        f[0] = s * (y[1] - y[0]);
        f[1] = y[0] * (r - y[2]) - y[1];
        f[2] = y[0] * y[1] - be * y[2];
    } break;
    case ORC_LV: {
        double al = p[0], be = p[1], ga = p[2], de = p[3];
        f[0] = al * y[0] - be * y[0] * y[1];
        f[1] = de * y[0] * y[1] - ga * y[1];
    } break;
    case ORC_MOL: {
        double nu = p[0], dx = 1.0 / d, k = nu / (dx * dx);
        for (int i = 0; i < d; ++i) {
            double um = y[(i + d - 1) % d], up = y[(i + 1) % d], u = y[i];
            f[i] = k * (um - 2.0 * u + up) + u * (1.0 - u);
        }
    } break;
    case ORC_AFFINE:
        for (int i = 0; i < d; ++i) {
            double s = p[d * d + i];
            for (int j = 0; j < d; ++j) s += p[i * d + j] * y[j];
            f[i] = s;
        }
        break;
    case ORC_RIGID:
        f[0] = -2.0 * y[1] * y[2];
        f[1] = 1.25 * y[0] * y[2];
        f[2] = -0.5 * y[0] * y[1];
        break;
    case ORC_VDP: {
        double mu = p[0];
        f[0] = y[1];
        f[1] = mu * ((1.0 - y[0] * y[0]) * y[1] - y[0]);
    } break;
    }
}

/* Jacobian F_y (d x d, row-major) */
void orc_field_jac(int field, const double *p, int d, const double *y, double *J)
{
    memset(J, 0, sizeof(double) * d * d);
    switch (field) {
    case ORC_LOGISTIC: J[0] = 1.0 - 2.0 * y[0]; break;
    case ORC_FHN: {
        double b = p[1], c = p[2], V = y[0];
        J[0] = c * (1.0 - V * V);
        J[1] = c;
        J[2] = -1.0 / c;
        J[3] = -b / c;
    } break;
    case ORC_LORENZ: {
        double s = p[0], r = p[1], be = p[2];
        J[0] = -s; J[1] = s; J[2] = 0.0;
        J[3] = r - y[2]; J[4] = -1.0; J[5] = -y[0];
        J[6] = y[1]; J[7] = y[0]; J[8] = -be;
    } break;
    case ORC_LV: {
        double al = p[0], be = p[1], ga = p[2], de = p[3];
        J[0] = al - be * y[1]; J[1] = -be * y[0];
        J[2] = de * y[1]; J[3] = de * y[0] - ga;
    } break;
    case ORC_MOL: {
        double nu = p[0], dx = 1.0 / d, k = nu / (dx * dx);
        for (int i = 0; i < d; ++i) {
            J[i * d + (i + d - 1) % d] += k;
            J[i * d + (i + 1) % d] += k;
            J[i * d + i] += -2.0 * k + 1.0 - 2.0 * y[i];
        }
    } break;
    case ORC_AFFINE:
        for (int i = 0; i < d * d; ++i) J[i] = p[i];
        break;
    case ORC_RIGID:
        J[1] = -2.0 * y[2]; J[2] = -2.0 * y[1];
        J[3] = 1.25 * y[2]; J[5] = 1.25 * y[0];
        J[6] = -0.5 * y[1]; J[7] = -0.5 * y[0];
        break;
    case ORC_VDP: {
        double mu = p[0];
        J[1] = 1.0;
        J[2] = mu * (-2.0 * y[0] * y[1] - 1.0);
        J[3] = mu * (1.0 - y[0] * y[0]);
    } break;
    }
}

/* ------------------------------------------------------------------------ */
/* truncated Taylor arithmetic for mu0 (eq. mu0)                            */
/* ------------------------------------------------------------------------ */

/* coefficient K of the product of two series a, b (coefficients 0..K known) */
static double cauchy(const double *a, const double *b, int K)
{
    double s = 0.0;
    for (int j = 0; j <= K; ++j) s += a[j] * b[K - j];
    return s;
}

/* coefficient K of f(y(t)) where c[i*(Q+1)+k] is coefficient k of y_i;
 * only coefficients 0..K of y are read.  All registry fields are polynomial. */
static void taylor_f(int field, const double *p, int d, int Q, const double *c, int K, double *out)
{
    int S = Q + 1;
    switch (field) {
    case ORC_LOGISTIC: out[0] = c[K] - cauchy(c, c, K); break;
    case ORC_FHN: {
        double a = p[0], b = p[1], cc = p[2];
        const double *V = c, *R = c + S;
        double *V2 = dalloc(S);
        for (int j = 0; j <= K; ++j) V2[j] = cauchy(V, V, j);
        double V3 = cauchy(V2, V, K);
        out[0] = cc * (V[K] - V3 / 3.0 + R[K]);
        out[1] = -(V[K] - (K == 0 ? a : 0.0) + b * R[K]) / cc;
        free(V2);
    } break;
    case ORC_LORENZ: {
        double s = p[0], r = p[1], be = p[2];
        const double *x = c, *y = c + S, *z = c + 2 * S;
        out[0] = s * (y[K] - x[K]);
        out[1] = r * x[K] - cauchy(x, z, K) - y[K];
        out[2] = cauchy(x, y, K) - be * z[K];
    } break;
    case ORC_LV: {
        double al = p[0], be = p[1], ga = p[2], de = p[3];
        const double *x = c, *y = c + S;
        double xy = cauchy(x, y, K);
        out[0] = al * x[K] - be * xy;
        out[1] = de * xy - ga * y[K];
    } break;
    case ORC_MOL: {
        double nu = p[0], dx = 1.0 / d, k = nu / (dx * dx);
        for (int i = 0; i < d; ++i) {
            const double *u = c + i * S, *um = c + ((i + d - 1) % d) * S, *up = c + ((i + 1) % d) * S;
            out[i] = k * (um[K] - 2.0 * u[K] + up[K]) + u[K] - cauchy(u, u, K);
        }
    } break;
    case ORC_AFFINE:
        for (int i = 0; i < d; ++i) {
            double s = K == 0 ? p[d * d + i] : 0.0;
            for (int j = 0; j < d; ++j) s += p[i * d + j] * c[j * S + K];
            out[i] = s;
        }
        break;
    case ORC_RIGID: {
        const double *y1 = c, *y2 = c + S, *y3 = c + 2 * S;
        out[0] = -2.0 * cauchy(y2, y3, K);
        out[1] = 1.25 * cauchy(y1, y3, K);
        out[2] = -0.5 * cauchy(y1, y2, K);
    } break;
    case ORC_VDP: {
        double mu = p[0];
        const double *y1 = c, *y2 = c + S;
        double *y1s = dalloc(S);
        for (int j = 0; j <= K; ++j) y1s[j] = cauchy(y1, y1, j);
        out[0] = y2[K];
        out[1] = mu * (y2[K] - cauchy(y1s, y2, K) - y1[K]);
        free(y1s);
    } break;
    }
}

/* mu0 (D = d(q+1), state ordering) = [y0, y'(0), ..., y^(q)(0)] per component */
void orc_taylor_mu0(int field, const double *p, int d, const double *y0, int q, double *mu0)
{
    int S = q + 1;
    double *c = dalloc((long)d * S);
    double *fk = dalloc(d);
    for (int i = 0; i < d; ++i) c[i * S] = y0[i];
    for (int K = 0; K < q; ++K) {
        taylor_f(field, p, d, q, c, K, fk);
        for (int i = 0; i < d; ++i) c[i * S + K + 1] = fk[i] / (double)(K + 1);
    }
    for (int i = 0; i < d; ++i) {
        double fact = 1.0;
        for (int j = 0; j <= q; ++j) {
            if (j > 0) fact *= j;
            mu0[i * S + j] = fact * c[i * S + j];
        }
    }
    free(c);
    free(fk);
}

/* ------------------------------------------------------------------------ */
/* IWP(q) prior and preconditioner (Sec. 2.1, Sec. 2.4)                      */
/* ------------------------------------------------------------------------ */

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* one-dimensional (q+1) x (q+1) blocks Phi(h), Q(h) in original coordinates */
void orc_iwp(int q, double h, double *Phi, double *Q)
{
    int S = q + 1;
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) {
            Phi[i * S + j] = j >= i ? pow(h, j - i) / factorial(j - i) : 0.0;
            int e = 2 * q + 1 - i - j;
            Q[i * S + j] = pow(h, e) / (e * factorial(q - i) * factorial(q - j));
        }
}

/* exp(A) for a small n x n matrix: scaling and squaring of the Taylor series */
static void expm_taylor(int n, const double *A, double *E)
{
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += fabs(A[i * n + j]);
        if (r > nrm) nrm = r;
    }
    int sq = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++sq;
    }
    double sc = ldexp(1.0, -sq);
    double *term = dalloc(n * n), *tmp = dalloc(n * n);
    for (int i = 0; i < n * n; ++i) {
        E[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
        term[i] = E[i];
    }
    for (int k = 1; k <= 24; ++k) {
        /* term <- term * (sc A) / k */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int l = 0; l < n; ++l) t += term[i * n + l] * A[l * n + j];
                tmp[i * n + j] = t * sc / k;
            }
        for (int i = 0; i < n * n; ++i) {
            term[i] = tmp[i];
            E[i] += term[i];
        }
    }
    for (int r = 0; r < sq; ++r) {
        mm(n, n, n, E, 0, E, 0, tmp);
        memcpy(E, tmp, sizeof(double) * n * n);
    }
    free(term);
    free(tmp);
}

/* Blocks of a prior whose derivatives 0..q follow X_i' = X_{i+1} (i < q) and
 * dX_q = sum_k c_k X_k dt + dW (the alternative Gauss-Markov priors of
 * Sec. 2.1).  Drift F: F[i][i+1] = 1, F[q][k] = c_k.  Phi = exp(F h);
 * Q = int_0^h exp(F s) e_q e_q^T exp(F s)^T ds, by composite 5-point
 * Gauss-Legendre quadrature over 64 panels (the integrand is smooth). */
static void lti_prior(int q, const double *c, double h, double *Phi, double *Q)
{
    int S = q + 1;
    double *F = dalloc(S * S), *A = dalloc(S * S), *E = dalloc(S * S);
    memset(F, 0, sizeof(double) * S * S);
    for (int i = 0; i < q; ++i) F[i * S + i + 1] = 1.0;
    for (int k = 0; k <= q; ++k) F[q * S + k] = c[k];
    for (int i = 0; i < S * S; ++i) A[i] = F[i] * h;
    expm_taylor(S, A, Phi);
    static const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                                 0.9061798459386640};
    static const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                                 0.2369268850561891};
    const int panels = 64;
    memset(Q, 0, sizeof(double) * S * S);
    double ph = h / panels;
    for (int p = 0; p < panels; ++p)
        for (int g = 0; g < 5; ++g) {
            double s = ph * (p + 0.5 + 0.5 * gx[g]);
            for (int i = 0; i < S * S; ++i) A[i] = F[i] * s;
            expm_taylor(S, A, E);
            /* column q of exp(F s) */
            for (int i = 0; i < S; ++i)
                for (int j = 0; j < S; ++j) Q[i * S + j] += 0.5 * ph * gw[g] * E[i * S + q] * E[j * S + q];
        }
    free(F); free(A); free(E);
}

/* Integrated Ornstein-Uhlenbeck prior IOUP(q, theta): dX_q = -theta X_q dt + dW.
 * theta = 0 is the integrated Wiener process. */
void orc_ioup(int q, double theta, double h, double *Phi, double *Q)
{
    double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    c[q] = -theta;
    lti_prior(q, c, h, Phi, Q);
}

/* Matern prior of smoothness nu = q + 1/2 and length scale ell: the
 * stationary process whose spectral density is proportional to
 * (lambda^2 + w^2)^-(q+1), lambda = sqrt(2 nu) / ell, i.e. the drift's
 * characteristic polynomial is (s + lambda)^(q+1):
 * c_k = -binom(q+1, k) lambda^(q+1-k).  Unit diffusion, as for the IWP. */
void orc_matern(int q, double ell, double h, double *Phi, double *Q)
{
    double lam = sqrt(2.0 * q + 1.0) / ell, c[5];
    for (int k = 0; k <= q; ++k) {
        double b = 1.0;
        for (int j = 1; j <= k; ++j) b = b * (q + 2 - j) / j;  /* binom(q+1, k) */
        c[k] = -b * pow(lam, q + 1 - k);
    }
    lti_prior(q, c, h, Phi, Q);
}

/* one-dimensional prior blocks: 0 IWP(q), 1 IOUP(q, theta), 2 Matern(q + 1/2,
 * length scale theta) */
static void prior_blocks_1d(int q, double h, int prior, double theta, double *Ph, double *Qh)
{
    if (prior == 1)
        orc_ioup(q, theta, h, Ph, Qh);
    else if (prior == 2)
        orc_matern(q, theta, h, Ph, Qh);
    else
        orc_iwp(q, h, Ph, Qh);
}

/* diagonal of the one-dimensional preconditioner T(h) */
void orc_precond_diag(int q, double h, double *T)
{
    for (int i = 0; i <= q; ++i) T[i] = sqrt(h) * pow(h, q - i) / factorial(q - i);
}

/* preconditioned full-state transition and process-noise square root:
 * Phibar = T^{-1} Phi T, Qbar = T^{-1} Q T^{-T}, sqrtQbar = chol(Qbar),
 * all D x D with D = d(q+1), block-diagonal (I_d (x) block). */
static void precond_model_prior(int d, int q, double h, int prior, double theta, double *PhiB, double *sQB,
                                double *Tfull)
{
    int S = q + 1, D = d * S;
    double *Ph = dalloc(S * S), *Qh = dalloc(S * S), *T = dalloc(S);
    double *Pb = dalloc(S * S), *Qb = dalloc(S * S), *Lb = dalloc(S * S);
    prior_blocks_1d(q, h, prior, theta, Ph, Qh);
    orc_precond_diag(q, h, T);
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) {
            Pb[i * S + j] = Ph[i * S + j] * T[j] / T[i];
            Qb[i * S + j] = Qh[i * S + j] / (T[i] * T[j]);
        }
    orc_chol(S, Qb, Lb);
    memset(PhiB, 0, sizeof(double) * D * D);
    memset(sQB, 0, sizeof(double) * D * D);
    for (int k = 0; k < d; ++k)
        for (int i = 0; i < S; ++i) {
            Tfull[k * S + i] = T[i];
            for (int j = 0; j < S; ++j) {
                PhiB[(k * S + i) * D + k * S + j] = Pb[i * S + j];
                sQB[(k * S + i) * D + k * S + j] = Lb[i * S + j];
            }
        }
    free(Ph); free(Qh); free(T); free(Pb); free(Qb); free(Lb);
}

static void precond_model(int d, int q, double h, double *PhiB, double *sQB, double *Tfull)
{
    precond_model_prior(d, q, h, 0, 0.0, PhiB, sQB, Tfull);
}

/* ------------------------------------------------------------------------ */
/* sequential square-root Kalman filter + RTS smoother on a linear model     */
/* ------------------------------------------------------------------------ */

/* Linear-Gaussian model of eq. affine-estimation with constant Phi, sqrtQ:
 *   Y0 ~ N(mu0, S0 S0^T), Y_n = Phi Y_{n-1} + w, w ~ N(0, sqrtQ sqrtQ^T),
 *   H_n Y_n = dv_n exactly (zero observation noise), n = 1..N.
 * H is [N][dobs][D], dv is [N][dobs].  Outputs are [N+1] stacks; row 0 holds
 * (mu0, S0) for the filter.  Smoothed marginals include n = 0 (conditioned on
 * all data).  Returns 0, or -4 when a non-finite value appears. */
/* Observation rows may carry independent noise: rstd[r] is the standard
 * deviation of row r (NULL or 0: noiseless).  The update factor then comes
 * from tria([[H sqrtP-, diag(rstd)], [sqrtP-, 0]]). */
/* qf (may be NULL) receives the sum over n of the innovations' quadratic
 * forms r_n^T S_n^-1 r_n, r_n = d_n - H_n m-_n, S_n = Psi11 Psi11^T: the
 * prediction-error decomposition of the data's log-likelihood, whose
 * maximiser over the diffusion sigma^2 is qf / (N dobs) (the quasi-maximum-
 * likelihood calibration of Sec. 2.4; every covariance scales with sigma^2). */
/* Step n (1..N) takes its transition and process-noise factor from
 * Phi + (n-1) pstride and sqrtQ + (n-1) pstride: pstride 0 is a constant model,
 * D*D a time-varying one (eq. affine-estimation with Phi_n, Q_n). */
static int kf_rts_core(int D, int dobs, long N, const double *mu0, const double *S0, const double *Phi0,
                       const double *sqrtQ0, long pstride, const double *H, const double *dv, const double *rstd,
                       double *mf, double *sPf, double *ms, double *sPs, double *qf)
{
    int n2 = dobs + D;
    double *mp = dalloc(D), *sPp = dalloc(D * D), *M = dalloc((long)n2 * n2), *Psi = dalloc((long)n2 * n2);
    double *W = dalloc(2L * D * 2 * D), *Pi = dalloc(4L * D * D);
    double *tmp = dalloc(D * D), *K = dalloc((long)D * dobs), *res = dalloc(dobs), *Ps11 = dalloc(dobs * dobs);
    double *Ps21 = dalloc((long)D * dobs), *E = dalloc(D * D), *v = dalloc(D), *v2 = dalloc(D);
    int bad = 0;
    memcpy(mf, mu0, sizeof(double) * D);
    memcpy(sPf, S0, sizeof(double) * D * D);
    for (long n = 1; n <= N; ++n) {
        const double *m = mf + (n - 1) * D, *sP = sPf + (n - 1) * D * D;
        const double *Hn = H + (n - 1) * dobs * D, *dn = dv + (n - 1) * dobs;
        const double *Phi = Phi0 + (n - 1) * pstride, *sqrtQ = sqrtQ0 + (n - 1) * pstride;
        /* predict: m- = Phi m, sqrtP- = tria([Phi sqrtP, sqrtQ]) */
        mv(D, D, Phi, 0, m, mp);
        mm(D, D, D, Phi, 0, sP, 0, tmp);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                W[r * 2 * D + c] = tmp[r * D + c];
                W[r * 2 * D + D + c] = sqrtQ[r * D + c];
            }
        orc_tria(D, 2 * D, W, sPp);
        /* update: Psi = tria([[H sqrtP-, 0], [sqrtP-, 0]]) */
        memset(M, 0, sizeof(double) * n2 * n2);
        mm(dobs, D, D, Hn, 0, sPp, 0, tmp);
        for (int r = 0; r < dobs; ++r) {
            for (int c = 0; c < D; ++c) M[r * n2 + c] = tmp[r * D + c];
            M[r * n2 + D + r] = rstd ? rstd[r] : 0.0;
        }
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) M[(dobs + r) * n2 + c] = sPp[r * D + c];
        orc_tria(n2, n2, M, Psi);
        for (int r = 0; r < dobs; ++r)
            for (int c = 0; c < dobs; ++c) Ps11[r * dobs + c] = Psi[r * n2 + c];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < dobs; ++c) Ps21[r * dobs + c] = Psi[(dobs + r) * n2 + c];
        right_solve_lower(D, dobs, Ps11, Ps21, K); /* K = Psi21 Psi11^{-1} */
        mv(dobs, D, Hn, 0, mp, res);
        for (int r = 0; r < dobs; ++r) res[r] = dn[r] - res[r];
        if (qf) {
            double *x = dalloc(dobs);
            lower_solve_vec(dobs, Ps11, res, x);
            for (int r = 0; r < dobs; ++r) *qf += x[r] * x[r];
            free(x);
        }
        double *mo = mf + n * D, *so = sPf + n * D * D;
        mv(D, dobs, K, 0, res, v);
        for (int r = 0; r < D; ++r) mo[r] = mp[r] + v[r];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) so[r * D + c] = Psi[(dobs + r) * n2 + dobs + c];
        for (int r = 0; r < D; ++r)
            if (!isfinite(mo[r])) bad = 1;
    }
    /* RTS backward pass */
    memcpy(ms + N * D, mf + N * D, sizeof(double) * D);
    memcpy(sPs + N * D * D, sPf + N * D * D, sizeof(double) * D * D);
    for (long n = N - 1; n >= 0; --n) {
        const double *m = mf + n * D, *sP = sPf + n * D * D;
        const double *Phi = Phi0 + n * pstride, *sqrtQ = sqrtQ0 + n * pstride; /* step n+1 */
        /* Pi = tria([[Phi sqrtPf, sqrtQ], [sqrtPf, 0]]) */
        memset(W, 0, sizeof(double) * 4 * D * D);
        mm(D, D, D, Phi, 0, sP, 0, tmp);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                W[r * 2 * D + c] = tmp[r * D + c];
                W[r * 2 * D + D + c] = sqrtQ[r * D + c];
                W[(D + r) * 2 * D + c] = sP[r * D + c];
            }
        orc_tria(2 * D, 2 * D, W, Pi);
        /* E = Pi21 Pi11^{-1} */
        double *P11 = dalloc(D * D), *P21 = dalloc(D * D), *P22 = dalloc(D * D);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                P11[r * D + c] = Pi[r * 2 * D + c];
                P21[r * D + c] = Pi[(D + r) * 2 * D + c];
                P22[r * D + c] = Pi[(D + r) * 2 * D + D + c];
            }
        right_solve_lower(D, D, P11, P21, E);
        /* m^s_n = m^f_n + E (m^s_{n+1} - Phi m^f_n) */
        mv(D, D, Phi, 0, m, v);
        for (int r = 0; r < D; ++r) v[r] = ms[(n + 1) * D + r] - v[r];
        mv(D, D, E, 0, v, v2);
        for (int r = 0; r < D; ++r) ms[n * D + r] = m[r] + v2[r];
        /* sqrtP^s_n = tria([E sqrtP^s_{n+1}, Pi22]) */
        mm(D, D, D, E, 0, sPs + (n + 1) * D * D, 0, tmp);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                W[r * 2 * D + c] = tmp[r * D + c];
                W[r * 2 * D + D + c] = P22[r * D + c];
            }
        orc_tria(D, 2 * D, W, sPs + n * D * D);
        for (int r = 0; r < D; ++r)
            if (!isfinite(ms[n * D + r])) bad = 1;
        free(P11); free(P21); free(P22);
    }
    free(mp); free(sPp); free(M); free(Psi); free(W); free(Pi); free(tmp); free(K); free(res);
    free(Ps11); free(Ps21); free(E); free(v); free(v2);
    return bad ? -4 : 0;
}

int orc_kf_rts_noise(int D, int dobs, long N, const double *mu0, const double *S0, const double *Phi,
                     const double *sqrtQ, const double *H, const double *dv, const double *rstd, double *mf,
                     double *sPf, double *ms, double *sPs)
{
    return kf_rts_core(D, dobs, N, mu0, S0, Phi, sqrtQ, 0, H, dv, rstd, mf, sPf, ms, sPs, NULL);
}

int orc_kf_rts(int D, int dobs, long N, const double *mu0, const double *S0, const double *Phi,
               const double *sqrtQ, const double *H, const double *dv, double *mf, double *sPf,
               double *ms, double *sPs)
{
    return kf_rts_core(D, dobs, N, mu0, S0, Phi, sqrtQ, 0, H, dv, NULL, mf, sPf, ms, sPs, NULL);
}

/* the sequential filter/smoother of a time-varying model: Phi, sqrtQ are
 * [N][D][D], step n using entry n-1 */
int orc_kf_rts_tv(int D, int dobs, long N, const double *mu0, const double *S0, const double *Phi,
                  const double *sqrtQ, const double *H, const double *dv, double *mf, double *sPf, double *ms,
                  double *sPs)
{
    return kf_rts_core(D, dobs, N, mu0, S0, Phi, sqrtQ, (long)D * D, H, dv, NULL, mf, sPf, ms, sPs, NULL);
}

/* the noiseless filter/smoother and the innovations' quadratic-form sum */
int orc_kf_rts_qf(int D, int dobs, long N, const double *mu0, const double *S0, const double *Phi,
                  const double *sqrtQ, const double *H, const double *dv, double *mf, double *sPf, double *ms,
                  double *sPs, double *qf)
{
    *qf = 0.0;
    return kf_rts_core(D, dobs, N, mu0, S0, Phi, sqrtQ, 0, H, dv, NULL, mf, sPf, ms, sPs, qf);
}

/* ------------------------------------------------------------------------ */
/* objective value (eq. objective-value)                                     */
/* ------------------------------------------------------------------------ */

/* V(eta) = 1/2 sum_{n=1}^N |eta_n - Phi eta_{n-1}|^2_{Q^-1} for a trajectory
 * traj [N+1][D] in original coordinates (the negative log-density of the
 * trajectory under the prior, up to a constant), Phi = Phi(h), Q = Q(h) of the
 * IWP(q), IOUP(q, theta) or Matern(q + 1/2, length scale theta) prior per ODE
 * component.  The residual is formed in
 * original coordinates; the weighted norm is taken as |L^-1 T^-1 r|^2 with
 * T = T(h) and L = chol(T^-1 Q T^-T) (Q(h) itself spans too many orders of
 * magnitude for a plain Cholesky at small h). */
double orc_objective(int d, int q, double h, long N, const double *traj, int prior, double theta)
{
    int S = q + 1, D = d * S;
    double *Ph = dalloc(S * S), *Qh = dalloc(S * S), *T = dalloc(S), *Qb = dalloc(S * S), *L = dalloc(S * S);
    double *r = dalloc(S), *w = dalloc(S);
    prior_blocks_1d(q, h, prior, theta, Ph, Qh);
    orc_precond_diag(q, h, T);
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) Qb[i * S + j] = Qh[i * S + j] / (T[i] * T[j]);
    orc_chol(S, Qb, L);
    double V = 0.0;
    for (long n = 1; n <= N; ++n)
        for (int c = 0; c < d; ++c) {
            const double *a = traj + (n - 1) * D + c * S, *b = traj + n * D + c * S;
            for (int i = 0; i < S; ++i) {
                double t = b[i];
                for (int j = 0; j < S; ++j) t -= Ph[i * S + j] * a[j];
                r[i] = t / T[i];
            }
            lower_solve_vec(S, L, r, w);
            for (int i = 0; i < S; ++i) V += 0.5 * w[i] * w[i];
        }
    free(Ph); free(Qh); free(T); free(Qb); free(L); free(r); free(w);
    return V;
}

/* ------------------------------------------------------------------------ */
/* IEKS (Alg. 2) with the sequential smoother                                */
/* ------------------------------------------------------------------------ */

/* Solves one IVP.  mean_out is [N+1][D], sqrtcov_out [N+1][D][D] (or NULL),
 * both in original coordinates; row 0 is (mu0, 0).  init_traj, when given, is
 * an [N+1][D] starting trajectory in original coordinates (the paper's choice,
 * used when it is NULL, is the constant mu0).  fixed_iters > 0 runs exactly
 * that many iterations; otherwise the loop stops once
 *   delta_k = max_n max_i |E0 (mu^(k)_n - mu^(k-1)_n)|_i  <  tol
 * or after max_iter iterations.  delta_hist[k-1] receives delta_k.
 * Returns 0 (converged or fixed count done), 1 (iteration cap), -1 (bad
 * arguments) or -4 (non-finite values). */
/* Alg. 2, optionally damped: lm_sigma > 0 adds to every step n >= 1 the
 * pseudo-observation E0 Y_n = E0 (current iterate)_n with standard deviation
 * lm_sigma / sqrt(h) per coordinate in the units of y (Levenberg-Marquardt
 * damping of the Gauss-Newton step, which the paper leaves as future work;
 * the fixed point is unchanged).  When damped, the returned factors come
 * from one more, undamped linearise-and-smooth pass at the final iterate. */
/* Approximate Jacobians (remark on linearizing with approximate Jacobians,
 * Sec. 3.2.1): lin 1 = EK0, F_y ~ 0; lin 2 = DiagonalEK1, F_y ~ diag(F_y);
 * lin 0 = EK1 (the exact Jacobian, unchanged). */
static void approx_jacobian(int lin, int d, double *J)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (lin == 1 || (lin == 2 && i != j)) J[i * d + j] = 0.0;
}

/* Alg. 2 with the prior of choice: prior 0 = IWP(q), 1 = IOUP(q, theta),
 * 2 = Matern(q + 1/2, length scale theta), and
 * the paper's stopping criteria (Sec. 3.2.2): stop_rule bit 0 -- the
 * trajectory change delta_k < tol; bit 1 -- the change of the objective value
 * (eq. objective-value) |V_k - V_{k-1}| <= obj_atol + obj_rtol |V_k|, with V_0
 * the objective of the starting trajectory; either met stops the loop.
 * obj_hist[k-1] receives V_k (may be NULL), *obj0 V_0 (may be NULL).
 * *sigma2 (may be NULL) receives the quasi-maximum-likelihood diffusion of
 * the last undamped filter pass (its innovations' quadratic forms over N d;
 * NaN when every pass was damped). */
int orc_ieks_ext(int field, const double *params, int nparams, int d_req, const double *y0, double t0, double t1,
                 int q, long N, int max_iter, double tol, int fixed_iters, const double *init_traj,
                 double lm_sigma, int prior, double theta, int stop_rule, double obj_atol, double obj_rtol,
                 int lin, double *mean_out, double *sqrtcov_out, double *delta_hist, double *obj_hist, double *obj0,
                 double *sigma2, int *iters_out)
{
    int d = orc_field_dim(field, d_req, nparams);
    if (d < 1 || q < 1 || N < 1 || !(t1 > t0)) return -1;
    int S = q + 1, D = d * S;
    double h = (t1 - t0) / (double)N;
    double *PhiB = dalloc(D * D), *sQB = dalloc(D * D), *T = dalloc(D);
    precond_model_prior(d, q, h, prior, theta, PhiB, sQB, T);
    double *mu0 = dalloc(D), *mu0b = dalloc(D);
    orc_taylor_mu0(field, params, d, y0, q, mu0);
    for (int k = 0; k < D; ++k) mu0b[k] = mu0[k] / T[k];
    double *eta = dalloc((N + 1) * D);
    for (long n = 0; n <= N; ++n)
        for (int k = 0; k < D; ++k) eta[n * D + k] = init_traj ? init_traj[n * D + k] / T[k] : mu0b[k];
    const int lm = lm_sigma > 0.0;
    const int dobs = lm ? 2 * d : d;
    double *H = dalloc(N * dobs * D), *dv = dalloc(N * dobs), *rstd = dalloc(dobs);
    double *mf = dalloc((N + 1) * D), *sPf = dalloc((N + 1) * D * D);
    double *ms = dalloc((N + 1) * D), *sPs = dalloc((N + 1) * D * D);
    double *S0 = dalloc(D * D), *y = dalloc(d), *fy = dalloc(d), *Jy = dalloc(d * d);
    /* scales: E0 coordinate T[i*S+0], E1 coordinate T[i*S+1] (same for all i) */
    double T0 = T[0], T1 = T[1];
    for (int r = 0; r < dobs; ++r) rstd[r] = r < d ? 0.0 : lm_sigma / (sqrt(h) * T0);
    int status = 0, k = 0;
    int limit = fixed_iters > 0 ? fixed_iters : max_iter;
    double *traj_o = dalloc((N + 1) * D), qf = 0.0, s2 = NAN;
    for (long n = 0; n <= N; ++n)
        for (int r = 0; r < D; ++r) traj_o[n * D + r] = T[r] * eta[n * D + r];
    double Vprev = orc_objective(d, q, h, N, traj_o, prior, theta);
    if (obj0) *obj0 = Vprev;
    for (k = 1; k <= limit; ++k) {
        /* EK1 linearisation at every grid point (Sec. 3.2.1), then the
         * preconditioned observation  (H T) Ybar = d  with rows divided by T1:
         *   Hbar = E1 - (T0/T1) F_y E0,   dbar = (f - F_y y) / T1 */
        memset(H, 0, sizeof(double) * N * dobs * D);
        for (long n = 1; n <= N; ++n) {
            for (int i = 0; i < d; ++i) y[i] = T0 * eta[n * D + i * S];
            orc_field_f(field, params, d, y, fy);
            orc_field_jac(field, params, d, y, Jy);
            approx_jacobian(lin, d, Jy);
            double *Hn = H + (n - 1) * dobs * D, *dn = dv + (n - 1) * dobs;
            for (int i = 0; i < d; ++i) {
                double s = fy[i];
                for (int j = 0; j < d; ++j) s -= Jy[i * d + j] * y[j];
                dn[i] = s / T1;
                Hn[i * D + i * S + 1] += 1.0;
                for (int j = 0; j < d; ++j) Hn[i * D + j * S] -= Jy[i * d + j] * T0 / T1;
            }
            for (int i = 0; i < d && lm; ++i) { /* damping rows: E0 Y_n = E0 eta_n */
                Hn[(d + i) * D + i * S] = 1.0;
                dn[d + i] = eta[n * D + i * S];
            }
        }
        qf = 0.0;
        int rc = kf_rts_core(D, dobs, N, mu0b, S0, PhiB, sQB, 0, H, dv, rstd, mf, sPf, ms, sPs, lm ? NULL : &qf);
        if (!lm) s2 = qf / ((double)N * d);
        double delta = 0.0;
        for (long n = 0; n <= N; ++n)
            for (int i = 0; i < d; ++i) {
                double a = fabs(T0 * (ms[n * D + i * S] - eta[n * D + i * S]));
                if (!(a <= delta)) delta = a; /* also propagates NaN */
            }
        if (delta_hist) delta_hist[k - 1] = delta;
        memcpy(eta, ms, sizeof(double) * (N + 1) * D);
        for (long n = 0; n <= N; ++n)
            for (int r = 0; r < D; ++r) traj_o[n * D + r] = T[r] * eta[n * D + r];
        double V = orc_objective(d, q, h, N, traj_o, prior, theta);
        if (obj_hist) obj_hist[k - 1] = V;
        if (rc != 0 || !isfinite(delta)) { status = -4; break; }
        int stop_traj = (stop_rule & 1) && delta < tol;
        int stop_obj = (stop_rule & 2) && fabs(V - Vprev) <= obj_atol + obj_rtol * fabs(V);
        Vprev = V;
        if (fixed_iters <= 0 && (stop_traj || stop_obj)) { status = 0; break; }
        if (fixed_iters <= 0 && k == max_iter) { status = 1; break; }
    }
    free(traj_o);
    if (k > limit) k = limit;
    if (iters_out) *iters_out = k;
    if (lm && sqrtcov_out && status != -4) {
        /* factors of the undamped model linearised at the final iterate */
        double *msk = dalloc((N + 1) * D);
        memcpy(msk, ms, sizeof(double) * (N + 1) * D);
        memset(H, 0, sizeof(double) * N * dobs * D);
        for (long n = 1; n <= N; ++n) {
            for (int i = 0; i < d; ++i) y[i] = T0 * eta[n * D + i * S];
            orc_field_f(field, params, d, y, fy);
            orc_field_jac(field, params, d, y, Jy);
            approx_jacobian(lin, d, Jy);
            double *Hn = H + (n - 1) * d * D, *dn = dv + (n - 1) * d;
            for (int i = 0; i < d; ++i) {
                double s = fy[i];
                for (int j = 0; j < d; ++j) s -= Jy[i * d + j] * y[j];
                dn[i] = s / T1;
                Hn[i * D + i * S + 1] += 1.0;
                for (int j = 0; j < d; ++j) Hn[i * D + j * S] -= Jy[i * d + j] * T0 / T1;
            }
        }
        qf = 0.0;
        kf_rts_core(D, d, N, mu0b, S0, PhiB, sQB, 0, H, dv, NULL, mf, sPf, ms, sPs, &qf);
        s2 = qf / ((double)N * d);
        memcpy(ms, msk, sizeof(double) * (N + 1) * D);
        free(msk);
    }
    for (long n = 0; n <= N; ++n)
        for (int r = 0; r < D; ++r) {
            mean_out[n * D + r] = T[r] * ms[n * D + r];
            if (sqrtcov_out)
                for (int c = 0; c < D; ++c) sqrtcov_out[(n * D + r) * D + c] = T[r] * sPs[(n * D + r) * D + c];
        }
    if (sigma2) *sigma2 = s2;
    free(PhiB); free(sQB); free(T); free(mu0); free(mu0b); free(eta); free(H); free(dv); free(rstd);
    free(mf); free(sPf); free(ms); free(sPs); free(S0); free(y); free(fy); free(Jy);
    return status;
}

int orc_ieks_prior(int field, const double *params, int nparams, int d_req, const double *y0, double t0, double t1,
                   int q, long N, int max_iter, double tol, int fixed_iters, const double *init_traj,
                   double lm_sigma, int prior, double theta, double *mean_out, double *sqrtcov_out,
                   double *delta_hist, int *iters_out)
{
    return orc_ieks_ext(field, params, nparams, d_req, y0, t0, t1, q, N, max_iter, tol, fixed_iters, init_traj,
                        lm_sigma, prior, theta, 1, 0.0, 0.0, 0, mean_out, sqrtcov_out, delta_hist, NULL, NULL, NULL,
                        iters_out);
}

/* preconditioned model constants, exposed for pins: PhiB, sqrtQB (D x D), T (D) */
void orc_precond_model(int d, int q, double h, double *PhiB, double *sQB, double *T)
{
    precond_model(d, q, h, PhiB, sQB, T);
}

/* ------------------------------------------------------------------------ */
/* paper-form elements and associative operators (pins only)                */
/* ------------------------------------------------------------------------ */

/* Square-root filtering element (eq. sqrt-filtering-elements), noiseless
 * observation (sqrt R = 0).  (m_prev, sP_prev) are m_{n-1}, sqrtP_{n-1} of the
 * element construction: (mu0, sqrtSigma0) for n = 1 and zero for n >= 2.  For
 * n = 1 ("first") the element is p(Y1 | Z1) and does not depend on Y0, so
 * A = 0, eta = 0, sqrtJ = 0.  sqrtJ is stored D x D with columns >= dobs zero. */
void orc_filter_element(int D, int dobs, const double *Phi, const double *sqrtQ, const double *H,
                        const double *dv, const double *m_prev, const double *sP_prev, int first,
                        double *A, double *b, double *sC, double *eta, double *sJ)
{
    int n2 = dobs + D;
    double *mp = dalloc(D), *W = dalloc(2L * D * D), *sPp = dalloc(D * D), *tmp = dalloc((long)n2 * D);
    double *M = dalloc((long)n2 * n2), *Psi = dalloc((long)n2 * n2), *P11 = dalloc(dobs * dobs);
    double *P21 = dalloc((long)D * dobs), *K = dalloc((long)D * dobs), *res = dalloc(dobs), *KH = dalloc(D * D);
    double *IKH = dalloc(D * D), *HP = dalloc((long)dobs * D), *sJd = dalloc((long)D * dobs), *u = dalloc(dobs);
    mv(D, D, Phi, 0, m_prev, mp);
    mm(D, D, D, Phi, 0, sP_prev, 0, tmp);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            W[r * 2 * D + c] = tmp[r * D + c];
            W[r * 2 * D + D + c] = sqrtQ[r * D + c];
        }
    orc_tria(D, 2 * D, W, sPp);
    mm(dobs, D, D, H, 0, sPp, 0, HP);
    for (int r = 0; r < dobs; ++r)
        for (int c = 0; c < D; ++c) M[r * n2 + c] = HP[r * D + c];
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) M[(dobs + r) * n2 + c] = sPp[r * D + c];
    orc_tria(n2, n2, M, Psi);
    for (int r = 0; r < dobs; ++r)
        for (int c = 0; c < dobs; ++c) P11[r * dobs + c] = Psi[r * n2 + c];
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < dobs; ++c) P21[r * dobs + c] = Psi[(dobs + r) * n2 + c];
    right_solve_lower(D, dobs, P11, P21, K);
    /* A = (I - K H) Phi */
    mm(D, D, dobs, K, 0, H, 0, KH);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) IKH[r * D + c] = (r == c ? 1.0 : 0.0) - KH[r * D + c];
    mm(D, D, D, IKH, 0, Phi, 0, A);
    /* b = m- - K (H m- - d) */
    mv(dobs, D, H, 0, mp, res);
    for (int r = 0; r < dobs; ++r) res[r] -= dv[r];
    mv(D, dobs, K, 0, res, b);
    for (int r = 0; r < D; ++r) b[r] = mp[r] - b[r];
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) sC[r * D + c] = Psi[(dobs + r) * n2 + dobs + c];
    /* sqrtJ = Phi^T H^T Psi11^{-T}  (D x dobs);  eta = sqrtJ Psi11^{-1} d */
    double *PtHt = dalloc((long)D * dobs);
    mm(D, dobs, D, Phi, 1, H, 1, PtHt);
    right_solve_lower_t(D, dobs, P11, PtHt, sJd);
    lower_solve_vec(dobs, P11, dv, u);
    mv(D, dobs, sJd, 0, u, eta);
    memset(sJ, 0, sizeof(double) * D * D);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < dobs; ++c) sJ[r * D + c] = sJd[r * dobs + c];
    if (first) {
        memset(A, 0, sizeof(double) * D * D);
        memset(eta, 0, sizeof(double) * D);
        memset(sJ, 0, sizeof(double) * D * D);
    }
    free(mp); free(W); free(sPp); free(tmp); free(M); free(Psi); free(P11); free(P21); free(K); free(res);
    free(KH); free(IKH); free(HP); free(sJd); free(u); free(PtHt);
}

/* Filtering operator a_ij = a_i (x)_f a_j, i earlier (eq.
 * sqrt-associative-filtering), with
 *   Xi = tria([[sqrtC_i^T sqrtJ_j, I], [sqrtJ_j, 0]])  (2D x 2D).
 * Output buffers may not alias the inputs. */
void orc_filter_combine(int D, const double *Ai, const double *bi, const double *sCi, const double *etai,
                        const double *sJi, const double *Aj, const double *bj, const double *sCj,
                        const double *etaj, const double *sJj, double *A, double *b, double *sC,
                        double *eta, double *sJ)
{
    int D2 = 2 * D;
    double *M = dalloc((long)D2 * D2), *Xi = dalloc((long)D2 * D2), *t1 = dalloc(D * D), *t2 = dalloc(D * D);
    double *X11 = dalloc(D * D), *X21 = dalloc(D * D), *X22 = dalloc(D * D), *G = dalloc(D * D);
    double *F = dalloc(D * D), *W = dalloc((long)D * D2), *v1 = dalloc(D), *v2 = dalloc(D), *v3 = dalloc(D);
    /* M = [[sCi^T sJj, I], [sJj, 0]] */
    mm(D, D, D, sCi, 1, sJj, 0, t1);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            M[r * D2 + c] = t1[r * D + c];
            M[r * D2 + D + c] = r == c ? 1.0 : 0.0;
            M[(D + r) * D2 + c] = sJj[r * D + c];
            M[(D + r) * D2 + D + c] = 0.0;
        }
    orc_tria(D2, D2, M, Xi);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            X11[r * D + c] = Xi[r * D2 + c];
            X21[r * D + c] = Xi[(D + r) * D2 + c];
            X22[r * D + c] = Xi[(D + r) * D2 + D + c];
        }
    /* G = sCi Xi11^{-T} (D x D);  F = I - G Xi21^T */
    right_solve_lower_t(D, D, X11, sCi, G);
    mm(D, D, D, G, 0, X21, 1, t1);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) F[r * D + c] = (r == c ? 1.0 : 0.0) - t1[r * D + c];
    /* A_ij = A_j F A_i */
    mm(D, D, D, F, 0, Ai, 0, t1);
    mm(D, D, D, Aj, 0, t1, 0, A);
    /* b_ij = A_j F (b_i + sCi sCi^T eta_j) + b_j */
    mv(D, D, sCi, 1, etaj, v1);
    mv(D, D, sCi, 0, v1, v2);
    for (int r = 0; r < D; ++r) v2[r] += bi[r];
    mv(D, D, F, 0, v2, v1);
    mv(D, D, Aj, 0, v1, v3);
    for (int r = 0; r < D; ++r) b[r] = v3[r] + bj[r];
    /* sqrtC_ij = tria([A_j G, sCj]) */
    mm(D, D, D, Aj, 0, G, 0, t1);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            W[r * D2 + c] = t1[r * D + c];
            W[r * D2 + D + c] = sCj[r * D + c];
        }
    orc_tria(D, D2, W, sC);
    /* eta_ij = A_i^T (I - Xi21 Xi11^{-1} sCi^T)(eta_j - sJj sJj^T b_i) + eta_i
     * and (I - Xi21 Xi11^{-1} sCi^T) = F^T */
    mv(D, D, sJj, 1, bi, v1);
    mv(D, D, sJj, 0, v1, v2);
    for (int r = 0; r < D; ++r) v2[r] = etaj[r] - v2[r];
    mv(D, D, F, 1, v2, v1);
    mv(D, D, Ai, 1, v1, v3);
    for (int r = 0; r < D; ++r) eta[r] = v3[r] + etai[r];
    /* sqrtJ_ij = tria([A_i^T Xi22, sJi]) */
    mm(D, D, D, Ai, 1, X22, 0, t2);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            W[r * D2 + c] = t2[r * D + c];
            W[r * D2 + D + c] = sJi[r * D + c];
        }
    orc_tria(D, D2, W, sJ);
    free(M); free(Xi); free(t1); free(t2); free(X11); free(X21); free(X22); free(G); free(F); free(W);
    free(v1); free(v2); free(v3);
}

/* Square-root smoothing element (eq. sqrt-smoothing-elements); for the last
 * step ("last") the element is p(Y_N | Z_{1:N}) itself: E = 0, g = m^f_N,
 * sqrtL = sqrtP^f_N. */
void orc_smoother_element(int D, const double *Phi, const double *sqrtQ, const double *mf, const double *sPf,
                          int last, double *E, double *g, double *sL)
{
    if (last) {
        memset(E, 0, sizeof(double) * D * D);
        memcpy(g, mf, sizeof(double) * D);
        memcpy(sL, sPf, sizeof(double) * D * D);
        return;
    }
    int D2 = 2 * D;
    double *M = dalloc((long)D2 * D2), *Pi = dalloc((long)D2 * D2), *t = dalloc(D * D), *P11 = dalloc(D * D);
    double *P21 = dalloc(D * D), *v = dalloc(D), *v2 = dalloc(D);
    mm(D, D, D, Phi, 0, sPf, 0, t);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            M[r * D2 + c] = t[r * D + c];
            M[r * D2 + D + c] = sqrtQ[r * D + c];
            M[(D + r) * D2 + c] = sPf[r * D + c];
        }
    orc_tria(D2, D2, M, Pi);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            P11[r * D + c] = Pi[r * D2 + c];
            P21[r * D + c] = Pi[(D + r) * D2 + c];
            sL[r * D + c] = Pi[(D + r) * D2 + D + c];
        }
    right_solve_lower(D, D, P11, P21, E);
    mv(D, D, Phi, 0, mf, v);
    mv(D, D, E, 0, v, v2);
    for (int r = 0; r < D; ++r) g[r] = mf[r] - v2[r];
    free(M); free(Pi); free(t); free(P11); free(P21); free(v); free(v2);
}

/* Smoothing operator b_ij = b_i (x)_s b_j (eq. sqrt-associative-smoothing) */
void orc_smoother_combine(int D, const double *Ei, const double *gi, const double *sLi, const double *Ej,
                          const double *gj, const double *sLj, double *E, double *g, double *sL)
{
    double *t = dalloc(D * D), *W = dalloc(2L * D * D);
    mm(D, D, D, Ei, 0, Ej, 0, E);
    mv(D, D, Ei, 0, gj, g);
    for (int r = 0; r < D; ++r) g[r] += gi[r];
    mm(D, D, D, Ei, 0, sLj, 0, t);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            W[r * 2 * D + c] = t[r * D + c];
            W[r * 2 * D + D + c] = sLi[r * D + c];
        }
    orc_tria(D, 2 * D, W, sL);
    free(t);
    free(W);
}

int orc_ieks_lm(int field, const double *params, int nparams, int d_req, const double *y0, double t0, double t1,
                int q, long N, int max_iter, double tol, int fixed_iters, const double *init_traj,
                double lm_sigma, double *mean_out, double *sqrtcov_out, double *delta_hist, int *iters_out)
{
    return orc_ieks_prior(field, params, nparams, d_req, y0, t0, t1, q, N, max_iter, tol, fixed_iters, init_traj,
                          lm_sigma, 0, 0.0, mean_out, sqrtcov_out, delta_hist, iters_out);
}

int orc_ieks(int field, const double *params, int nparams, int d_req, const double *y0, double t0, double t1,
             int q, long N, int max_iter, double tol, int fixed_iters, const double *init_traj,
             double *mean_out, double *sqrtcov_out, double *delta_hist, int *iters_out)
{
    return orc_ieks_lm(field, params, nparams, d_req, y0, t0, t1, q, N, max_iter, tol, fixed_iters, init_traj, 0.0,
                       mean_out, sqrtcov_out, delta_hist, iters_out);
}

/* ------------------------------------------------------------------------ */
/* starting trajectory from a coarse grid (remark "Other choices for the     */
/* initial state trajectory", Sec. 3.2.2)                                    */
/* ------------------------------------------------------------------------ */

/* The coarse grid: s = ceil(N / M_target) fine steps per coarse step and
 * M = ceil(N / s) coarse steps of length H = s h from t0 (the last coarse
 * node may lie past t1; the vector fields are autonomous). */
void orc_coarse_grid(long N, long M_target, long *s_out, long *M_out)
{
    if (M_target < 1) M_target = 1;
    long s = (N + M_target - 1) / M_target;
    if (s < 1) s = 1;
    *s_out = s;
    *M_out = (N + s - 1) / s;
}

/* Mean of the IWP(q) prior at t_k + tau conditioned on its full states x_k at
 * t_k and x_k1 at t_k + H (one ODE component, q+1 derivatives), i.e. the
 * Gaussian bridge
 *   x(tau) = Phi(tau) x_k + Q(tau) Phi(H - tau)^T Q(H)^{-1} (x_k1 - Phi(H) x_k),
 * the conditional mean of the first of the two jointly Gaussian transitions
 * given their sum (Sec. 2.1 transition densities). */
void orc_iwp_bridge(int q, double H, double tau, const double *xk, const double *xk1, double *out)
{
    int S = q + 1;
    double *Pt = dalloc(S * S), *Qt = dalloc(S * S), *Pr = dalloc(S * S), *Qr = dalloc(S * S);
    double *PH = dalloc(S * S), *QH = dalloc(S * S), *L = dalloc(S * S), *v = dalloc(S), *w = dalloc(S);
    double *z = dalloc(S), *u = dalloc(S);
    orc_iwp(q, tau, Pt, Qt);
    orc_iwp(q, H - tau, Pr, Qr);
    orc_iwp(q, H, PH, QH);
    /* v = x_k1 - Phi(H) x_k ; w = Q(H)^{-1} v by Cholesky */
    mv(S, S, PH, 0, xk, v);
    for (int i = 0; i < S; ++i) v[i] = xk1[i] - v[i];
    orc_chol(S, QH, L);
    lower_solve_vec(S, L, v, z);
    for (int i = S - 1; i >= 0; --i) { /* L^T w = z */
        double t = z[i];
        for (int k = i + 1; k < S; ++k) t -= L[k * S + i] * w[k];
        w[i] = t / L[i * S + i];
    }
    mv(S, S, Pr, 1, w, u);   /* Phi(H - tau)^T w */
    mv(S, S, Qt, 0, u, z);   /* Q(tau) (...) */
    mv(S, S, Pt, 0, xk, out);
    for (int i = 0; i < S; ++i) out[i] += z[i];
    free(Pt); free(Qt); free(Pr); free(Qr); free(PH); free(QH); free(L); free(v); free(w); free(z); free(u);
}

/* Sequential extended Kalman smoother on the coarse grid, then the bridge to
 * the fine grid.  Filter: at each coarse step, predict with the prior
 * (preconditioned coordinates of step H), linearise the ODE at the predicted
 * mean (EK1, Sec. 3.2.1: Hbar = E1 - (T0/T1) F_y E0, innovation
 * (f(y-) - y-')/T1), update in square-root form (Psi = tria([[Hbar sqrtP-],
 * [sqrtP-]])).  Smoother: RTS,
 *   m^s_k = m^f_k + G_k (m^s_{k+1} - Phi m^f_k),  G_k = Pi21 Pi11^{-1},
 *   Pi = tria([[Phi sqrtP^f_k, sqrtQ], [sqrtP^f_k, 0]]).
 * traj_out: [N+1][D] fine-grid trajectory in original coordinates, row 0 =
 * mu0.  Returns 0, -1 (bad arguments) or -4 (non-finite coarse values). */
int orc_coarse_start(int field, const double *params, int nparams, int d_req, const double *y0, double t0,
                     double t1, int q, long N, long M_target, double *traj_out)
{
    int d = orc_field_dim(field, d_req, nparams);
    if (d < 1 || q < 1 || N < 1 || !(t1 > t0)) return -1;
    long s, M;
    orc_coarse_grid(N, M_target, &s, &M);
    int S = q + 1, D = d * S, n2 = d + D;
    double h = (t1 - t0) / (double)N, H = s * h;
    double *PhiB = dalloc(D * D), *sQB = dalloc(D * D), *T = dalloc(D), *mu0 = dalloc(D);
    precond_model(d, q, H, PhiB, sQB, T);
    orc_taylor_mu0(field, params, d, y0, q, mu0);
    double *mf = dalloc((M + 1) * D), *sPf = dalloc((M + 1) * D * D), *ms = dalloc((M + 1) * D);
    double *mp = dalloc(D), *sPp = dalloc(D * D), *tmp = dalloc(D * D), *W = dalloc(4L * D * D);
    double *Mx = dalloc((long)n2 * n2), *Psi = dalloc((long)n2 * n2), *Hn = dalloc(d * D), *res = dalloc(d);
    double *Ps11 = dalloc(d * d), *Ps21 = dalloc(D * d), *K = dalloc(D * d), *v = dalloc(D), *v2 = dalloc(D);
    double *y = dalloc(d), *fy = dalloc(d), *Jy = dalloc(d * d), *Pi = dalloc(4L * D * D);
    double *P11 = dalloc(D * D), *P21 = dalloc(D * D), *G = dalloc(D * D);
    double T0 = T[0], T1 = T[1];
    int bad = 0;
    for (int k = 0; k < D; ++k) mf[k] = mu0[k] / T[k];
    for (long n = 1; n <= M; ++n) {
        const double *m = mf + (n - 1) * D, *sP = sPf + (n - 1) * D * D;
        mv(D, D, PhiB, 0, m, mp);
        mm(D, D, D, PhiB, 0, sP, 0, tmp);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                W[r * 2 * D + c] = tmp[r * D + c];
                W[r * 2 * D + D + c] = sQB[r * D + c];
            }
        orc_tria(D, 2 * D, W, sPp);
        for (int i = 0; i < d; ++i) y[i] = T0 * mp[i * S];
        orc_field_f(field, params, d, y, fy);
        orc_field_jac(field, params, d, y, Jy);
        memset(Hn, 0, sizeof(double) * d * D);
        for (int i = 0; i < d; ++i) {
            Hn[i * D + i * S + 1] = 1.0;
            for (int j = 0; j < d; ++j) Hn[i * D + j * S] -= Jy[i * d + j] * T0 / T1;
            res[i] = (fy[i] - T1 * mp[i * S + 1]) / T1;
        }
        memset(Mx, 0, sizeof(double) * n2 * n2);
        mm(d, D, D, Hn, 0, sPp, 0, tmp);
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < D; ++c) Mx[r * n2 + c] = tmp[r * D + c];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) Mx[(d + r) * n2 + c] = sPp[r * D + c];
        orc_tria(n2, n2, Mx, Psi);
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) Ps11[r * d + c] = Psi[r * n2 + c];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < d; ++c) Ps21[r * d + c] = Psi[(d + r) * n2 + c];
        right_solve_lower(D, d, Ps11, Ps21, K);
        mv(D, d, K, 0, res, v);
        double *mo = mf + n * D, *so = sPf + n * D * D;
        for (int r = 0; r < D; ++r) {
            mo[r] = mp[r] + v[r];
            if (!isfinite(mo[r])) bad = 1;
            for (int c = 0; c < D; ++c) so[r * D + c] = Psi[(d + r) * n2 + d + c];
        }
        if (bad) break;
    }
    if (!bad) {
        memcpy(ms + M * D, mf + M * D, sizeof(double) * D);
        for (long n = M - 1; n >= 0; --n) {
            const double *m = mf + n * D, *sP = sPf + n * D * D;
            memset(W, 0, sizeof(double) * 4 * D * D);
            mm(D, D, D, PhiB, 0, sP, 0, tmp);
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    W[r * 2 * D + c] = tmp[r * D + c];
                    W[r * 2 * D + D + c] = sQB[r * D + c];
                    W[(D + r) * 2 * D + c] = sP[r * D + c];
                }
            orc_tria(2 * D, 2 * D, W, Pi);
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    P11[r * D + c] = Pi[r * 2 * D + c];
                    P21[r * D + c] = Pi[(D + r) * 2 * D + c];
                }
            right_solve_lower(D, D, P11, P21, G);
            mv(D, D, PhiB, 0, m, v);
            for (int r = 0; r < D; ++r) v[r] = ms[(n + 1) * D + r] - v[r];
            mv(D, D, G, 0, v, v2);
            for (int r = 0; r < D; ++r) {
                ms[n * D + r] = m[r] + v2[r];
                if (!isfinite(ms[n * D + r])) bad = 1;
            }
        }
    }
    if (!bad) {
        /* bridge every fine point between its two coarse nodes, original coordinates */
        double *xa = dalloc(S), *xb = dalloc(S), *xo = dalloc(S);
        for (long j = 0; j <= N; ++j) {
            long k = j / s, o = j % s;
            for (int i = 0; i < d; ++i) {
                for (int c = 0; c < S; ++c) {
                    xa[c] = T[i * S + c] * ms[k * D + i * S + c];
                    xb[c] = o ? T[i * S + c] * ms[(k + 1) * D + i * S + c] : 0.0;
                }
                if (o == 0)
                    memcpy(xo, xa, sizeof(double) * S);
                else
                    orc_iwp_bridge(q, H, o * h, xa, xb, xo);
                for (int c = 0; c < S; ++c) traj_out[j * D + i * S + c] = xo[c];
            }
        }
        for (int k = 0; k < D; ++k) traj_out[k] = mu0[k];
        free(xa); free(xb); free(xo);
    }
    free(PhiB); free(sQB); free(T); free(mu0); free(mf); free(sPf); free(ms); free(mp); free(sPp); free(tmp);
    free(W); free(Mx); free(Psi); free(Hn); free(res); free(Ps11); free(Ps21); free(K); free(v); free(v2);
    free(y); free(fy); free(Jy); free(Pi); free(P11); free(P21); free(G);
    return bad ? -4 : 0;
}
