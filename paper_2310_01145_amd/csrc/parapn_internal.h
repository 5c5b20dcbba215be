// Internal interface between the C-ABI layer (host code) and the templated
// kernel launchers.  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace parapn {

constexpr int kMaxParams = 16;
constexpr int kMaxLevels = 24;  // scan levels per request (tree width >= 2, <= 2^24 chunks)
constexpr int kCounters = 5;    // per-request counter words (ReqDev::dbits)

// Doubles per node record of the coarse-grid smoother (k_coarse_eks), with
// D = d (q+1): m^f (D), P (D x D), the 2d columns of A = I - K Hbar that
// differ from I (D each) and c = Hbar^T z (D).
constexpr __host__ __device__ int coarse_record_doubles(int d, int q)
{
    return d * (q + 1) * (2 + d * (q + 1) + 2 * d);
}

// One request of a pack (device-side table, filled by the host).
struct ReqDev {
    int field;
    int lin;                    // Jacobian used by the linearisation: 0 exact (EK1), 1 zero (EK0), 2 its diagonal
                                // (DiagonalEK1)
    double p[kMaxParams];       // field parameters; for F_MOL_COMPONENT: nu d^2, then the element offsets from
                                // this trajectory to its left and right neighbours' trajectories
    double T0, T1, invT1, hq;   // scales of the E0 / E1 coordinates and h/q
    double lm_s;                // damping: std of the E0 pseudo-observations (preconditioned), packs with lm only
    double *traj;               // FP64 preconditioned trajectory [N+1][D]; null for a given linear model
    unsigned long long *dbits;  // kCounters words: delta and max |E0 mu| (bit patterns of doubles, atomic
                                // max), then as doubles the innovations' quadratic-form sum, the objective of
                                // the updated trajectory and the objective of the trajectory before the pass
    int64_t N;                  // steps of this request
    int64_t row;                // packed row of its step 0 in the per-step scratch arrays
    int64_t fchunk;             // index of its first forward step-level chunk
    int64_t schunk;             // index of its first reverse step-level chunk
    int32_t b1;                 // its forward chunk length (a function of N alone)
    int32_t pad2_;
};

// The levels of one request's scan in one direction, laid out exactly as for
// the request alone.  Level 1 holds its step-level chunk aggregates; launch l
// (l = 1 .. L-1) folds level l into level l+1; level L is scanned by one
// group or block per request.  Records of all levels sit in the request's own
// region of the pack array (from base; tree partials of the forward scan from
// pbase).
struct ScanTab {
    int32_t L;
    int32_t pad_;
    int64_t base, pbase;
    int32_t n[kMaxLevels + 1];     // nodes at level l
    int32_t off[kMaxLevels + 1];   // record offset of level l in the request's region
    int32_t poff[kMaxLevels + 1];  // forward: record offset of launch l's tree partials
    int32_t first[kMaxLevels + 1]; // launch l: pack-wide index of the request's first block (forward) or group
                                   // (reverse); for launches it takes no part in, the running count
};

// Starting trajectory of one request from its coarse grid (host-filled).
// The request's field, parameters and resident trajectory come from the
// ReqDev of the same index.
struct CoarseDev {
    int64_t M, s;                // coarse steps; fine steps per coarse step
    double T0, T1, invT1, hq;    // scales of E0 / E1 in the coordinates of the coarse step H, and H/q
    double *node;                // [M+1][D] FP64: filtering means, then (in place) smoothed means
    void *gain;                  // [M+1] FP64 records: m^f_k, P_k (D x D), then for k >= 1 Hbar_k (d x D),
                                 // K_k (D x d) and S_k^-1 r_k (d)
    const double *mu0c;          // [D] mu0 in the coordinates of H
    const double *W;             // [s][q+1][2(q+1)] bridge weights per fine offset o = 0..s-1
    int *status;                 // written by the smoother: 0, or 1 when a coarse value is not finite
    int pad_;
};

// A pack: requests of one (precision, d, q), scanned together.  Every
// request is scanned with its own chunking and its own tree of levels, so its
// arithmetic is that of a solve of it alone; the launches of one level serve
// all requests that have that level.
struct Pack {
    const ReqDev *reqs;  // device tables, nreq entries each, ordered by row
    const ScanTab *ftab, *stab;
    int nreq;
    int64_t rows;        // sum over requests of N_r + 1
    int64_t nf, ns;      // forward / reverse step-level chunks
    int bu, btop;        // reverse upper levels: fold bu per group until <= btop remain
    int Lf, Ls;          // most levels of any request, forward / reverse
    int64_t fblocks[kMaxLevels + 1];  // blocks of forward tree launch l
    int64_t sgroups[kMaxLevels + 1];  // groups of reverse launch l
    int64_t frecs, fprecs, srecs;     // records: forward aggregates (= prefix states), tree partials, reverse
    int mode;            // 0: linearise the vector field at the trajectories; 1: H, d given (one request)
    int lm;              // 1: every request is damped (Levenberg-Marquardt rows, mode 0 only)
    const void *H;       // mode 1: [N][dobs][D]
    const void *dv;      // mode 1: [N][dobs]
    const void *phin;    // mode 1, time-varying model: Phi_n, sqrtQ_n of step n at entry n-1 of [N][D][D+1]
    const void *sqn;     // (rows padded to the LDS constants' stride); null: the constant Phi, sqrtQ
};

// forward chunk length of a request of N steps
int forward_chunk(int64_t N);
// Host: fill chunk indices, rows and b1 of the requests, their scan tables
// and the pack totals (the device pointers of pk are left alone).  Returns 0,
// or -1 if a request needs more than kMaxLevels levels.
int pack_layout(int fp64, int d, int q, ReqDev *reqs, ScanTab *ftab, ScanTab *stab, int nreq, Pack *pk);

// Device workspace of one pack (element type T of the path).
struct Work {
    void *se;      // [rows][D*D+D+1] smoothing elements (E, g, last-flag)
    void *sL;      // [rows][DP]      smoothing element factors
    void *sPs;     // [rows][DP]      smoothed factors (covariance pass), or null
    void *mf;      // [rows][D]       scratch / filtered means
    void *sPf;     // [rows][DP]      filtered factors
    void *filt_mf; // filtered means wanted: = mf, else null
    void *filt_sPf;// filtered factors wanted: = sPf, else null
    void *fagg;    // filter aggregates, all levels [frecs]
    void *fpart;   // filter tree partials [fprecs]
    void *fpref;   // filter prefix states, all levels [frecs]
    void *sagg;    // smoother aggregates, all levels
    void *spref;   // smoother suffix states, all levels
};

// Constant model data on the device (element type T): Phi, sqrtQ [D][D] and
// the initial state record m0 [D] followed by S0 [D][D].
struct ModelDev {
    const void *Phi;
    const void *sQ;
    const void *init;
};


// Launch sequences.  Each returns hipSuccess or the first launch error.
template <typename T>
hipError_t launch_forward_t(int d, int q, const Pack &pk, const ModelDev &m, const Work &w, hipStream_t s);
// Reverse scan.  with_cov: also the smoothed factors (into w.sPs).  update:
// add the smoothed increments to each request's trajectory and accumulate its
// delta; otherwise write the smoothed means to mean_out ([rows][D]).
template <typename T>
hipError_t launch_smoother_t(int d, int q, const Pack &pk, const ModelDev &m, const Work &w, bool with_cov,
                             bool update, void *mean_out, hipStream_t s);
template <typename T>
hipError_t launch_filter_combine_t(int d, int q, int64_t count, const void *a, const void *c, void *out,
                                   hipStream_t s);
// canonical lower-triangular factor of a D x D square root, D = d(q+1)
template <typename T>
hipError_t launch_tria_square_t(int d, int q, const void *full, void *out, hipStream_t s);

inline hipError_t launch_forward(int fp64, int d, int q, const Pack &pk, const ModelDev &m, const Work &w,
                                 hipStream_t s)
{
    return fp64 ? launch_forward_t<double>(d, q, pk, m, w, s) : launch_forward_t<float>(d, q, pk, m, w, s);
}
inline hipError_t launch_smoother(int fp64, int d, int q, const Pack &pk, const ModelDev &m, const Work &w,
                                  bool with_cov, bool update, void *mean_out, hipStream_t s)
{
    return fp64 ? launch_smoother_t<double>(d, q, pk, m, w, with_cov, update, mean_out, s)
                : launch_smoother_t<float>(d, q, pk, m, w, with_cov, update, mean_out, s);
}
inline hipError_t launch_filter_combine(int fp64, int d, int q, int64_t count, const void *a, const void *c,
                                        void *out, hipStream_t s)
{
    return fp64 ? launch_filter_combine_t<double>(d, q, count, a, c, out, s)
                : launch_filter_combine_t<float>(d, q, count, a, c, out, s);
}
inline hipError_t launch_tria_square(int fp64, int d, int q, const void *full, void *out, hipStream_t s)
{
    return fp64 ? launch_tria_square_t<double>(d, q, full, out, s) : launch_tria_square_t<float>(d, q, full, out, s);
}
// mean_out [N+1][D] = Tdiag * src (src FP64 when src_fp64); cov_out [N+1][D][D]
// = cov_scale * Tdiag * unpack(srcP); either output may be null; Tdiag_dev null means 1
hipError_t launch_unscale(int fp64, int D, int64_t N, const double *Tdiag_dev, const void *src_mean,
                          const void *src_packed, void *mean_out, void *cov_out, hipStream_t s,
                          bool src_fp64 = false, double cov_scale = 1.0);
// Coarse-grid start for nreq requests of one (precision, d, q): the
// sequential extended Kalman smoother on each request's coarse grid
// (k_coarse_eks, one wavefront per request, FP64 for either precision),
// then the bridge of the smoothed coarse means to every fine row of the
// request's resident trajectory (k_coarse_bridge).  Phi, Q: the IWP prior's
// preconditioned transition and process-noise covariance, FP64 [D][D].
// reqs and cds are device arrays; maxN is the largest N among the requests.
template <typename T>
hipError_t launch_coarse_t(int d, int q, const ReqDev *reqs, const CoarseDev *cds, int nreq, int64_t maxN,
                           const void *Phi, const void *Q, hipStream_t s);
inline hipError_t launch_coarse(int fp64, int d, int q, const ReqDev *reqs, const CoarseDev *cds, int nreq,
                                int64_t maxN, const void *Phi, const void *Q, hipStream_t s)
{
    return fp64 ? launch_coarse_t<double>(d, q, reqs, cds, nreq, maxN, Phi, Q, s)
                : launch_coarse_t<float>(d, q, reqs, cds, nreq, maxN, Phi, Q, s);
}
// Objective value (eq. objective-value) of every request's resident
// trajectory under the prior (Phi, sQ: the preconditioned transition and the
// process-noise factor, FP64 [D][D]), added to counter word `slot` of each
// request (its dbits, FP64).
hipError_t launch_objective(int d, int q, const Pack &pk, const double *Phi, const double *sQ, int slot, hipStream_t s);
// p[0..n) = 0 by a kernel (graph-capturable, unlike a memset node)
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);
// [N][D][D] -> [N][D][D+1] (the row stride of the kernels' constants), path precision
hipError_t launch_pad_rows(int fp64, int D, int64_t N, const void *src, void *dst, hipStream_t s);
// traj [N+1][D] = preconditioned starting trajectory (k_init_traj)
hipError_t launch_init_traj(int D, int64_t N, const double *init, const double *Td, double *traj, hipStream_t s);

// Decoupled chains (d grid points of state size S = q+1 each, trajectories
// [B][d][N+1][S]): blocks_in writes every instance's preconditioned starting
// trajectories from mu0/T ([B][d S]) and, unless init is null, a starting
// trajectory init [N+1][d S] in original coordinates shared by all instances
// (rows n >= 1; row 0 is mu0).  blocks_out writes instance b's mean
// [N+1][d S] and, when cov_out is set, its block-diagonal square-root factors
// [N+1][d S][d S] in original coordinates (scaled by cov_scale) from the
// packed lower factors of the pack rows row0 + i (N+1) + n.
hipError_t launch_blocks_in(int B, int d, int S, int64_t N, const double *init, const double *Td, const double *mu0b,
                            double *traj, hipStream_t s);
hipError_t launch_blocks_out(int fp64, int d, int S, int64_t N, const double *Td, const double *traj,
                             const void *packed, int64_t row0, void *mean_out, void *cov_out, double cov_scale,
                             hipStream_t s);
// index of an instantiated (d, q) configuration, or -1
int config_supported(int d, int q);

// Opt-in per-kernel timing: when enabled, launches are bracketed by HIP
// events on their stream and the elapsed times are summed per kernel name.
bool prof_on();
void prof_enable(bool on);
// time only launches of this kernel name (null or empty: every kernel)
void prof_only(const char *name);
void prof_begin(const char *name, hipStream_t s, hipEvent_t *start);
void prof_end(const char *name, hipStream_t s, hipEvent_t start);
// resolve pending events; fills up to max entries; returns the number of names
int prof_read(int max, char *names, int name_len, double *total_ms, int64_t *launches);

#define PARAPN_LAUNCH(name, s, ...)                             \
    do {                                                        \
        hipEvent_t ev_start_ = nullptr;                         \
        const bool ev_on_ = ::parapn::prof_on();                \
        if (ev_on_) ::parapn::prof_begin(name, s, &ev_start_);  \
        hipLaunchKernelGGL(__VA_ARGS__);                        \
        if (ev_on_) ::parapn::prof_end(name, s, ev_start_);     \
    } while (0)

}  // namespace parapn
