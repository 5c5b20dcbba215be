// Internal interface between the C-ABI layer (host code) and the templated
// kernel launchers.  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace parapn {

constexpr int kMaxParams = 16;

// How the observation (H_n, d_n) of step n is obtained.
struct ObsSpec {
    int mode;            // 0: linearise the vector field at the trajectory (IEKS)
                         // 1: read dense H [N][d][D] and d [N][d] from memory
    const void *traj;    // mode 0: preconditioned FP64 trajectory [N+1][D]
    int field;           // mode 0: field id
    double p[kMaxParams];// mode 0: field parameters
    double T0;           // mode 0: scale of the E0 coordinate (y = T0 * E0 traj)
    double T1;           // mode 0: scale of the E1 coordinate (y' = T1 * E1 traj)
    double invT1;        // mode 0: 1 / T1 (row scaling of the observation)
    double hq;           // mode 0: T0 / T1 = h / q
    const void *H;       // mode 1
    const void *dv;      // mode 1
};

// Chunk sizes of the hierarchical scans.
struct ScanPlan {
    int64_t N;     // steps (elements n = 1..N for the filter, 0..N for the smoother)
    int b1;        // steps per group in the forward step-level kernels
    int bs1;       // steps per group in the reverse step-level kernels (8)
    int bu;        // aggregates per group in the upper levels
    int btop;      // largest count handled by the single-group top scan
};

// Device workspace (element type T of the path).
struct Work {
    void *traj;    // [N+1][D]   FP64 trajectory (IEKS), updated in place
    void *mf;      // [N+1][D]   filtered means
    void *sPf;     // [N+1][DP]  filtered factors, packed lower rows
    void *se;      // [N+1][D*D+D] smoothing elements (E, g)
    void *sL;      // [N+1][DP]  smoothing element factors
    void *sPs;     // [N+1][DP]  smoothed factors (covariance pass)
    void *filt_mf; // [N+1][D]   filtered means, or null when not wanted
    void *filt_sPf;// [N+1][DP]  filtered factors, or null when not wanted
    void *fagg;    // filter aggregates, all levels
    void *fpref;   // filter prefix states, all levels
    void *sagg;    // smoother aggregates, all levels
    void *spref;   // smoother suffix states, all levels
    unsigned long long *dbits;  // [2] bit patterns of delta and max|E0 mu| (double)
};

// Constant model data on the device (element type T): Phi, sqrtQ [D][D],
// initial filter state m0 [D], sqrtS0 [D][D].
struct ModelDev {
    const void *Phi;
    const void *sQ;
    const void *m0;
    const void *S0;
    const void *init;  // the initial state as one record: m0 [D] followed by S0 [D][D]
};

struct Dims {
    int d, q, D, DP;
};

// workspace sizes in elements for a plan
size_t work_elems_fagg(int D, const ScanPlan &p);
size_t work_elems_sagg(int D, const ScanPlan &p);
size_t work_records_fpref(const ScanPlan &p);

// Launch sequences.  Each returns hipSuccess or the first launch error.
// T selects the precision (float or double) via `fp64`.
template <typename T>
hipError_t launch_forward_t(int d, int q, const ScanPlan &plan, const ModelDev &m, const ObsSpec &obs, const Work &w,
                            hipStream_t s);
// Reverse scan.  with_cov: also build smoothing factors and write sPs.
// update_traj: write smoothed means into w.traj and accumulate delta (IEKS);
// otherwise write them to mean_out ([N+1][D]).
template <typename T>
hipError_t launch_smoother_t(int d, int q, const ScanPlan &plan, const ModelDev &m, const Work &w, bool with_cov,
                             bool update_traj, void *mean_out, double T0, hipStream_t s);
template <typename T>
hipError_t launch_filter_combine_t(int d, int q, int64_t count, const void *a, const void *c, void *out,
                                   hipStream_t s);
// canonical lower-triangular factor of a D x D square root, D = d(q+1)
template <typename T>
hipError_t launch_tria_square_t(int d, int q, const void *full, void *out, hipStream_t s);

inline hipError_t launch_forward(int fp64, int d, int q, const ScanPlan &plan, const ModelDev &m, const ObsSpec &obs,
                                 const Work &w, hipStream_t s)
{
    return fp64 ? launch_forward_t<double>(d, q, plan, m, obs, w, s) : launch_forward_t<float>(d, q, plan, m, obs, w, s);
}
inline hipError_t launch_smoother(int fp64, int d, int q, const ScanPlan &plan, const ModelDev &m, const Work &w,
                                  bool with_cov, bool update_traj, void *mean_out, double T0, hipStream_t s)
{
    return fp64 ? launch_smoother_t<double>(d, q, plan, m, w, with_cov, update_traj, mean_out, T0, s)
                : launch_smoother_t<float>(d, q, plan, m, w, with_cov, update_traj, mean_out, T0, s);
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
// out mean [N+1][D] = Tdiag * src; out cov [N+1][D][D] = Tdiag * unpack(srcP) (either may be null;
// Tdiag_dev null means 1)
hipError_t launch_unscale(int fp64, int D, int64_t N, const double *Tdiag_dev, const void *src_mean,
                          const void *src_packed, void *mean_out, void *cov_out, hipStream_t s,
                          bool src_fp64 = false);
hipError_t launch_fill_traj(int fp64, int D, int64_t N, const void *row, void *traj, hipStream_t s);
// index of an instantiated (d, q) configuration, or -1
int config_supported(int d, int q);

// Opt-in per-kernel timing: when enabled, launches are bracketed by HIP
// events on their stream and the elapsed times are summed per kernel name.
bool prof_on();
void prof_enable(bool on);
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
