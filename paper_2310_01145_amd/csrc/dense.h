// Dense engine: ParaIEKS (Alg. 2) for state dimensions too large for the
// row-per-lane kernels (the method-of-lines field, D = d(q+1) up to 256).
// Internal interface between the C-ABI layer and dense_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "parapn_internal.h"

namespace parapn {

constexpr int kDenseMaxD = 256;

// One batch of B instances of the same problem (field, parameters, d, q, N,
// step); instances differ in their initial values only.
struct DenseModel {
    int field, d, q, D, B, pad_;
    int64_t N;
    double hq;            // h / q
    double T0, T1;        // preconditioner entries of derivatives 0 and 1
    double p[kMaxParams];
    double phib[25];      // (q+1) x (q+1) block of the preconditioned transition
    double sqb[25];       // (q+1) x (q+1) lower factor of the preconditioned process noise
};

// Device buffers, element type of the precision (float or double) unless
// stated.  Per instance b and step index k = 0..N-1 (step n = k + 1):
// filtering elements A, C, J (D x D row-major), b, e (D); smoothing elements
// E, L (D x D), g (D).  Both scans run in place on them.
struct DenseWork {
    void *A, *b, *C, *e, *J;
    void *E, *g, *L;              // L: only for the covariance pass (may be null otherwise)
    void *scratch;                // nwg slots of dense_scratch_elems(D) elements
    double *traj;                 // instance b at traj + b * traj_stride: [N+1][D], then T (D), mu0/T (D)
    int64_t traj_stride;
    unsigned long long *dbits;    // [2B]: bit patterns of delta and max |E0 mu| per instance
    const int *active;            // [B] device flags: 0 = instance frozen (skipped); null = all active
    int nwg;                      // workgroups per launch (scratch slots)
};

size_t dense_scratch_elems(int D);
// workgroups per launch (and scratch slots) of the precision's kernels
int dense_workgroups(int fp64);
// one Gauss-Newton iteration: linearise, both scans, trajectory update, delta
hipError_t dense_iteration(int fp64, const DenseModel &m, const DenseWork &w, hipStream_t s);
// smoothed factors at the last linearisation (filtering marginals still in
// w.b / w.C): rebuilds the smoothing elements with their factors, runs the
// reverse scan with factors and writes cov_out [B][N+1][D][D] (original
// coordinates, row 0 zero)
hipError_t dense_covariance(int fp64, const DenseModel &m, const DenseWork &w, void *cov_out, hipStream_t s);
// objective value V (eq. objective-value, FP64) of each active instance's
// trajectory, added to obj[2b + slot] (slot 0 or 1; the caller zeroes obj)
hipError_t dense_objective(const DenseModel &m, const DenseWork &w, double *obj, int slot, hipStream_t s);

}  // namespace parapn
