"""Algorithmic work per step for each kernel of one ParaIEKS iteration.

Flops count a multiply-add as 2.  The counts follow the formulas each kernel
evaluates (Householder tria of an nr x nc stack, dense products, triangular
solves), not the instructions the lanes issue: work a kernel repeats for
SIMD uniformity (e.g. updating already-finished rows in tria) is excluded.
Bytes are the compulsory HBM traffic of the kernel's inputs and outputs (the
trajectory is FP64: the forward step kernels read rows n-1 and n).
"""
from __future__ import annotations


def tria(nr, nc):
    """Householder LQ of an nr x nc matrix: reflection k forms its vector
    from row k (2(nc-k)) and updates the rows below it (4(nc-k) each)."""
    f = 0
    for k in range(min(nr, nc)):
        f += 2 * (nc - k) + 4 * (nc - k) * (nr - k - 1)
    return f


def mm(n, k, m):
    return 2 * n * k * m


def trsolve(rows, n):
    return rows * n * n


def obs_setup(D, d):
    return mm(d, D, D) + 4 * d * d  # H Phi and the linearised data


def filter_element(D, d):
    return (mm(d, D, D) + tria(d + D, D) + trsolve(D, d) + mm(D, d, D) + 2 * D * d + trsolve(D, d) + d * d
            + 2 * D * d)


def filter_combine(D, nj=None, ncj=None):
    """Filtering operator with nj (ncj) leading columns of sqrtJ_j (sqrtC_j)
    that can be nonzero: D, D for aggregates; d, D - d for one step's element."""
    nj = D if nj is None else nj
    ncj = D if ncj is None else ncj
    return (mm(D, D, nj) + tria(2 * D, D + nj) + trsolve(D, D) + mm(D, D, D) + 2 * D * D + 2 * D * nj
            + 2 * mm(D, D, D) + 6 * D * D + 2 * D * nj + mm(D, D, D) + tria(D, D + ncj) + 2 * D * D
            + mm(D, D, nj) + tria(D, D + nj))


def state_apply(D):
    return (mm(D, D, D) + tria(2 * D, 2 * D) + trsolve(D, D) + mm(D, D, D) + 2 * D * D + mm(D, D, D)
            + 4 * D * D + mm(D, D, D) + tria(D, 2 * D))


def kf_step_with_smoothing_element(D, d):
    """Kalman step whose prediction is the leading block of the 2D x 2D
    smoothing-element tria, plus E, g of the previous step."""
    return (mm(D, D, D) + 2 * D * D + tria(2 * D, 2 * D) + trsolve(D, D) + 2 * D * D + mm(d, D, D)
            + tria(d + D, D) + 2 * d * D + trsolve(D, d) + 2 * D * d)


def smoother_combine(D, with_cov=False):
    return mm(D, D, D) + 2 * D * D + ((mm(D, D, D) + tria(D, 2 * D)) if with_cov else 0)


def smoother_apply(D, with_cov=False):
    return 2 * D * D + ((mm(D, D, D) + tria(D, 2 * D)) if with_cov else 0)


def forward_chunk(N):
    """Forward chunk length the library picks for a request of N steps (the
    same rule as the host code: double from 4 while N / (2 b1) >= 8192, at
    most 32)."""
    b1 = 4
    while b1 < 32 and N // (2 * b1) >= 8192:
        b1 *= 2
    return b1


def per_step(d, q, esize, b1=32, bs1=8):
    """{kernel: (flops per step, bytes per step)} for a means-only iteration,
    with forward chunks of b1 steps and reverse chunks of bs1 steps.  The tree
    kernels are charged per step as their per-aggregate work / b1.  Bytes
    count each FP64 trajectory row once per kernel (steps n-1 and n share
    rows) and the stored records with their flag word."""
    D = d * (q + 1)
    DP = D * (D + 1) // 2
    FEF, FS, SAF = 3 * D * D + 2 * D + 1, D + D * D, 2 * D * D + D + 1
    # smoothing record: E, offset, filtering mean, flag (the reverse reduce
    # reads all but the mean)
    SEF, SEF_R = D * D + 2 * D + 1, D * D + D + 1
    s = esize
    return {
        "fwd_reduce1": (obs_setup(D, d) + filter_element(D, d) + filter_combine(D, d, D - d) * (b1 - 1) / b1,
                        8 * D + s * FEF / b1),
        "fwd_tree_up": (filter_combine(D) / b1, s * 2 * FEF / b1),
        "fwd_tree_down": (state_apply(D) / b1, s * (FEF + 2 * FS) / b1),
        "fwd_down1": (obs_setup(D, d) + kf_step_with_smoothing_element(D, d),
                      8 * D + s * (FS / b1 + SEF + DP)),
        "bwd_reduce1": (smoother_combine(D) * (bs1 - 1) / bs1, s * (SEF_R + SAF / bs1)),
        "bwd_down1": (smoother_apply(D), s * (SEF + FS / bs1) + 16 * D),
    }


def coarse_points(N):
    """Coarse grid of the library's default start: target max(1024,
    64 ceil(log2 N)) capped at N, s = ceil(N / target) fine steps per coarse
    step, M = ceil(N / s) coarse steps."""
    import math

    target = min(N, max(1024, 64 * max(1, math.ceil(math.log2(max(N, 2))))))
    s = -(-N // target)
    return -(-N // s)


def coarse_step_flops(d, q):
    """FP64 flops of one step of the coarse extended Kalman filter and its RTS
    means (block-structured prior products, column-sparse Joseph update)."""
    S = q + 1
    D = d * S
    DD = D * D
    fwd = (2 * DD * S * 2 + DD            # Phi P, (Phi P) Phi^T + Q
           + 2 * D * S                    # m- = Phi m
           + 2 * D * d * (1 + d)          # U = P- Hbar^T
           + 2 * d * d * (1 + d) + d ** 3  # S and its factor
           + 2 * D * d * d + 2 * D * d    # gain rows, mean update
           + 2 * DD * (2 * d + d * d) * 2)  # B = A P-, P = B A^T
    bwd = 2 * D * S + 2 * D * D + 2 * d * D + 2 * D * d
    return fwd + bwd


def iteration_flops(d, q, b1=32):
    return sum(v[0] for v in per_step(d, q, 4, b1).values())


# ---------------------------------------------------------------------------
# dense engine (one workgroup per element operation, Blelloch sweeps)
# ---------------------------------------------------------------------------
def dense_element(D, d):
    """linearised filtering element of one step (step 1 stops after b, sqrtC)"""
    return tria(d + D, D) + trsolve(D, d) + mm(D, d, D) + trsolve(D, d) + 2 * D * d + d * d + 2 * D * d


def dense_fcombine(D, state):
    """filtering operator on dense D x D operands; state: the left operand is
    a prefix state (only b and sqrtC are formed)"""
    f = (mm(D, D, D) + tria(2 * D, 2 * D) + trsolve(D, D) + mm(D, D, D) + mm(D, D, D) + 6 * D * D
         + mm(D, D, D) + tria(D, 2 * D))
    if not state:
        f += mm(D, D, D) + 8 * D * D + mm(D, D, D) + tria(D, 2 * D)
    return f


def dense_selement(D, q):
    return 2 * D * D * (q + 1) + tria(2 * D, 2 * D) + trsolve(D, D) + 2 * D * D + 2 * D * (q + 1)


def dense_bcombine(D, state, with_L=False):
    f = 2 * D * D + (0 if state else mm(D, D, D))
    if with_L:
        f += mm(D, D, D) + tria(D, 2 * D)
    return f


def dense_sweep_pairs(N):
    """(general, state) pair counts of the up-sweep and the state pairs of the
    down-sweep, as the level launches enumerate them"""
    up_g = up_s = down = 0
    s = 1
    smax = 0
    while 2 * s <= N:
        np_ = N // (2 * s)
        up_s += 1
        up_g += np_ - 1
        smax = s
        s *= 2
    s = smax
    while s >= 1:
        if N >= 3 * s:
            down += (N - 3 * s) // (2 * s) + 1
        s //= 2
    return up_g, up_s, down


def dense_iteration_flops(D, d, q, N, B=1):
    """Algorithmic flops of one dense iteration per kernel name (whole batch)."""
    up_g, up_s, down = dense_sweep_pairs(N)
    fc = dense_fcombine(D, False)
    fs = dense_fcombine(D, True)
    out = {
        "dense_elements": B * (N * dense_element(D, d)),
        "dense_fcombine_up": B * (up_g * fc + up_s * fs),
        "dense_fcombine_down": B * down * fs,
        "dense_selements": B * max(N - 1, 0) * dense_selement(D, q),
        "dense_bcombine_up": B * (up_g * dense_bcombine(D, False) + up_s * dense_bcombine(D, True)),
        "dense_bcombine_down": B * down * dense_bcombine(D, True),
        "dense_update": B * N * D,
    }
    return out
