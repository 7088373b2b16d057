"""Iterative Stereo Reconstruction (Alg. 1). Test infrastructure only.

D_f <- 0, C_f <- t_hi, sz_occ <- sz_occ0; S_1 <- SparseStereo(I_l, I_r);
G(S_1) <- Delaunay; for it = 1..n_iters: D_it <- interpolation over G(S_it),
C_it <- CostEvaluation, (C_g, C_b) <- DisparityRefinement, and unless it is the
last iteration: S_it+1 <- SupportResampling, G(S_it+1) <- Delaunay,
sz_occ <- max(1, sz_occ / 2).

The output is the semi-dense D_f on Omega_I; ``mask`` = Omega_I and C_f < t_hi,
which (C_f starting at t_hi) is exactly the set of pixels that passed validation.
"""
import time

import numpy as np

from .census import census, high_gradient
from .fast import fast_candidates
from .delaunay import triangulate
from .interp import interpolate
from .matching import grid_candidates, sparse_stereo
from .params import Params
from .refine import cost_evaluation, disparity_refinement
from .resample import support_resampling


def occupancy_size(p: Params, it: int) -> int:
    """sz_occ used by refinement at iteration ``it`` (1-based): halved after each
    resampling, never below 1."""
    sz = p.sz_occ0
    for _ in range(it - 1):
        sz = max(1, sz // 2)
    return sz


class _Clock:
    """Wall time per stage, summed into ``times`` (a dict) when one is given; timing only."""

    def __init__(self, times):
        self.times = times
        self.t = time.perf_counter()

    def lap(self, stage):
        if self.times is not None:
            now = time.perf_counter()
            self.times[stage] = self.times.get(stage, 0.0) + (now - self.t)
            self.t = now


def solve(left: np.ndarray, right: np.ndarray, p: Params, trace: bool = False, times=None):
    """Alg. 1 on a rectified uint8 pair. Returns a dict with D_f, C_f, mask and, with
    ``trace``, every intermediate (supports, triangles, D_it, C_it, cells). With a dict
    ``times``, the wall time of each stage is added to it (seconds)."""
    H, W = left.shape
    clk = _Clock(times)
    cL, valid = census(left, p.census_w, p.census_h)
    cR, _ = census(right, p.census_w, p.census_h)
    omega = high_gradient(left, valid, p.grad_thr)
    D_f = np.zeros((H, W), dtype=np.float32)
    C_f = np.full((H, W), p.t_hi, dtype=np.uint8)
    clk.lap("census")
    if getattr(p, "support_mode", 0) == 1:
        cands = fast_candidates(left, p.fast_threshold, p.fast_bins_x, p.fast_bins_y, p.fast_per_bin)
    else:
        cands = grid_candidates(W, H, p.support_step, omega)
    S = sparse_stereo(cL, cR, cands, p)
    clk.lap("match")
    tris = triangulate(S, W)
    clk.lap("triangulate")
    out = {"cL": cL, "cR": cR, "omega": omega, "iters": []}
    for it in range(1, p.n_iters + 1):
        sz = occupancy_size(p, it)
        D_it = interpolate(S, tris, W, H)
        clk.lap("interpolate")
        C_it = cost_evaluation(cL, cR, omega, D_it, p)
        Cg, Cb = disparity_refinement(D_it, C_it, D_f, C_f, p, sz)
        clk.lap("validate")
        rec = {"S": list(S), "tris": tris, "sz_occ": sz}
        if trace:
            rec.update(D_it=D_it, C_it=C_it, Cg=Cg, Cb=Cb, D_f=D_f.copy(), C_f=C_f.copy())
        if it != p.n_iters:
            S, X, conf, matched = support_resampling(Cg, Cb, S, cL, cR, p)
            clk.lap("resample")
            tris = triangulate(S, W)
            clk.lap("triangulate")
            if trace:
                rec.update(X=X, confident=conf, matched=matched)
        out["iters"].append(rec)
    out["D_f"] = D_f
    out["C_f"] = C_f
    out["mask"] = omega & (C_f < p.t_hi)
    out["S_final"] = S
    return out
