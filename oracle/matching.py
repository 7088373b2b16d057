"""Support candidates and sparse epipolar matching. Test infrastructure only.

Sec. III-A: support points s = (u, v, d) are found by matching keypoints along
their epipolar lines (rows of a rectified pair); Alg. 4 re-uses the same epipolar
search ("SparseEpipolarStereo") for resampled pixels. The paper delegates the
matcher's details to prior work, so the following readings are used:

* candidates: nodes ``(g//2 + i*g, g//2 + j*g)`` of a regular grid of pitch
  ``g = support_step``, in raster order, kept when they lie in Omega_I (this grid
  stands in for the paper's FAST keypoints sampled from spatial bins);
* cost: Hamming distance between census words;
* d* = argmin over d in [d_min, d_max] with u - d >= rx (the right window fits),
  ties to the smallest d;
* rejected when no disparity is admissible, when cost(d*) >= t_hi, or, with
  ``uniqueness = m > 0``, when some admissible d with |d - d*| >= 2 has
  cost(d) < cost(d*) + m;
* left-right check: from u_r = u - d*, the right-to-left argmin d' over
  d in [d_min, d_max] with u_r + d <= W - 1 - rx (ties to the smallest d) must
  satisfy |d' - d*| <= lr_tol;
* accepted matches are returned as (u, v, float(d*)) in candidate order.
"""
from typing import List, Optional, Tuple

import numpy as np


def hamming(a, b) -> int:
    """Hamming distance of two census words (popcount of their XOR)."""
    return bin(int(a) ^ int(b)).count("1")


def _hamming_vec(word, words: np.ndarray) -> np.ndarray:
    x = np.bitwise_xor(np.uint64(word), words.astype(np.uint64))
    return np.bitwise_count(x).astype(np.int64)


def grid_candidates(W: int, H: int, step: int, omega: np.ndarray) -> List[Tuple[int, int]]:
    """Grid nodes (step//2 + i*step, step//2 + j*step) in raster order, kept iff in Omega_I."""
    out = []
    for v in range(step // 2, H, step):
        for u in range(step // 2, W, step):
            if omega[v, u]:
                out.append((u, v))
    return out


def _argmin_smallest(ds: np.ndarray, costs: np.ndarray) -> int:
    best = costs.min()
    return int(ds[costs == best].min())


def match_point(cL: np.ndarray, cR: np.ndarray, u: int, v: int, p) -> Optional[int]:
    """Integer disparity of left pixel (u, v) or None when the match is rejected."""
    H, W = cL.shape
    rx = p.rx
    ds = np.arange(p.d_min, p.d_max + 1)
    ds = ds[u - ds >= rx]
    if ds.size == 0:
        return None
    costs = _hamming_vec(cL[v, u], cR[v, u - ds])
    d_star = _argmin_smallest(ds, costs)
    c_star = int(costs[ds == d_star][0])
    if c_star >= p.t_hi:
        return None
    if p.uniqueness > 0:
        far = np.abs(ds - d_star) >= 2
        if np.any(costs[far] < c_star + p.uniqueness):
            return None
    ur = u - d_star
    ds2 = np.arange(p.d_min, p.d_max + 1)
    ds2 = ds2[ur + ds2 <= W - 1 - rx]
    costs2 = _hamming_vec(cR[v, ur], cL[v, ur + ds2])
    d_lr = _argmin_smallest(ds2, costs2)
    if abs(d_lr - d_star) > p.lr_tol:
        return None
    return d_star


def sparse_stereo(cL: np.ndarray, cR: np.ndarray, cands, p) -> List[Tuple[int, int, float]]:
    """Match every candidate; accepted ones as (u, v, float(d)) in candidate order."""
    out = []
    for (u, v) in cands:
        d = match_point(cL, cR, u, v, p)
        if d is not None:
            out.append((int(u), int(v), float(d)))
    return out
