"""CostEvaluation (Alg. 2) and DisparityRefinement (Alg. 3). Test infrastructure only.

Alg. 2: every pixel of Omega_I gets one census matching cost between the left
pixel and the right pixel displaced by its interpolated disparity. Readings: the
real disparity is rounded to a column as floor(float32(D + 0.5)); the pixel is
evaluated only when D is defined (inside the mesh), the rounded disparity lies in
[d_min, d_max] and the right window fits (u - d >= rx). The cost is the raw Hamming
distance (the paper's "normalised" cost, kept in Hamming units so thresholds are
integers); 0xFF marks a pixel that was not evaluated.

Alg. 3: with an occupancy grid of sz_occ x sz_occ cells, the pixels are visited in
raster order and
  * if C_it < C_f, the final disparity/cost take the interpolated ones;
  * if C_it < t_lo and C_it < the cell's stored confident cost, the cell C_g records
    (u, v, D_it, C_it);
  * if C_it > t_hi and C_it > the cell's stored invalid cost, the cell C_b records
    (u, v, C_it).
C_g starts at cost t_lo and C_b at cost t_hi, so only strictly better/worse pixels
are recorded, and the first pixel in raster order wins ties. Cells cover the image
edge: H' = ceil(H / sz_occ), W' = ceil(W / sz_occ), u' = floor(u / sz_occ). A cell
is "set" when some pixel was recorded (the paper's "!= 0" test would miss pixel
(0, 0) and cost 0).
"""
from dataclasses import dataclass

import numpy as np

NOT_EVALUATED = 0xFF


@dataclass
class Cell:
    set: bool = False
    u: int = 0
    v: int = 0
    d: float = 0.0
    cost: int = 0


def cost_evaluation(cL, cR, omega, D_it, p) -> np.ndarray:
    """Alg. 2: C_it uint8 [H, W], 0xFF where not evaluated.

    With ``p.levels`` = L > 1 (the "3-5 disparity levels" of Sec. III-B), the cost of an
    evaluated pixel is the smallest Hamming distance over the L integer disparities
    d - k .. d + k (k = (L - 1) / 2) around the rounded d that are themselves admissible
    (in [d_min, d_max], u - d' >= rx); which pixels are evaluated, and D_it itself, do not
    change."""
    H, W = cL.shape
    C = np.full((H, W), NOT_EVALUATED, dtype=np.uint8)
    vs, us = np.nonzero(omega & np.isfinite(D_it))
    if vs.size == 0:
        return C
    D = D_it[vs, us].astype(np.float32)
    dint = np.floor(D + np.float32(0.5)).astype(np.int64)
    ok = (dint >= p.d_min) & (dint <= p.d_max) & (us - dint >= p.rx)
    vs, us, dint = vs[ok], us[ok], dint[ok]
    x = np.bitwise_xor(cL[vs, us], cR[vs, us - dint])
    cost = np.bitwise_count(x).astype(np.int64)
    k = (getattr(p, "levels", 1) - 1) // 2
    for delta in range(-k, k + 1):
        if delta == 0:
            continue
        d2 = dint + delta
        ok2 = (d2 >= p.d_min) & (d2 <= p.d_max) & (us - d2 >= p.rx)
        c2 = np.full(cost.shape, 255, dtype=np.int64)
        c2[ok2] = np.bitwise_count(np.bitwise_xor(cL[vs[ok2], us[ok2]], cR[vs[ok2], us[ok2] - d2[ok2]]))
        cost = np.minimum(cost, c2)
    C[vs, us] = cost.astype(np.uint8)
    return C


def disparity_refinement(D_it, C_it, D_f, C_f, p, sz_occ):
    """Alg. 3. Updates D_f, C_f in place; returns the cell grids (C_g, C_b) as lists of
    rows of ``Cell``."""
    H, W = C_it.shape
    Hc = -(-H // sz_occ)
    Wc = -(-W // sz_occ)
    Cg = [[Cell(cost=p.t_lo) for _ in range(Wc)] for _ in range(Hc)]
    Cb = [[Cell(cost=p.t_hi) for _ in range(Wc)] for _ in range(Hc)]
    evaluated = C_it != NOT_EVALUATED
    # per-pixel final update (independent per pixel)
    better = evaluated & (C_it < C_f)
    D_f[better] = D_it[better]
    C_f[better] = C_it[better]
    # cell records: the sequential raster-order loop over the pixels that can touch a cell
    cand = evaluated & ((C_it < p.t_lo) | (C_it > p.t_hi))
    for v, u in zip(*np.nonzero(cand)):          # np.nonzero walks in raster order
        c = int(C_it[v, u])
        cell_g = Cg[v // sz_occ][u // sz_occ]
        cell_b = Cb[v // sz_occ][u // sz_occ]
        if c < p.t_lo and c < cell_g.cost:
            cell_g.set, cell_g.u, cell_g.v, cell_g.d, cell_g.cost = True, int(u), int(v), float(D_it[v, u]), c
        if c > p.t_hi and c > cell_b.cost:
            cell_b.set, cell_b.u, cell_b.v, cell_b.cost = True, int(u), int(v), c
    return Cg, Cb
