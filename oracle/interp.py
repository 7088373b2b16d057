"""Disparity planes and piecewise-planar interpolation. Test infrastructure only.

Sec. III-B: every triangle of the Delaunay mesh is a plane in disparity space,
d = pi1' u + pi2' v + pi3' (Eq. 3), whose parameters come from the linear system
through the triangle's three support points and are re-estimated after every
triangulation; a lookup table gives, for every left pixel, its triangle, and the
interpolated disparity D_it is that triangle's plane evaluated at the pixel.

Readings used (the paper fixes neither precision nor edge ownership):

* plane in anchor form around the triangle's first vertex (u0, v0, d0):
  with integer du_k = u_k - u0, dv_k = v_k - v0 (k = 1, 2),
  det = du1*dv2 - du2*dv1 > 0, e_k = d_k - d0, solved in float64 (Cramer's rule):
  a = (e1*dv2 - e2*dv1) / det, b = (du1*e2 - du2*e1) / det, each rounded to float32;
* a pixel (u, v) belongs to the triangle containing the perturbed point
  (u + eps, v + eps^2): for an edge a->b of a counter-clockwise triangle with
  E = orient(a, b, p), the pixel is on the inner side iff E > 0, or E == 0 and
  (a.v > b.v, or a.v == b.v and b.u > a.u). Every pixel whose perturbed point lies
  in the hull has exactly one owner; pixels outside the hull have none (NaN);
* evaluation in float32 with each operation rounded separately:
  D = (d0 + a * float(u - u0)) + b * float(v - v0).
"""
from typing import Sequence

import numpy as np

F32 = np.float32


def plane_of(S: Sequence, t):
    """(a, b, d0, u0, v0) of triangle ``t`` = (i0, i1, i2) over supports ``S``."""
    u0, v0, d0 = int(S[t[0]][0]), int(S[t[0]][1]), F32(S[t[0]][2])
    u1, v1, d1 = int(S[t[1]][0]), int(S[t[1]][1]), F32(S[t[1]][2])
    u2, v2, d2 = int(S[t[2]][0]), int(S[t[2]][1]), F32(S[t[2]][2])
    du1, dv1, du2, dv2 = u1 - u0, v1 - v0, u2 - u0, v2 - v0
    det = du1 * dv2 - du2 * dv1
    assert det > 0, "triangle must be counter-clockwise and non-degenerate"
    e1 = np.float64(d1) - np.float64(d0)
    e2 = np.float64(d2) - np.float64(d0)
    a = (e1 * np.float64(dv2) - e2 * np.float64(dv1)) / np.float64(det)
    b = (np.float64(du1) * e2 - np.float64(du2) * e1) / np.float64(det)
    return F32(a), F32(b), d0, u0, v0


def planes(S, tris):
    return [plane_of(S, t) for t in tris]


def _inside_edge(ax, ay, bx, by, pu, pv):
    """Ownership test of pixel centres (arrays pu, pv) against edge a->b."""
    E = (bx - ax) * (pv - ay) - (by - ay) * (pu - ax)
    tie = (ay > by) or (ay == by and bx > ax)
    return (E > 0) | ((E == 0) & tie)


def owned_pixels(S, t, W, H):
    """(us, vs) of the pixels owned by triangle ``t`` (bounding box scan)."""
    xs = [int(S[i][0]) for i in t]
    ys = [int(S[i][1]) for i in t]
    u_lo, u_hi = max(min(xs), 0), min(max(xs), W - 1)
    v_lo, v_hi = max(min(ys), 0), min(max(ys), H - 1)
    if u_lo > u_hi or v_lo > v_hi:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    vv, uu = np.mgrid[v_lo:v_hi + 1, u_lo:u_hi + 1]
    uu = uu.ravel().astype(np.int64)
    vv = vv.ravel().astype(np.int64)
    m = np.ones(uu.shape, dtype=bool)
    for k in range(3):
        ax, ay = xs[k], ys[k]
        bx, by = xs[(k + 1) % 3], ys[(k + 1) % 3]
        m &= _inside_edge(ax, ay, bx, by, uu, vv)
    return uu[m], vv[m]


def interpolate(S: Sequence, tris, W: int, H: int) -> np.ndarray:
    """DisparityInterpolation: float32 [H, W], NaN where no triangle owns the pixel."""
    D = np.full((H, W), np.nan, dtype=F32)
    owner = np.full((H, W), -1, dtype=np.int64)
    for k, t in enumerate(tris):
        a, b, d0, u0, v0 = plane_of(S, t)
        us, vs = owned_pixels(S, t, W, H)
        if us.size == 0:
            continue
        assert (owner[vs, us] < 0).all(), "pixel owned by two triangles"
        owner[vs, us] = k
        t1 = a * (us - u0).astype(F32)
        t2 = b * (vs - v0).astype(F32)
        D[vs, us] = (d0 + t1) + t2
    return D
