"""FAST support keypoints sampled from spatial bins (Sec. III-A). Test infrastructure only.

Sec. III-A detects the support keypoints with FAST (Rosten and Drummond's segment test)
and samples them from 12 x 10 spatial bins. The paper gives no further detail; the
readings followed here (and by the library) are:

* Segment test on the 16-pixel Bresenham circle of radius 3 around p, taken clockwise
  from the pixel straight above p. With diff_k = I(circle_k) - I(p), p is a corner for
  threshold t when some 9 contiguous circle pixels all have diff > t (all brighter than
  I(p) + t) or all have diff < -t (all darker than I(p) - t): FAST-9.
* Score: the arc contrast, max over the 16 arcs of 9 contiguous circle pixels of
  max(min diff over the arc, min (-diff) over the arc), floored at 0. p is a corner
  exactly when score > t. Pixels whose circle leaves the image score 0.
* Non-maximum suppression over the 3 x 3 neighbourhood: a corner p is a keypoint when
  every neighbour scores lower, except that a neighbour later in raster order may score
  the same (the first of equal neighbours wins).
* Bins: pixel (u, v) falls in bin (floor(u * bins_x / W), floor(v * bins_y / H)). Each
  bin keeps at most ``per_bin`` keypoints: the highest scores, ties to the earlier
  raster position.
* Output order: bins row-major; inside a bin, raster order.
"""
from typing import List, Tuple

import numpy as np

# Bresenham circle of radius 3, clockwise from the top (image rows grow downwards).
CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]
ARC = 9


def fast_score(img: np.ndarray) -> np.ndarray:
    """Arc-contrast score (int32 [H, W], 0..255) of every pixel; 0 where the circle does
    not fit (u < 3, u > W-4, v < 3, v > H-4)."""
    I = img.astype(np.int32)
    H, W = I.shape
    score = np.zeros((H, W), dtype=np.int32)
    if H < 7 or W < 7:
        return score
    c = I[3:H - 3, 3:W - 3]
    diffs = np.stack([I[3 + dy:H - 3 + dy, 3 + dx:W - 3 + dx] - c for (dx, dy) in CIRCLE])
    best = np.zeros(c.shape, dtype=np.int32)
    for s in range(16):
        arc = diffs[[(s + j) % 16 for j in range(ARC)]]
        best = np.maximum(best, arc.min(axis=0))      # all brighter by more than min
        best = np.maximum(best, (-arc).min(axis=0))   # all darker by more than min
    score[3:H - 3, 3:W - 3] = best
    return score


def keypoints(score: np.ndarray, t: int) -> np.ndarray:
    """Corners (score > t) that survive the 3 x 3 non-maximum suppression (bool [H, W])."""
    H, W = score.shape
    corner = score > t
    keep = corner.copy()
    pad = np.full((H + 2, W + 2), -1, dtype=np.int64)
    pad[1:H + 1, 1:W + 1] = score
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            nb = pad[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx]
            later = dy > 0 or (dy == 0 and dx > 0)   # neighbour after p in raster order
            if later:
                keep &= nb <= score
            else:
                keep &= nb < score
    return keep


def bin_of(u: int, v: int, W: int, H: int, bins_x: int, bins_y: int) -> Tuple[int, int]:
    return (u * bins_x) // W, (v * bins_y) // H


def fast_candidates(img: np.ndarray, t: int, bins_x: int, bins_y: int,
                    per_bin: int) -> List[Tuple[int, int]]:
    """Support candidates (u, v): FAST keypoints, at most ``per_bin`` per spatial bin,
    bins row-major and raster order inside a bin."""
    H, W = img.shape
    score = fast_score(img)
    kp = keypoints(score, t)
    bins = {}
    for v, u in zip(*np.nonzero(kp)):                 # raster order
        bins.setdefault(bin_of(int(u), int(v), W, H, bins_x, bins_y), []).append(
            (int(score[v, u]), int(v), int(u)))
    out = []
    for by in range(bins_y):
        for bx in range(bins_x):
            pts = bins.get((bx, by), [])
            best = sorted(pts, key=lambda k: (-k[0], k[1], k[2]))[:per_bin]
            out.extend((u, v) for (_, v, u) in sorted(best, key=lambda k: (k[1], k[2])))
    return out
