"""SupportResampling (Alg. 4). Test infrastructure only.

The cells are visited in raster order. A cell whose invalid record C_b is set puts
its pixel into X (pixels to re-match by epipolar search); a cell whose confident
record C_g is set adds its pixel as a new support with the interpolated disparity
D_it(u, v). X is then matched like the initial supports ("SparseEpipolarStereo")
and the matches are appended. The new support set is S_it, then the confident
supports, then the matched ones, dropping any pixel already present (S_it is a
subset of S_it+1).
"""
from .matching import sparse_stereo


def support_resampling(Cg, Cb, S, cL, cR, p):
    X = []
    confident = []
    for row_g, row_b in zip(Cg, Cb):
        for cg, cb in zip(row_g, row_b):
            if cb.set:
                X.append((cb.u, cb.v))
            if cg.set:
                confident.append((cg.u, cg.v, cg.d))
    matched = sparse_stereo(cL, cR, X, p)
    out = list(S)
    seen = {(int(s[0]), int(s[1])) for s in S}
    for s in confident + matched:
        key = (int(s[0]), int(s[1]))
        if key not in seen:
            seen.add(key)
            out.append((int(s[0]), int(s[1]), float(s[2])))
    return out, X, confident, matched
