"""Oracle results shared by the GPU test modules of one pytest process.

The CPU oracle takes seconds per large frame (about 14 s for a 1280x720 pair with 256
disparities), and several GPU tests compare the same frames with it; each distinct
(left, right, parameters) triple is solved once. Helpers only: no test lives here.
"""
import hashlib

import numpy as np

import oracle

_CACHE = {}


def _key(left, right, params):
    h = hashlib.sha1()
    for a in (left, right):
        a = np.ascontiguousarray(a)
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    h.update(repr(sorted(params.items())).encode())
    return h.hexdigest()


def oracle_solve(left, right, params):
    """oracle.solve of the pair under ``params`` (a dict), memoised."""
    k = _key(left, right, params)
    if k not in _CACHE:
        _CACHE[k] = oracle.solve(np.ascontiguousarray(left), np.ascontiguousarray(right),
                                 oracle.Params.from_dict(params))
    return _CACHE[k]


def assert_equals_oracle(D, C, M, left, right, params, what=""):
    """Bit-exact C_f and mask, and D_f bit for bit (the 1e-3 px tolerance is never
    needed: both sides round the same float32 operations in the same order)."""
    ref = oracle_solve(left, right, params)
    D = D.cpu().numpy() if hasattr(D, "cpu") else D
    C = C.cpu().numpy() if hasattr(C, "cpu") else C
    M = M.cpu().numpy() if hasattr(M, "cpu") else M
    assert (C == ref["C_f"]).all(), f"C_f differs from the oracle {what}"
    assert (M.astype(bool) == ref["mask"]).all(), f"mask differs from the oracle {what}"
    err = float(np.nanmax(np.abs(D.astype(np.float64) - ref["D_f"].astype(np.float64)), initial=0.0))
    assert err <= 1e-3, f"D_f differs from the oracle by {err} px {what}"
    assert (D.view(np.uint32) == ref["D_f"].view(np.uint32)).all(), f"D_f bits differ from the oracle {what}"
