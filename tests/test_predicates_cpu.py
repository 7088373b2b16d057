"""CPU pin of the device in-circle predicate (csrc/predicates.hpp) at the largest
coordinates the library accepts (0..8191): the double-precision filter must never decide
a wrong sign, must decide every determinant beyond its threshold plus its error bound,
and must hand exact ties to the perturbation rule; the perturbed sign must equal the
oracle's (Sec. III-A Delaunay; ties by Simulation of Simplicity). Exact values come from
Python integers; the driver runs the C++ functions themselves."""
import numpy as np
import pytest

import oracle
from mesh_driver_build import build_driver, run_driver

THRESH = 64     # the filter decides when |double determinant| > 64
ERR = 9         # its worst-case rounding error for coordinates in [0, 8191]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = build_driver(tmp_path_factory.mktemp("pred"))
    if out is None:
        pytest.skip("g++ not available")
    return out


def _ccw(a, b, c):
    return (a, b, c) if oracle.orient(a, b, c) > 0 else (a, c, b)


def _run(driver, quads):
    text = f"0 0 {len(quads)} 3\n" + "\n".join(" ".join(f"{x} {y}" for (x, y) in q) for q in quads) + "\n"
    out = run_driver(driver, text).split()
    return [(int(out[2 * k]), int(out[2 * k + 1])) for k in range(len(quads))]


def _double_det(a, b, c, d):
    """The filter's arithmetic in IEEE double, operation for operation."""
    fadx, fady = float(a[0] - d[0]), float(a[1] - d[1])
    fbdx, fbdy = float(b[0] - d[0]), float(b[1] - d[1])
    fcdx, fcdy = float(c[0] - d[0]), float(c[1] - d[1])
    fal, fbl, fcl = fadx * fadx + fady * fady, fbdx * fbdx + fbdy * fbdy, fcdx * fcdx + fcdy * fcdy
    return fadx * (fbdy * fcl - fcdy * fbl) - fady * (fbdx * fcl - fcdx * fbl) + fal * (fbdx * fcdy - fcdx * fbdy)


def _extreme_quads(rng, n):
    """Coordinates drawn mostly from the ends of [0, 8191], where the products of the
    determinant approach 2^54."""
    quads = []
    ends = np.array([0, 1, 2, 8189, 8190, 8191])
    while len(quads) < n:
        pts = []
        for _ in range(4):
            x = int(rng.choice(ends)) if rng.random() < 0.7 else int(rng.integers(0, 8192))
            y = int(rng.choice(ends)) if rng.random() < 0.7 else int(rng.integers(0, 8192))
            pts.append((x, y))
        if len(set(pts)) < 4 or oracle.orient(*pts[:3]) == 0:
            continue
        quads.append(_ccw(*pts[:3]) + (pts[3],))
    return quads


def _cocircular_quads(rng, n):
    """Exact ties at large coordinates: corners of axis-aligned rectangles up to
    8191 x 8191, and points of one lattice circle of radius 3315 about (4095, 4095)."""
    quads = []
    for _ in range(n // 2):
        x0, x1 = sorted(int(v) for v in rng.choice(8192, 2, replace=False))
        y0, y1 = sorted(int(v) for v in rng.choice(8192, 2, replace=False))
        corners = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        rng.shuffle(corners)
        quads.append(_ccw(*corners[:3]) + (corners[3],))
    # r = 3 * 5 * 13 * 17: r^2 is a sum of two squares in many ways
    r2 = (3 * 5 * 13 * 17) ** 2
    on = [(x, int(round((r2 - x * x) ** 0.5))) for x in range(0, 3316)]
    on = [(x, y) for (x, y) in on if x * x + y * y == r2 and y <= 4095]
    ring = sorted({(4095 + sx * x, 4095 + sy * y) for (x, y) in on for sx in (1, -1) for sy in (1, -1)})
    assert len(ring) >= 16
    while len(quads) < n:
        idx = rng.choice(len(ring), 4, replace=False)
        pts = [ring[i] for i in idx]
        if oracle.orient(*pts[:3]) == 0:
            continue
        quads.append(_ccw(*pts[:3]) + (pts[3],))
    return quads


def _near_threshold_quads(rng, n):
    """Determinants within a few dozen of +-64 (small configurations, exact in double),
    placed anywhere in the 8192 x 8192 range, up to the far corner."""
    quads = []
    while len(quads) < n:
        ox, oy = int(rng.integers(0, 8192 - 12)), int(rng.integers(0, 8192 - 12))
        if rng.random() < 0.3:
            ox, oy = 8191 - 11, 8191 - 11
        pts = [(ox + int(rng.integers(0, 12)), oy + int(rng.integers(0, 12))) for _ in range(4)]
        if len(set(pts)) < 4 or oracle.orient(*pts[:3]) == 0:
            continue
        q = _ccw(*pts[:3]) + (pts[3],)
        if 40 <= abs(oracle.incircle(*q)) <= 90:
            quads.append(q)
    return quads


def test_filter_error_bound_in_double():
    """|double determinant - exact determinant| <= 9 on extreme inputs (the bound the
    filter's threshold relies on)."""
    rng = np.random.default_rng(1)
    worst = 0.0
    for q in _extreme_quads(rng, 20000) + _cocircular_quads(rng, 2000):
        worst = max(worst, abs(_double_det(*q) - oracle.incircle(*q)))
    assert worst <= ERR, worst


@pytest.mark.parametrize("kind", ["extreme", "cocircular", "near_threshold"])
def test_filter_and_sos_against_exact(driver, kind):
    rng = np.random.default_rng({"extreme": 2, "cocircular": 3, "near_threshold": 4}[kind])
    make = {"extreme": _extreme_quads, "cocircular": _cocircular_quads, "near_threshold": _near_threshold_quads}[kind]
    quads = make(rng, 3000)
    got = _run(driver, quads)
    decided = 0
    for q, (filt, sos) in zip(quads, got):
        det = oracle.incircle(*q)
        if filt != 0:                      # a decided filter is always right
            decided += 1
            assert filt == (1 if det > 0 else -1), (q, det, filt)
        if abs(det) > THRESH + ERR:        # and it decides everything clearly beyond its threshold
            assert filt != 0, (q, det)
        if det == 0:                       # an exact tie always reaches the perturbation rule
            assert filt == 0, q
        prio = [p[1] * 8192 + p[0] for p in q]
        assert sos == oracle.incircle_sos(*q, prio), (q, det)
    if kind == "cocircular":
        assert decided == 0
    if kind == "near_threshold":           # both sides of the threshold occur
        dets = [abs(oracle.incircle(*q)) for q in quads]
        assert min(dets) <= THRESH < max(dets)
