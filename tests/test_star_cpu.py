"""CPU check of the device triangulation steps (csrc/mesh_star.hpp: per-point Delaunay
stars over a bucket grid) against the oracle's Delaunay triangulation (Sec. III-A, the
mesh G(S)): a small C++ driver runs the same steps with one lane per point, in shuffled
point order, and the triangle list of every batch's points so far must equal the
oracle's. Covers random sets, lattices (co-circular quadruples everywhere: the tie-break
of the perturbed in-circle test), point sets with large holes and clusters (the walk's
square widened, disks reaching far outside it), collinear and tiny sets (no triangle, or
hull edges only), frame corners and borders, and duplicates (an error, never triangles).
The host triangulation (mode 0 of the driver) is checked the same way."""
import numpy as np
import pytest

import oracle
from mesh_driver_build import build_driver, run_driver

ERR_DUP = 20  # two supports on one pixel


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = build_driver(tmp_path_factory.mktemp("mesh"))
    if out is None:
        pytest.skip("g++ not available")
    return out


def _run(driver, W, H, batches, mode=4):
    lines = [f"{W} {H} {len(batches)} {mode}"]
    for b in batches:
        lines.append(str(len(b)))
        lines += [f"{u} {v}" for (u, v) in b]
    it = iter(run_driver(driver, "\n".join(lines) + "\n").split("\n"))
    out = []
    for _ in batches:
        head = next(it).split()
        n, status = int(head[2]), int(head[3])
        tris = [tuple(int(x) for x in next(it).split()) for _ in range(n)]
        out.append((status, tris))
    return out


def _dedup(batches):
    seen, out = set(), []
    for b in batches:
        nb = []
        for q in b:
            if q not in seen:
                seen.add(q)
                nb.append(q)
        out.append(nb)
    return out


def _cases():
    rng = np.random.default_rng(2016)
    cases = []
    for c in range(16):  # random and lattice first batches, then random later batches
        kind = c % 2
        W, H = int(rng.integers(30, 160)), int(rng.integers(20, 120))
        if kind == 0:
            first = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(int(rng.integers(10, 120)))]
        else:
            st = int(rng.integers(3, 9))
            first = [(x, y) for y in range(1, H, st) for x in range(2, W, st)]
        batches = [first]
        for _ in range(2):
            batches.append([(int(rng.integers(0, W)), int(rng.integers(0, H)))
                            for _ in range(int(rng.integers(5, 120)))])
        cases.append((f"mix{c}_kind{kind}", W, H, _dedup(batches)))
    for c in range(12):  # lattice subsets with a large hole, plus scattered points
        W, H = int(rng.integers(40, 300)), int(rng.integers(30, 200))
        step = int(rng.integers(4, 12))
        pts = [(x, y) for y in range(step // 2, H, step) for x in range(step // 2, W, step) if rng.random() < 0.6]
        hx, hy, hr = rng.integers(0, W), rng.integers(0, H), rng.integers(5, 60)
        pts = [p for p in pts if (p[0] - hx) ** 2 + (p[1] - hy) ** 2 > hr * hr]
        extra = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(int(rng.integers(0, 50)))]
        cases.append((f"holes{c}", W, H, _dedup([pts, extra])))
    for c in range(4):  # a few tight clusters far apart: long edges across empty cells
        W, H = 400, 300
        pts = []
        for _ in range(int(rng.integers(2, 5))):
            cx, cy = int(rng.integers(10, W - 10)), int(rng.integers(10, H - 10))
            pts += [(min(W - 1, max(0, cx + int(rng.integers(-6, 7)))), min(H - 1, max(0, cy + int(rng.integers(-6, 7)))))
                    for _ in range(int(rng.integers(3, 25)))]
        cases.append((f"clusters{c}", W, H, _dedup([pts])))
    cases.append(("corners", 64, 48, [[(0, 0), (63, 0), (0, 47), (63, 47)], [(31, 23), (0, 23), (63, 24)]]))
    cases.append(("borders", 100, 80, [[(x, 0) for x in range(0, 100, 9)] + [(x, 79) for x in range(3, 100, 11)] +
                                        [(0, y) for y in range(5, 80, 13)] + [(99, y) for y in range(2, 80, 7)]]))
    cases.append(("collinear", 50, 50, [[(x, 10) for x in range(0, 50, 3)], [(x, 10) for x in range(1, 50, 3)]]))
    cases.append(("vertical", 50, 50, [[(7, y) for y in range(0, 50, 4)]]))
    cases.append(("diagonal", 50, 50, [[(x, x) for x in range(0, 50, 3)], [(40, 3)]]))
    cases.append(("three", 50, 50, [[(1, 1), (40, 2), (3, 45)]]))
    cases.append(("two", 50, 50, [[(1, 1), (40, 2)]]))
    cases.append(("one", 50, 50, [[(7, 9)]]))
    cases.append(("none", 50, 50, [[]]))
    cases.append(("two_rows", 300, 40, [[(x, 10) for x in range(0, 300, 5)] + [(x, 30) for x in range(2, 300, 7)]]))
    # fans at a frame border: two points on the first column and a second column with a long
    # gap, then a lattice: the border points' walks step along long thin triangles (squares
    # without a point left of the edge, the other end's square, the walk's square growing)
    fan = [(5, 35), (5, 45)] + [(15, y) for y in range(35, 190, 10)] + [(15, y) for y in range(425, 480, 10)]
    fan += [(x, y) for y in range(5, 480, 10) for x in range(35, 200, 10)]
    cases.append(("border_fan", 240, 480, [fan, [(5, 300), (25, 250)]]))
    holes = [(x, y) for y in range(5, 200, 10) for x in range(5, 300, 10)
             if (x - 150) ** 2 + (y - 100) ** 2 > 70 ** 2 or (x, y) in ((150, 105), (145, 95))]
    cases.append(("hole_hub", 300, 200, [holes]))
    return cases


_CASES = _cases()


@pytest.mark.parametrize("mode", [4, 0], ids=["stars", "host"])
@pytest.mark.parametrize("name,W,H,batches", _CASES, ids=[c[0] for c in _CASES])
def test_triangulation_equals_oracle(driver, name, W, H, batches, mode):
    got = _run(driver, W, H, batches, mode)
    pts = []
    for b, (status, tris) in zip(batches, got):
        pts += b
        assert status == 0, name
        ref = oracle.triangulate([(u, v) for (u, v) in pts], W)
        assert tris == [tuple(t) for t in ref], name


def test_stars_large_random_frame(driver):
    """A VGA frame of a few thousand supports, denser in some regions than in others (the
    support density of a textured scene), with lattice runs: equal to the oracle."""
    rng = np.random.default_rng(33)
    W, H = 640, 480
    pts = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(1500)]
    pts += [(int(rng.integers(100, 260)), int(rng.integers(50, 150))) for _ in range(1500)]
    pts += [(x, y) for y in range(300, H, 10) for x in range(400, W, 10)]
    pts = list(dict.fromkeys(pts))
    (status, tris), = _run(driver, W, H, [pts])
    assert status == 0
    assert tris == [tuple(t) for t in oracle.triangulate(pts, W)]


def test_stars_duplicate_is_an_error(driver):
    """Two points on one pixel: the star steps report it (the frame goes to the host path)
    and write no triangle."""
    (status, tris), = _run(driver, 50, 50, [[(1, 1), (20, 3), (5, 30), (20, 3)]])
    assert status == ERR_DUP and tris == []


def test_stars_independent_of_point_order(driver):
    """The same points in another input order: the same triangles up to the renumbering."""
    rng = np.random.default_rng(4)
    W, H = 120, 90
    pts = list(dict.fromkeys((int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(300)))
    perm = rng.permutation(len(pts))
    shuffled = [pts[i] for i in perm]
    (s0, t0), = _run(driver, W, H, [pts])
    (s1, t1), = _run(driver, W, H, [shuffled])
    assert s0 == 0 and s1 == 0

    def canon(tris, P):
        return sorted(tuple(P[i] for i in t) for t in tris)
    assert canon(t0, pts) == canon(t1, shuffled)
