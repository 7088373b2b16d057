"""CPU check of the device mesh insertion steps (csrc/mesh_core.hpp) against the oracle's
Delaunay triangulation (Sec. III-A): a small C++ driver runs the per-item propose /
execute steps one item after another in shuffled order, starting from the host
triangulation of the first batch, and the triangle list after every batch must equal
the oracle's triangulation of all points so far. Covers random sets, lattices (many
co-circular quadruples: the tie-break of the perturbed in-circle test), points on hull
edges, duplicates of mesh vertices and several batches."""
import numpy as np
import pytest

import oracle
from mesh_driver_build import build_driver, run_driver


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = build_driver(tmp_path_factory.mktemp("mesh_core"))
    if out is None:
        pytest.skip("g++ not available")
    return out


def _run(driver, W, H, batches, mode=0):
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


def _inside_hull(points, cand):
    """Candidates inside the closed convex hull of points (monotone chain)."""
    P = sorted(set(points))
    if len(P) < 3:
        return []

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    lo, hi = [], []
    for p in P:
        while len(lo) >= 2 and cross(lo[-2], lo[-1], p) <= 0:
            lo.pop()
        lo.append(p)
    for p in reversed(P):
        while len(hi) >= 2 and cross(hi[-2], hi[-1], p) <= 0:
            hi.pop()
        hi.append(p)
    hull = lo[:-1] + hi[:-1]
    return [q for q in cand if all(cross(hull[i], hull[(i + 1) % len(hull)], q) >= 0 for i in range(len(hull)))]


def _cases():
    rng = np.random.default_rng(2016)
    cases = []
    for c in range(24):
        kind = c % 4
        W, H = int(rng.integers(30, 120)), int(rng.integers(20, 90))
        if kind == 0:   # random first batch
            first = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(int(rng.integers(10, 80)))]
        else:           # lattice: co-circular quadruples everywhere
            st = int(rng.integers(3, 9))
            first = [(x, y) for y in range(1, H, st) for x in range(2, W, st)]
        first = list(dict.fromkeys(first))
        xs = [p[0] for p in first]
        ys = [p[1] for p in first]
        batches = [first]
        seen = set(first)
        for _ in range(2):
            cand = []
            for _ in range(int(rng.integers(5, 120))):
                q = (int(rng.integers(min(xs), max(xs) + 1)), int(rng.integers(min(ys), max(ys) + 1)))
                if kind == 2 and rng.random() < 0.5:       # on the bounding rows (hull edges of a lattice)
                    q = (q[0], min(ys) if rng.random() < 0.5 else max(ys))
                if kind == 3 and rng.random() < 0.3:       # a vertex already in the mesh
                    q = first[int(rng.integers(0, len(first)))]
                cand.append(q)
            cand = _inside_hull(first, cand)
            batch = []
            for q in cand:  # duplicates within a batch are order-dependent: keep the first
                if q not in batch:
                    batch.append(q)
            batches.append(batch)
            seen.update(batch)
        cases.append((f"case{c}_kind{kind}", W, H, batches))
    return cases


@pytest.mark.parametrize("name,W,H,batches", _cases(), ids=[c[0] for c in _cases()])
def test_device_insertion_steps_equal_oracle(driver, name, W, H, batches):
    got = _run(driver, W, H, batches)
    pts = []
    for b, (status, tris) in zip(batches, got):
        pts += b
        assert status == 0
        ref = oracle.triangulate([(u, v) for (u, v) in pts], W)
        assert tris == [tuple(t) for t in ref], name


@pytest.mark.parametrize("links", ["hash", "pairs"])
@pytest.mark.parametrize("name,W,H,batches", _cases(), ids=[c[0] for c in _cases()])
def test_device_start_mesh_equals_oracle(driver, name, W, H, batches, links):
    """The first batch built on the device from supports in raster order (rows, ladders,
    hull pockets, edge links through the hash table or by pairing undirected edges,
    Lawson flips), then the later batches inserted."""
    first = sorted(batches[0], key=lambda p: (p[1], p[0]))
    if len({p[1] for p in first}) < 2:
        pytest.skip("one row: no triangle")
    batches = [first] + batches[1:]
    got = _run(driver, W, H, batches, mode=1 if links == "hash" else 2)
    pts = []
    for b, (status, tris) in zip(batches, got):
        pts += b
        assert status == 0, name
        ref = oracle.triangulate([(u, v) for (u, v) in pts], W)
        assert tris == [tuple(t) for t in ref], name

