"""CPU: the host triangulation (csrc/delaunay.cpp) and the device triangulation steps run
sequentially on the host (csrc/mesh_star.hpp and predicates.hpp, through
tests/mesh_driver.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer;
any out-of-bounds access, use after free, leak, signed overflow or misaligned access
aborts the driver and fails the test. The outputs must still equal the oracle's
triangulation (Sec. III-A)."""
import os

import numpy as np
import pytest

import oracle
from mesh_driver_build import build_driver, run_driver
from test_star_cpu import _CASES
from test_predicates_cpu import _cocircular_quads, _extreme_quads, _near_threshold_quads


@pytest.fixture(scope="module")
def san_driver(tmp_path_factory):
    try:
        out = build_driver(tmp_path_factory.mktemp("san"), sanitize=True)
    except Exception as e:  # a toolchain without the sanitizer runtimes
        pytest.skip(f"sanitizer build unavailable: {e}")
    if out is None:
        pytest.skip("g++ not available")
    return out


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    return env


@pytest.mark.parametrize("mode", [0, 4], ids=["host", "stars"])
def test_mesh_steps_under_sanitizers(san_driver, mode):
    """The host triangulation (mode 0) and the per-point stars (mode 4) on every third case
    of the triangulation suite."""
    env = _env()
    for name, W, H, batches in _CASES[::3]:
        lines = [f"{W} {H} {len(batches)} {mode}"]
        for b in batches:
            lines.append(str(len(b)))
            lines += [f"{u} {v}" for (u, v) in b]
        it = iter(run_driver(san_driver, "\n".join(lines) + "\n", env=env).split("\n"))
        pts = []
        for b in batches:
            head = next(it).split()
            n, status = int(head[2]), int(head[3])
            tris = [tuple(int(x) for x in next(it).split()) for _ in range(n)]
            pts += b
            assert status == 0, name
            assert tris == [tuple(t) for t in oracle.triangulate(pts, W)], name


def test_host_triangulation_large_under_sanitizers(san_driver):
    """A few thousand random points with collinear runs and lattice ties through the host
    triangulation alone (distinct points: duplicates are removed before it by its callers)."""
    rng = np.random.default_rng(9)
    W, H = 1242, 375
    pts = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(3000)]
    pts += [(x, 200) for x in range(0, W, 7)]            # a collinear run
    pts += [(x, y) for y in range(5, H, 40) for x in range(3, W, 40)]   # co-circular quadruples
    pts = list(dict.fromkeys(pts))
    text = f"{W} {H} 1 0\n{len(pts)}\n" + "\n".join(f"{u} {v}" for (u, v) in pts) + "\n"
    out = run_driver(san_driver, text, env=_env()).split("\n")
    head = out[0].split()
    assert int(head[3]) == 0
    tris = [tuple(int(x) for x in out[1 + k].split()) for k in range(int(head[2]))]
    assert tris == [tuple(t) for t in oracle.triangulate(pts, W)]


def test_predicates_under_sanitizers(san_driver):
    rng = np.random.default_rng(11)
    quads = _extreme_quads(rng, 300) + _cocircular_quads(rng, 300) + _near_threshold_quads(rng, 300)
    text = f"0 0 {len(quads)} 3\n" + "\n".join(" ".join(f"{x} {y}" for (x, y) in q) for q in quads) + "\n"
    got = run_driver(san_driver, text, env=_env()).split()
    for k, q in enumerate(quads):
        prio = [p[1] * 8192 + p[0] for p in q]
        assert int(got[2 * k + 1]) == oracle.incircle_sos(*q, prio)
