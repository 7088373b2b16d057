"""Seeded synthetic rectified stereo pairs.

This module only makes inputs. It renders scenes built from textured planar
surfaces into a left/right ``uint8`` pair plus the ground-truth disparity, and it
holds no step of the stereo method itself (no census, matching, triangulation,
interpolation or validation). The CPU oracle tests, the GPU parity tests and the
benchmark all draw their inputs from here, so both sides of every comparison see
the same bytes.

Geometry. Every surface ``k`` is a plane in disparity space written in left-image
coordinates, ``d = a*u + b*v + c`` (the disparity-plane form of the paper's
interpolation section, Eq. 3), limited to a region of the left image. The left
image shows, at every pixel, the surface with the largest disparity (the nearest
one). A right-image pixel ``(u_r, v)`` sees surface ``k`` at the left abscissa
``u_l = (u_r + b*v + c) / (1 - a)``, i.e. at disparity ``u_l - u_r``; again the
nearest surface whose region contains ``u_l`` wins. Texture is a function of the
surface's left coordinates, sampled continuously, so both views are consistent.

Texture. Two octaves of value noise: lattice pitches 8 px (weight 0.65) and 2 px
(weight 0.35), lattice values uniform in [0, 1) from ``numpy.random.default_rng``,
bilinear interpolation with smoothstep weights, mapped to [24, 232]. Untextured
patches are the constant 128. Independent Gaussian noise is then added to each
image, rounded half-to-even and clipped to ``uint8``.

Workloads. ``CONFIGS`` lists the five workloads (sizes, disparity ranges,
census windows, iteration counts, thresholds); ``make_scene(config, seed)``
renders one frame of workloads 1-3, ``make_rect_scene`` renders the rectangle
scene at any resolution (used for the mixed-size batch and stream workloads),
and ``slanted_plane`` / ``fronto_shift`` make the special scenes used to pin
the oracle (one slanted plane, a pure horizontal shift).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

INF = float("inf")

# ----------------------------------------------------------------------------------
# Workloads. Thresholds are raw Hamming distances (validation threshold tau = t_hi,
# confidence threshold t_lo = tau // 2); grad_thr is the high-gradient threshold.
# ----------------------------------------------------------------------------------
CONFIGS = {
    1: dict(name="qvga_4planes", W=320, H=240, census_w=5, census_h=5, d_min=0, d_max=63,
            support_step=10, n_iters=1, t_hi=8, t_lo=4, grad_thr=16, lr_tol=1,
            uniqueness=1, sz_occ0=32, sigma=2.0),
    2: dict(name="vga_20planes", W=640, H=480, census_w=7, census_h=7, d_min=0, d_max=127,
            support_step=10, n_iters=3, t_hi=12, t_lo=6, grad_thr=16, lr_tol=1,
            uniqueness=1, sz_occ0=32, sigma=2.0),
    3: dict(name="drive_1242x375_boxes", W=1242, H=375, census_w=7, census_h=7, d_min=0,
            d_max=191, support_step=10, n_iters=3, t_hi=12, t_lo=6, grad_thr=16, lr_tol=1,
            uniqueness=1, sz_occ0=32, sigma=2.0, tau_sweep=(8, 12, 16)),
    4: dict(name="batch64_mixed", sizes=((320, 240), (640, 480), (1242, 375), (1280, 720)),
            per_size=16, d_ranges=(64, 128, 192, 256), census_w=7, census_h=7,
            support_step=10, n_iters=3, t_hi=12, t_lo=6, grad_thr=16, lr_tol=1,
            uniqueness=1, sz_occ0=32, sigma=2.0),
    5: dict(name="serve16_streams", sizes=((640, 480), (1280, 720), (1920, 1080)),
            n_streams=16, rate_hz=30.0, seconds=10.0, d_min=0, d_max=255, census_w=7,
            census_h=7, support_step=10, n_iters=3, t_hi=12, t_lo=6, grad_thr=16,
            lr_tol=1, uniqueness=1, sz_occ0=32, sigma=2.0),
}

PARAM_KEYS = ("d_min", "d_max", "census_w", "census_h", "support_step", "n_iters", "t_hi",
              "t_lo", "grad_thr", "lr_tol", "uniqueness", "sz_occ0")


def params_of(config: int, **override) -> dict:
    """Method parameters of a workload as a plain dict (names as in the C header)."""
    cfg = CONFIGS[config]
    p = {k: cfg[k] for k in PARAM_KEYS if k in cfg}
    p.setdefault("d_min", 0)
    p.update(override)
    return p


def seed_of(config: int, frame: int) -> int:
    """Seed convention: 1000 * config + frame."""
    return 1000 * config + frame


# ----------------------------------------------------------------------------------
# Surfaces and texture
# ----------------------------------------------------------------------------------
@dataclass
class Surface:
    a: float
    b: float
    c: float
    rect: Tuple[float, float, float, float]  # (u0, v0, u1, v1), half-open, left coords
    lat8: np.ndarray = field(repr=False, default=None)
    lat2: np.ndarray = field(repr=False, default=None)
    flat: List[Tuple[float, float, float, float]] = field(default_factory=list)
    textured: bool = True


@dataclass
class Scene:
    left: np.ndarray        # uint8 [H, W]
    right: np.ndarray       # uint8 [H, W]
    disp: np.ndarray        # float32 [H, W], ground-truth disparity of the left view
    visible: np.ndarray     # bool [H, W], left pixel visible in the right view
    textured: np.ndarray    # bool [H, W], left pixel lies on textured surface area
    params: dict            # method parameters of the workload (empty for custom scenes)
    name: str = ""
    seed: int = 0

    @property
    def shape(self):
        return self.left.shape


_LAT_LO = -16.0   # lattice origin (both axes), px
_LAT_PAD = 320.0  # lattice margin beyond the image on the right/bottom, px


def _new_lattice(rng, W, H, pitch):
    nu = int(np.ceil((W + _LAT_PAD - _LAT_LO) / pitch)) + 2
    nv = int(np.ceil((H + 16.0 - _LAT_LO) / pitch)) + 2
    return rng.random((nv, nu))


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def _value_noise(lat, pitch, x, y):
    gx = (x - _LAT_LO) / pitch
    gy = (y - _LAT_LO) / pitch
    gx = np.clip(gx, 0.0, lat.shape[1] - 1.000001)
    gy = np.clip(gy, 0.0, lat.shape[0] - 1.000001)
    i = np.floor(gx).astype(np.int64)
    j = np.floor(gy).astype(np.int64)
    sx = _smoothstep(gx - i)
    sy = _smoothstep(gy - j)
    top = (1.0 - sx) * lat[j, i] + sx * lat[j, i + 1]
    bot = (1.0 - sx) * lat[j + 1, i] + sx * lat[j + 1, i + 1]
    return (1.0 - sy) * top + sy * bot


def _texture(s: Surface, x, y):
    if not s.textured:
        return np.full(np.shape(x), 128.0)
    n = 0.65 * _value_noise(s.lat8, 8.0, x, y) + 0.35 * _value_noise(s.lat2, 2.0, x, y)
    val = 24.0 + 208.0 * n
    for (u0, v0, u1, v1) in s.flat:
        m = (x >= u0) & (x < u1) & (y >= v0) & (y < v1)
        val = np.where(m, 128.0, val)
    return val


def _in_rect(rect, x, y):
    u0, v0, u1, v1 = rect
    return (x >= u0) & (x < u1) & (y >= v0) & (y < v1)


def _flat_mask(s: Surface, x, y):
    if not s.textured:
        return np.ones(np.shape(x), dtype=bool)
    m = np.zeros(np.shape(x), dtype=bool)
    for r in s.flat:
        m |= _in_rect(r, x, y)
    return m


def render(W: int, H: int, surfaces: List[Surface], rng, sigma: float) -> Tuple:
    """Render the left/right views of ``surfaces`` (see the module docstring)."""
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    # left view: nearest surface at each pixel
    best_d = np.full((H, W), -INF)
    best_k = np.full((H, W), -1, dtype=np.int64)
    for k, s in enumerate(surfaces):
        d = s.a * uu + s.b * vv + s.c
        m = _in_rect(s.rect, uu, vv) & (d > best_d)
        best_d = np.where(m, d, best_d)
        best_k = np.where(m, k, best_k)
    if (best_k < 0).any():
        raise ValueError("surfaces leave left-image pixels uncovered")
    left = np.zeros((H, W))
    textured = np.zeros((H, W), dtype=bool)
    for k, s in enumerate(surfaces):
        m = best_k == k
        if m.any():
            left[m] = _texture(s, uu[m], vv[m])
            textured[m] = ~_flat_mask(s, uu[m], vv[m])
    # right view: nearest surface along each right-image pixel's ray
    rbest_d = np.full((H, W), -INF)
    rbest_k = np.full((H, W), -1, dtype=np.int64)
    rbest_ul = np.zeros((H, W))
    for k, s in enumerate(surfaces):
        ul = (uu + s.b * vv + s.c) / (1.0 - s.a)
        d = ul - uu
        m = _in_rect(s.rect, ul, vv) & (d > rbest_d)
        rbest_d = np.where(m, d, rbest_d)
        rbest_k = np.where(m, k, rbest_k)
        rbest_ul = np.where(m, ul, rbest_ul)
    if (rbest_k < 0).any():
        raise ValueError("surfaces leave right-image pixels uncovered")
    right = np.zeros((H, W))
    for k, s in enumerate(surfaces):
        m = rbest_k == k
        if m.any():
            right[m] = _texture(s, rbest_ul[m], vv[m])
    # visibility of each left pixel in the right view
    ur = uu - best_d
    visible = (ur >= 0.0) & (ur <= W - 1.0)
    for k, s in enumerate(surfaces):
        ul = (ur + s.b * vv + s.c) / (1.0 - s.a)
        d = ul - ur
        occl = _in_rect(s.rect, ul, vv) & (d > best_d + 1e-6) & (best_k != k)
        visible &= ~occl
    if sigma > 0:
        left = left + rng.normal(0.0, sigma, size=left.shape)
        right = right + rng.normal(0.0, sigma, size=right.shape)
    left8 = np.clip(np.rint(left), 0, 255).astype(np.uint8)
    right8 = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    return left8, right8, best_d.astype(np.float32), visible, textured


def _surface(rng, W, H, a, b, c, rect, textured=True):
    return Surface(a=float(a), b=float(b), c=float(c), rect=rect,
                   lat8=_new_lattice(rng, W, H, 8.0), lat2=_new_lattice(rng, W, H, 2.0),
                   textured=textured)


def _plane_in_range(rng, rect_eval, dlo, dhi, slope):
    """Random slanted plane whose disparity stays in [dlo, dhi] over ``rect_eval``."""
    u0, v0, u1, v1 = rect_eval
    corners = [(u0, v0), (u1, v0), (u0, v1), (u1, v1)]
    a = rng.uniform(-slope, slope)
    b = rng.uniform(-slope, slope)
    vals = [a * u + b * v for (u, v) in corners]
    span = max(vals) - min(vals)
    if span > 0.8 * (dhi - dlo):
        f = 0.8 * (dhi - dlo) / span
        a, b = a * f, b * f
        vals = [x * f for x in vals]
    lo = dlo - min(vals)
    hi = dhi - max(vals)
    c = rng.uniform(lo, hi)
    return a, b, c


# ----------------------------------------------------------------------------------
# Workload scenes
# ----------------------------------------------------------------------------------
def scene_four_planes(W, H, seed, sigma=2.0, dlo=4.0, dhi=60.0) -> Scene:
    """Four slanted planes on a 2x2 split with a jittered split point."""
    rng = np.random.default_rng(seed)
    su = W / 2 + rng.uniform(-0.15, 0.15) * W
    sv = H / 2 + rng.uniform(-0.15, 0.15) * H
    quads = [(-INF, -INF, su, sv), (su, -INF, INF, sv), (-INF, sv, su, INF), (su, sv, INF, INF)]
    evals = [(0, 0, su, sv), (su, 0, W, sv), (0, sv, su, H), (su, sv, W, H)]
    surfaces = []
    for q, e in zip(quads, evals):
        a, b, c = _plane_in_range(rng, e, dlo, dhi, 0.1)
        surfaces.append(_surface(rng, W, H, a, b, c, q))
    surfaces.append(_surface(rng, W, H, 0.0, 0.0, 1.0, (-INF, -INF, INF, INF)))
    l, r, d, vis, tex = render(W, H, surfaces, rng, sigma)
    return Scene(l, r, d, vis, tex, {}, "four_planes", seed)


def make_rect_scene(W, H, seed, n_rects=19, dlo=2.0, dhi=124.0, flat_frac=0.05,
                    sigma=2.0) -> Scene:
    """Background plane plus ``n_rects`` slanted rectangles (sides 40-200 px, scaled
    with the image width) and untextured patches covering about ``flat_frac``."""
    rng = np.random.default_rng(seed)
    scale = W / 640.0
    bg_d = (dlo, min(dhi, dlo + 0.25 * (dhi - dlo)))
    a, b, c = _plane_in_range(rng, (0, 0, W, H), bg_d[0], bg_d[1], 0.03)
    surfaces = [_surface(rng, W, H, a, b, c, (-INF, -INF, INF, INF))]
    for _ in range(n_rects):
        w = rng.uniform(40, 200) * scale
        h = rng.uniform(40, 200) * scale
        u0 = rng.uniform(-0.1 * W, W - 0.5 * w)
        v0 = rng.uniform(-0.1 * H, H - 0.5 * h)
        rect = (u0, v0, u0 + w, v0 + h)
        a, b, c = _plane_in_range(rng, rect, dlo, dhi, 0.1)
        surfaces.append(_surface(rng, W, H, a, b, c, rect))
    target = flat_frac * W * H
    if flat_frac > 0:
        # visibility does not depend on texture: compute the nearest surface once, then
        # add untextured patches (texture coordinates = left coordinates) until enough
        # visible pixels are untextured
        vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
        best_d = np.full((H, W), -INF)
        best_k = np.full((H, W), -1, dtype=np.int64)
        for k, s in enumerate(surfaces):
            d = s.a * uu + s.b * vv + s.c
            m = _in_rect(s.rect, uu, vv) & (d > best_d)
            best_d = np.where(m, d, best_d)
            best_k = np.where(m, k, best_k)
        flat = np.zeros((H, W), dtype=bool)
        for _attempt in range(200):
            if flat.sum() >= target:
                break
            k = int(rng.integers(0, len(surfaces)))
            w = rng.uniform(30, 90) * scale
            h = rng.uniform(30, 90) * scale
            u0 = rng.uniform(0, W - w)
            v0 = rng.uniform(0, H - h)
            surfaces[k].flat.append((u0, v0, u0 + w, v0 + h))
            r0, r1 = int(np.ceil(v0)), int(np.ceil(v0 + h))
            c0, c1 = int(np.ceil(u0)), int(np.ceil(u0 + w))
            flat[r0:r1, c0:c1] |= best_k[r0:r1, c0:c1] == k
    l, r, d, vis, tex = render(W, H, surfaces, rng, sigma)
    return Scene(l, r, d, vis, tex, {}, "rects", seed)


def scene_drive(W, H, seed, n_boxes=30, sigma=2.0, d_bottom=120.0, d_far=1.0,
                box_d=(8.0, 180.0)) -> Scene:
    """Driving-camera shape: ground plane below the horizon, a far background plane
    and fronto-parallel boxes standing on the ground at random depths."""
    rng = np.random.default_rng(seed)
    vh = 0.4 * H
    k = d_bottom / (H - 1 - vh)
    surfaces = [_surface(rng, W, H, 0.0, 0.0, d_far, (-INF, -INF, INF, INF)),
                _surface(rng, W, H, 0.0, k, -k * vh, (-INF, vh, INF, INF))]
    for _ in range(n_boxes):
        d = rng.uniform(*box_d)
        vbase = vh + d / k
        h = min(1.2 * d, 0.9 * H)
        w = min(1.5 * d, 0.4 * W)
        uc = rng.uniform(0, W)
        rect = (uc - w / 2, vbase - h, uc + w / 2, vbase)
        surfaces.append(_surface(rng, W, H, 0.0, 0.0, d, rect))
    l, r, d, vis, tex = render(W, H, surfaces, rng, sigma)
    return Scene(l, r, d, vis, tex, {}, "drive", seed)


def make_scene(config: int, seed: int, **param_override) -> Scene:
    """One frame of workload 1, 2 or 3 with that workload's method parameters."""
    cfg = CONFIGS[config]
    if config == 1:
        sc = scene_four_planes(cfg["W"], cfg["H"], seed, sigma=cfg["sigma"])
    elif config == 2:
        sc = make_rect_scene(cfg["W"], cfg["H"], seed, sigma=cfg["sigma"])
    elif config == 3:
        sc = scene_drive(cfg["W"], cfg["H"], seed, sigma=cfg["sigma"])
    else:
        raise ValueError("make_scene covers workloads 1-3; use make_rect_scene for 4-5")
    sc.params = params_of(config, **param_override)
    sc.name = cfg["name"]
    return sc


# ----------------------------------------------------------------------------------
# Special scenes used to pin the oracle
# ----------------------------------------------------------------------------------
def slanted_plane(W, H, d0, p, q, g=10, seed=0, sigma=0.0) -> Scene:
    """One textured plane ``d(u,v) = d0 + p*(u - g//2)/g + q*(v - g//2)/g``.

    With integers ``d0, p, q`` the disparity is an integer at every node of the
    support grid of pitch ``g``."""
    rng = np.random.default_rng(seed)
    a = p / g
    b = q / g
    c = d0 - a * (g // 2) - b * (g // 2)
    s = _surface(rng, W, H, a, b, c, (-INF, -INF, INF, INF))
    l, r, d, vis, tex = render(W, H, [s], rng, sigma)
    return Scene(l, r, d, vis, tex, {}, "slanted_plane", seed)


def fronto_shift(W, H, d, seed=0) -> Scene:
    """Pure horizontal shift without noise: ``right(u, v) = left(u + d, v)``."""
    rng = np.random.default_rng(seed)
    s = _surface(rng, W, H, 0.0, 0.0, float(d), (-INF, -INF, INF, INF))
    l, r, dd, vis, tex = render(W, H, [s], rng, 0.0)
    return Scene(l, r, dd, vis, tex, {}, "fronto_shift", seed)


def fan_pair(W, H, d=20, seed=0) -> Tuple[np.ndarray, np.ndarray]:
    """A flat grey pair with two random-textured spots that both shift by ``d``: a band of
    15 rows around row 405 and a 9 x 9 patch at the top of the centre column. The support
    grid then finds one point at the top and one row of points near row 405 (nothing in
    between), whose Delaunay mesh is a fan of about W / 10 long triangles around the top
    point: the case of a mesh vertex with far more triangles than any natural scene."""
    rng = np.random.default_rng(seed)
    left = np.full((H, W), 128, np.uint8)
    left[398:413, :] = rng.integers(0, 256, size=(15, W), dtype=np.uint8)
    left[1:10, W // 2 + 1:W // 2 + 10] = rng.integers(0, 256, size=(9, 9), dtype=np.uint8)
    right = np.full((H, W), 128, np.uint8)
    right[:, :W - d] = left[:, d:]
    return left, right


def random_pair(W, H, seed) -> Tuple[np.ndarray, np.ndarray]:
    """Two independent uniform-random uint8 images (for census/matching edge cases)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 256, size=(H, W), dtype=np.uint8),
            rng.integers(0, 256, size=(H, W), dtype=np.uint8))


def stream_schedule(seed: int, n_streams=16, rate_hz=30.0, seconds=10.0):
    """Poisson frame arrivals per stream: list of (t_arrival_s, stream_id), sorted."""
    out = []
    for s in range(n_streams):
        rng = np.random.default_rng(seed * 100 + s)
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= seconds:
                break
            out.append((t, s))
    out.sort()
    return out
