"""Pins of the oracle's census words, Hamming costs and high-gradient set."""
import os

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_census_golden():
    cases = []
    img = win = None
    for line in open(os.path.join(GOLDEN, "census_3x3.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        if key == "image":
            img = np.array([int(v) for v in vals], dtype=np.uint8).reshape(3, 3)
        elif key == "window":
            win = (int(vals[0]), int(vals[1]))
        elif key == "centre_word":
            cases.append((img, win, int(vals[0])))
    return cases


def test_census_golden_hand_worked():
    for img, (cw, ch), word in _read_census_golden():
        words, valid = oracle.census(img, cw, ch)
        assert valid[1, 1] and valid.sum() == 1
        assert int(words[1, 1]) == word


def _census_brute(img, cw, ch):
    """Per-pixel, per-bit restatement with Python loops (independent of the oracle)."""
    H, W = img.shape
    rx, ry = cw // 2, ch // 2
    out = {}
    for v in range(ry, H - ry):
        for u in range(rx, W - rx):
            word, k = 0, 0
            for dy in range(-ry, ry + 1):
                for dx in range(-rx, rx + 1):
                    if dx == 0 and dy == 0:
                        continue
                    if int(img[v + dy, u + dx]) < int(img[v, u]):
                        word |= 1 << k
                    k += 1
            out[(u, v)] = word
    return out


@pytest.mark.parametrize("cw,ch", [(3, 3), (5, 5), (7, 7), (9, 7), (5, 3)])
def test_census_brute_force(cw, ch):
    rng = np.random.default_rng(cw * 10 + ch)
    img = rng.integers(0, 6, size=(13, 17), dtype=np.uint8)  # many equal values
    words, valid = oracle.census(img, cw, ch)
    ref = _census_brute(img, cw, ch)
    assert valid.sum() == len(ref)
    for (u, v), w in ref.items():
        assert valid[v, u]
        assert int(words[v, u]) == w
    assert (words[~valid] == 0).all()


@pytest.mark.parametrize("cw,ch", [(5, 5), (7, 7)])
def test_census_special_cases(cw, ch):
    nbits = cw * ch - 1
    const = np.full((11, 11), 77, dtype=np.uint8)
    words, valid = oracle.census(const, cw, ch)
    assert (words == 0).all()
    bright = np.full((11, 11), 10, dtype=np.uint8)
    bright[5, 5] = 200
    words, _ = oracle.census(bright, cw, ch)
    assert int(words[5, 5]) == (1 << nbits) - 1
    dark = np.full((11, 11), 200, dtype=np.uint8)
    dark[5, 5] = 10
    words, _ = oracle.census(dark, cw, ch)
    assert int(words[5, 5]) == 0


def test_census_too_small_image():
    words, valid = oracle.census(np.zeros((4, 4), np.uint8), 5, 5)
    assert not valid.any() and (words == 0).all()


def test_hamming_properties():
    rng = np.random.default_rng(3)
    xs = rng.integers(0, 2**63, size=50, dtype=np.uint64)
    for a in xs:
        assert oracle.hamming(a, a) == 0
        for b in xs[:5]:
            assert oracle.hamming(a, b) == oracle.hamming(b, a)
            assert 0 <= oracle.hamming(a, b) <= 64
    assert oracle.hamming(0, (1 << 48) - 1) == 48
    assert oracle.hamming(0b1011, 0b0110) == 3


@pytest.mark.parametrize("slope", [1, 3, 8, 9])
def test_high_gradient_ramp_closed_form(slope):
    """Horizontal ramp of slope s: the central-difference L1 gradient is exactly 2s."""
    W, H = 20, 9
    img = (np.arange(W) * slope).astype(np.uint8)[None, :].repeat(H, axis=0)
    _, valid = oracle.census(img, 5, 5)
    for thr in (2 * slope, 2 * slope + 1):
        om = oracle.high_gradient(img, valid, thr)
        assert (om == (valid & (2 * slope >= thr))).all()


def test_high_gradient_zero_threshold_is_valid_set():
    sc = scenes.make_scene(1, scenes.seed_of(1, 0))
    _, valid = oracle.census(sc.left, 5, 5)
    assert (oracle.high_gradient(sc.left, valid, 0) == valid).all()
