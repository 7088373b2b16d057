"""CPU: the Python binding rejects tensors of the wrong dtype, shape, device, layout or
count before any pointer reaches the library (the kernels trust the sizes they are
given). The checks take the device type as a parameter, so they run here on CPU
tensors, and the solver-level rejections need no GPU either."""
import numpy as np
import pytest
import torch

from paper_1511_00758_amd import api

CPU = dict(dev_type="cpu")


def _img(H=24, W=32, dtype=torch.uint8):
    return torch.zeros((H, W), dtype=dtype)


def _outs(H=24, W=32):
    return (torch.zeros((H, W), dtype=torch.float32), torch.zeros((H, W), dtype=torch.uint8),
            torch.zeros((H, W), dtype=torch.uint8))


def test_good_pair_and_outputs_pass():
    assert api.check_pair(_img(), _img(), **CPU) == (24, 32)
    api.check_outputs(*_outs(), (24, 32), torch.device("cpu"), **CPU)
    api.check_frames([(_img(), _img(), {}), (_img(8, 9), _img(8, 9), {})], [_outs(), _outs(8, 9)], **CPU)


@pytest.mark.parametrize("bad,what", [
    (_img(dtype=torch.int16), "dtype"),                 # non-uint8 image: pitch would count elements
    (_img(dtype=torch.float32), "dtype"),
    (torch.zeros((2, 24, 32), dtype=torch.uint8), "2-D"),
    (torch.zeros((32, 24), dtype=torch.uint8).t(), "contiguous"),
    (torch.zeros((2, 32), dtype=torch.uint8), "outside"),
    (np.zeros((24, 32), np.uint8), "torch tensor"),
])
def test_bad_images_rejected(bad, what):
    with pytest.raises(ValueError, match=what):
        api.check_image(bad, "left", **CPU)


def test_pair_must_match():
    with pytest.raises(ValueError, match="shape"):
        api.check_pair(_img(), _img(24, 33), **CPU)
    with pytest.raises(ValueError, match="expected a cuda tensor"):
        api.check_pair(_img(), _img())  # CPU tensors where device tensors are required


@pytest.mark.parametrize("k,bad,what", [
    (0, torch.zeros((24, 32), dtype=torch.float64), "D_f: dtype"),
    (1, torch.zeros((24, 32), dtype=torch.int32), "C_f: dtype"),
    (2, torch.zeros((24, 31), dtype=torch.uint8), "mask: shape"),
    (0, torch.zeros((24 * 32,), dtype=torch.float32), "D_f: shape"),
    (1, torch.zeros((32, 24), dtype=torch.uint8).t(), "C_f: must be contiguous"),
])
def test_bad_outputs_rejected(k, bad, what):
    outs = list(_outs())
    outs[k] = bad
    with pytest.raises(ValueError, match=what):
        api.check_outputs(*outs, (24, 32), torch.device("cpu"), **CPU)


def test_batch_output_count_must_match():
    frames = [(_img(), _img(), {}), (_img(), _img(), {})]
    with pytest.raises(ValueError, match="1 output triples for 2 frames"):
        api.check_frames(frames, [_outs()], **CPU)
    with pytest.raises(ValueError, match="frame 1: D_f: shape"):
        api.check_frames(frames, [_outs(), _outs(24, 16)], **CPU)
    with pytest.raises(ValueError, match="frame 0: right"):
        api.check_frames([(_img(), _img(dtype=torch.int8), {})], [_outs()], **CPU)


def test_check_tensor_min_numel_and_device():
    t = torch.zeros(10, dtype=torch.int64)
    api.check_tensor(t, "cell_g", torch.int64, min_numel=10, **CPU)
    with pytest.raises(ValueError, match="at least 11"):
        api.check_tensor(t, "cell_g", torch.int64, min_numel=11, **CPU)
    with pytest.raises(ValueError, match="expected meta"):
        api.check_tensor(t, "cell_g", torch.int64, device="meta", **CPU)


def test_census_pair_checks():
    api.check_census_pair(torch.zeros((4, 5), dtype=torch.int64), torch.zeros((4, 5), dtype=torch.int64), **CPU)
    with pytest.raises(ValueError, match="cR: shape"):
        api.check_census_pair(torch.zeros((4, 5), dtype=torch.int64), torch.zeros((4, 6), dtype=torch.int64), **CPU)
    with pytest.raises(ValueError, match="cL: dtype"):
        api.check_census_pair(torch.zeros((4, 5), dtype=torch.int32), torch.zeros((4, 5), dtype=torch.int64), **CPU)


def test_wrappers_reject_host_tensors_before_the_library():
    """The public wrappers refuse CPU tensors (no library call happens on them)."""
    with pytest.raises(ValueError):
        api.census(_img(), 5, 5)
    with pytest.raises(ValueError):
        api.ManySolver(device="cpu")([(_img(), _img(), {})])
    with pytest.raises(ValueError, match="triangle indices"):
        api.interpolate(torch.zeros(16, dtype=torch.uint8), 2, np.array([[0, 1, 2]]), 32, 24)


def test_set_launch_shape_checks():
    """sm_set_launch_shape accepts the documented kinds, keys and values, clears with 0, and
    rejects anything else with SM_ERR_ARG (host only: no GPU needed)."""
    from paper_1511_00758_amd import _lib
    L = _lib.load()
    ok = [(0, 4, 8), (1, 0, 2048), (2, 128, 32), (3, 3 << 8 | 3, 8), (2, 128, 0), (3, 3 << 8 | 3, 0)]
    for kind, key, value in ok:
        assert L.sm_set_launch_shape(kind, 640, 480, key, value) == 0, (kind, key, value)
    bad = [(0, 4, 3), (1, 1, 2048), (1, 0, 100), (2, 0, 32), (2, 300, 32), (2, 128, 48), (3, 0, 12), (4, 0, 8),
           (-1, 0, 8)]
    for kind, key, value in bad:
        assert L.sm_set_launch_shape(kind, 640, 480, key, value) != 0, (kind, key, value)
    assert L.sm_set_launch_shape(2, 0, 480, 128, 32) != 0  # (no such frame size)
