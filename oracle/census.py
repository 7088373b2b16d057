"""Census words and the high-gradient set. Test infrastructure only.

The cost-evaluation section of the paper validates disparities with a census
window match (5x5), citing Zabih & Woodfill's census transform: each pixel is
described by one bit per window neighbour telling whether that neighbour is darker
than the centre. Bit order (a reading, the paper does not fix it): neighbours are
taken in row-major order over the window, the centre skipped, the first neighbour
in the least significant bit; the comparison is strict.

The high-gradient subset Omega_I of Sec. III is not given an operator; the reading
used here is the L1 central difference |I(u+1,v)-I(u-1,v)| + |I(u,v+1)-I(u,v-1)|
compared with ``grad_thr``, restricted to pixels whose census window fits in the
image.
"""
import numpy as np


def census(img: np.ndarray, cw: int, ch: int):
    """Census transform of a uint8 image with a ``cw`` x ``ch`` window.

    Returns ``(words, valid)``: ``uint64[H, W]`` census words and ``bool[H, W]``.
    Pixels whose window does not fit inside the image get word 0 and valid False.
    """
    assert cw % 2 == 1 and ch % 2 == 1 and cw * ch - 1 <= 64
    H, W = img.shape
    rx, ry = (cw - 1) // 2, (ch - 1) // 2
    words = np.zeros((H, W), dtype=np.uint64)
    valid = np.zeros((H, W), dtype=bool)
    if H <= 2 * ry or W <= 2 * rx:
        return words, valid
    valid[ry:H - ry, rx:W - rx] = True
    I = img.astype(np.int32)
    centre = I[ry:H - ry, rx:W - rx]
    acc = np.zeros(centre.shape, dtype=np.uint64)
    k = 0
    for dy in range(-ry, ry + 1):          # window rows, top to bottom
        for dx in range(-rx, rx + 1):      # window columns, left to right
            if dx == 0 and dy == 0:
                continue
            nb = I[ry + dy:H - ry + dy, rx + dx:W - rx + dx]
            acc |= (nb < centre).astype(np.uint64) << np.uint64(k)
            k += 1
    words[ry:H - ry, rx:W - rx] = acc
    return words, valid


def high_gradient(img: np.ndarray, valid: np.ndarray, grad_thr: int) -> np.ndarray:
    """Omega_I: valid census pixels whose L1 central-difference gradient >= grad_thr."""
    H, W = img.shape
    I = img.astype(np.int32)
    g = np.zeros((H, W), dtype=np.int32)
    if H >= 3 and W >= 3:
        gx = np.abs(I[1:H - 1, 2:] - I[1:H - 1, :W - 2])
        gy = np.abs(I[2:, 1:W - 1] - I[:H - 2, 1:W - 1])
        g[1:H - 1, 1:W - 1] = gx + gy
    return valid & (g >= grad_thr)
