"""Torch-tensor wrappers of the stereomesh C ABI.

PyTorch provides device memory and the current HIP stream; every step of the method
runs in the library's kernels (or, for the triangulation, its host code). These
wrappers only allocate outputs, pass pointers and raise on a non-OK status.

Census words are returned as ``torch.int64`` tensors holding the uint64 bit patterns;
supports live in flat ``uint8`` device buffers of 8-byte records (int16 u, int16 v,
float32 d) and are converted to NumPy with ``SUPPORT_DTYPE``.
"""
import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, make_params

SUPPORT_DTYPE = np.dtype([("u", "<i2"), ("v", "<i2"), ("d", "<f4")])
TRI_DTYPE = np.dtype([("i0", "<i4"), ("i1", "<i4"), ("i2", "<i4")])


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream(stream=None, device_index=None):
    if stream is None:
        if device_index is not None:  # the raw handle, without building a Stream object
            return torch._C._cuda_getCurrentRawStream(device_index)
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# Argument checks run before any pointer reaches the library: the kernels trust the
# sizes they are given, so a tensor of the wrong dtype, shape or device would be read or
# written out of bounds. ``dev_type`` is "cuda" in use; the CPU tests pass "cpu" to
# exercise the same checks without a GPU.
def check_tensor(t, name, dtype, shape=None, device=None, dev_type="cuda", min_numel=None):
    """Raises ValueError unless ``t`` is a contiguous tensor of ``dtype`` (and ``shape``,
    on ``device``, with at least ``min_numel`` elements, when given)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != dev_type:
        raise ValueError(f"{name}: expected a {dev_type} tensor, got one on {t.device}")
    if device is not None and t.device != torch.device(device):
        raise ValueError(f"{name}: on {t.device}, expected {torch.device(device)}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, need at least {min_numel}")


def check_image(t, name="image", shape=None, device=None, dev_type="cuda"):
    """A uint8 [H, W] image (3 <= W, H <= 8192), contiguous, on ``device`` when given."""
    if isinstance(t, torch.Tensor) and t.dim() != 2:
        raise ValueError(f"{name}: expected a 2-D [H, W] image, got shape {tuple(t.shape)}")
    check_tensor(t, name, torch.uint8, shape, device, dev_type)
    H, W = t.shape
    if not (3 <= W <= 8192 and 3 <= H <= 8192):
        raise ValueError(f"{name}: size {W}x{H} outside [3, 8192]^2")


def check_pair(left, right, device=None, dev_type="cuda"):
    """Left and right uint8 images of one size on one device; returns (H, W)."""
    check_image(left, "left", None, device, dev_type)
    check_image(right, "right", tuple(left.shape), left.device if device is None else device, dev_type)
    return tuple(left.shape)


def check_outputs(D, C, M, shape, device, dev_type="cuda"):
    """Caller-given outputs of one frame: D_f float32, C_f and mask uint8, all [H, W]."""
    check_tensor(D, "D_f", torch.float32, shape, device, dev_type)
    check_tensor(C, "C_f", torch.uint8, shape, device, dev_type)
    check_tensor(M, "mask", torch.uint8, shape, device, dev_type)


def check_frames(frames, outs, dev_type="cuda"):
    """A batch: one output triple per frame, each frame's images and outputs of one size
    and on one device."""
    if len(outs) != len(frames):
        raise ValueError(f"{len(outs)} output triples for {len(frames)} frames")
    for i, ((l, r, prm), o) in enumerate(zip(frames, outs)):
        try:
            shape = check_pair(l, r, None, dev_type)
            if not isinstance(prm, dict):
                raise ValueError("parameters must be a dict")
            if len(o) != 3:
                raise ValueError("outputs must be (D_f, C_f, mask)")
            check_outputs(*o, shape, l.device, dev_type)
        except ValueError as e:
            raise ValueError(f"frame {i}: {e}") from None


def check_census_pair(cL, cR, dev_type="cuda"):
    """Census words of the left and right image: int64 [H, W], one size, one device."""
    if isinstance(cL, torch.Tensor) and cL.dim() != 2:
        raise ValueError(f"cL: expected [H, W] census words, got shape {tuple(cL.shape)}")
    check_tensor(cL, "cL", torch.int64, None, None, dev_type)
    check_tensor(cR, "cR", torch.int64, tuple(cL.shape), cL.device, dev_type)


def census(img: torch.Tensor, census_w: int, census_h: int, grad_thr: int = 0,
           with_omega: bool = True, stream=None):
    """Census words (int64 bit patterns) and Omega_I (uint8) of a uint8 [H, W] image."""
    check_image(img, "img")
    H, W = img.shape
    words = torch.empty((H, W), dtype=torch.int64, device=img.device)
    omega = torch.empty((H, W), dtype=torch.uint8, device=img.device) if with_omega else None
    L = _lib.load()
    check(L.sm_census(img.data_ptr(), W, H, img.stride(0), census_w, census_h, grad_thr,
                      words.data_ptr(), _ptr(omega), _stream(stream)))
    return words, omega


def new_support_buffer(cap: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(cap, 1) * 8, dtype=torch.uint8, device=device)


def supports_to_numpy(buf: torch.Tensor, n: int) -> np.ndarray:
    return buf[: n * 8].cpu().numpy().view(SUPPORT_DTYPE).copy()


def supports_to_device(S: np.ndarray, device="cuda") -> torch.Tensor:
    arr = np.ascontiguousarray(S, dtype=SUPPORT_DTYPE)
    if arr.size == 0:
        return new_support_buffer(1, device)
    return torch.from_numpy(arr.view(np.uint8).copy()).to(device)


def match_support(cL, cR, omega, params: dict, cand_uv=None, stream=None, n_cand=None):
    """Matched supports: (device buffer, device int32 count). ``cand_uv`` is an (n, 2)
    int16 array or device tensor of (u, v) candidates (the first ``n_cand`` rows when
    given), or None for the support grid."""
    check_census_pair(cL, cR)
    H, W = cL.shape
    if omega is not None:
        check_tensor(omega, "omega", torch.uint8, (H, W), cL.device)
    elif cand_uv is None:
        raise ValueError("omega is required for grid candidates")
    p = make_params(params)
    L = _lib.load()
    cand = None
    if cand_uv is not None:
        if isinstance(cand_uv, torch.Tensor):
            cand = cand_uv.reshape(-1, 2)
            if cand.dtype != torch.int16 or not cand.is_contiguous() or cand.device != cL.device:
                raise ValueError("cand_uv tensor must be contiguous int16 on the census device")
        else:
            cand = torch.from_numpy(np.ascontiguousarray(cand_uv, dtype=np.int16).reshape(-1, 2)).to(cL.device)
        n = cand.shape[0] if n_cand is None else int(n_cand)
        if not 0 <= n <= cand.shape[0]:
            raise ValueError(f"n_cand {n} outside [0, {cand.shape[0]}]")
    else:
        n = L.sm_grid_candidates(W, H, p.support_step)
    out = new_support_buffer(n, cL.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=cL.device)
    check(L.sm_match_support(cL.data_ptr(), cR.data_ptr(), _ptr(omega), W, H, _ptr(cand),
                             n, p, out.data_ptr(), max(n, 1), n_out.data_ptr(), _stream(stream)))
    return out, n_out


def fast_candidates(img, params: dict, stream=None):
    """FAST keypoints sampled from spatial bins: (score uint8 [H, W], candidates int16
    [cap, 2] with the first n valid, device int32 n)."""
    check_image(img, "img")
    H, W = img.shape
    p = make_params(params)
    L = _lib.load()
    cap = max(p.fast_bins_x * p.fast_bins_y * p.fast_per_bin, 1)
    score = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    cand = torch.empty((cap, 2), dtype=torch.int16, device=img.device)
    n_out = torch.zeros(1, dtype=torch.int32, device=img.device)
    check(L.sm_fast_candidates(img.data_ptr(), W, H, img.stride(0), p, score.data_ptr(),
                               cand.data_ptr(), cap, n_out.data_ptr(), _stream(stream)))
    return score, cand, n_out


def triangulate(S: np.ndarray) -> np.ndarray:
    """Delaunay triangles (int32 [T, 3]) of host supports (SUPPORT_DTYPE records)."""
    arr = np.ascontiguousarray(S, dtype=SUPPORT_DTYPE)
    n = arr.size
    cap = max(2 * n, 1)
    tris = np.zeros(cap, dtype=TRI_DTYPE)
    nt = ctypes_int()
    L = _lib.load()
    check(L.sm_triangulate(arr.ctypes.data if n else None, n, tris.ctypes.data, cap, nt))
    return tris[: nt.value].view(np.int32).reshape(-1, 3).copy()


def ctypes_int():
    import ctypes
    return ctypes.c_int32(0)


def interpolate(S_dev: torch.Tensor, n_support: int, tris: np.ndarray, W: int, H: int,
                stream=None) -> torch.Tensor:
    """D_it (float32 [H, W], NaN outside the mesh) from device supports and host triangles."""
    n_support = int(n_support)
    if not (3 <= W <= 8192 and 3 <= H <= 8192):
        raise ValueError(f"size {W}x{H} outside [3, 8192]^2")
    tri_arr = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    if tri_arr.size and (tri_arr.min() < 0 or tri_arr.max() >= n_support):
        raise ValueError(f"triangle indices must lie in [0, {n_support})")
    check_tensor(S_dev, "S_dev", torch.uint8, min_numel=8 * n_support)
    T = torch.from_numpy(tri_arr.reshape(-1)).to(S_dev.device)
    n_tris = int(T.numel() // 3)
    D = torch.empty((H, W), dtype=torch.float32, device=S_dev.device)
    L = _lib.load()
    check(L.sm_interpolate(S_dev.data_ptr(), n_support, T.data_ptr() if n_tris else None, n_tris,
                           W, H, D.data_ptr(), _stream(stream)))
    if stream is not None:
        T.record_stream(stream)
    return D


def validate(cL, cR, omega, D_it, params: dict, sz_occ: int, D_f, C_f, want_C_it=True,
             stream=None):
    """Cost evaluation + refinement; returns (C_it or None, cell_g, cell_b). D_f, C_f are
    updated in place."""
    check_census_pair(cL, cR)
    H, W = cL.shape
    dev = cL.device
    check_tensor(omega, "omega", torch.uint8, (H, W), dev)
    check_tensor(D_it, "D_it", torch.float32, (H, W), dev)
    check_tensor(D_f, "D_f", torch.float32, (H, W), dev)
    check_tensor(C_f, "C_f", torch.uint8, (H, W), dev)
    p = make_params(params)
    L = _lib.load()
    n_cells = L.sm_cells(W, H, sz_occ)
    C_it = torch.empty((H, W), dtype=torch.uint8, device=dev) if want_C_it else None
    cell_g = torch.empty(n_cells, dtype=torch.int64, device=dev)
    cell_b = torch.empty(n_cells, dtype=torch.int64, device=dev)
    check(L.sm_validate(cL.data_ptr(), cR.data_ptr(), omega.data_ptr(), D_it.data_ptr(), W, H, p,
                        sz_occ, _ptr(C_it), D_f.data_ptr(), C_f.data_ptr(), cell_g.data_ptr(),
                        cell_b.data_ptr(), _stream(stream)))
    return C_it, cell_g, cell_b


def resample(cL, cR, D_it, cell_g, cell_b, params: dict, sz_occ: int, S_dev, n_S: int,
             stream=None):
    """New supports of Alg. 4: (device buffer, device int32 count)."""
    check_census_pair(cL, cR)
    H, W = cL.shape
    dev = cL.device
    p = make_params(params)
    L = _lib.load()
    n_cells = L.sm_cells(W, H, sz_occ)
    n_S = int(n_S)
    check_tensor(D_it, "D_it", torch.float32, (H, W), dev)
    check_tensor(cell_g, "cell_g", torch.int64, None, dev, min_numel=n_cells)
    check_tensor(cell_b, "cell_b", torch.int64, None, dev, min_numel=n_cells)
    check_tensor(S_dev, "S_dev", torch.uint8, None, dev, min_numel=8 * max(n_S, 0))
    cap = 2 * n_cells
    out = new_support_buffer(cap, dev)
    occ = torch.empty((H, W), dtype=torch.uint8, device=dev)
    n_out = torch.zeros(1, dtype=torch.int32, device=dev)
    check(L.sm_resample(cL.data_ptr(), cR.data_ptr(), D_it.data_ptr(), cell_g.data_ptr(),
                        cell_b.data_ptr(), W, H, sz_occ, p, S_dev.data_ptr(), n_S, occ.data_ptr(),
                        out.data_ptr(), max(cap, 1), n_out.data_ptr(), _stream(stream)))
    return out, n_out


@dataclass
class SolveResult:
    D_f: torch.Tensor
    C_f: torch.Tensor
    mask: torch.Tensor
    stats: Optional[dict]


_STAGE_ITEMS = tuple(_lib.STAGES.items())


def stats_dict(st: "_lib.SmStats", n_iters: int) -> dict:
    us = st.stage_us[:]  # one conversion of each ctypes array
    launches = st.stage_launches[:]
    return {
        "n_support": st.n_support[:n_iters],
        "n_tris": st.n_tris[:n_iters],
        "n_valid": int(st.n_valid),
        "stage_us": {k: us[i] for k, i in _STAGE_ITEMS},
        "stage_launches": {k: launches[i] for k, i in _STAGE_ITEMS},
        "mesh_device": int(st.mesh_device),
        "mesh_fallback": int(st.mesh_fallback),
    }


class Solver:
    """Alg. 1 on frames of one size with a workspace allocated once."""

    def __init__(self, W: int, H: int, params: dict, device="cuda"):
        self.W, self.H = W, H
        self.params = dict(params)
        self.p = make_params(params)
        L = _lib.load()
        nbytes = L.sm_solve_workspace_bytes(W, H, self.p)
        if nbytes == 0:
            raise ValueError("invalid image size or parameters")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.ws_bytes = nbytes
        self.D_f = torch.empty((H, W), dtype=torch.float32, device=device)
        self.C_f = torch.empty((H, W), dtype=torch.uint8, device=device)
        self.mask = torch.empty((H, W), dtype=torch.uint8, device=device)
        self._out = (self.D_f.data_ptr(), self.C_f.data_ptr(), self.mask.data_ptr())
        self._dev = self.D_f.device.index
        self._shape = torch.Size((H, W))
        self.st = _lib.SmStats()

    def __call__(self, left: torch.Tensor, right: torch.Tensor, stats=False, timing=False,
                 stream=None) -> SolveResult:
        check_image(left, "left", self._shape, self.D_f.device)
        check_image(right, "right", self._shape, self.D_f.device)
        pitch = left.stride(0)
        L = _lib.load()
        st = None
        if stats or timing:
            self.st.timing = _lib.timing_flag(timing)
            st = self.st
        check(L.sm_solve(left.data_ptr(), right.data_ptr(), self.W, self.H, pitch, self.p,
                         self.ws_ptr, self.ws_bytes, *self._out, st, _stream(stream, self._dev)))
        return SolveResult(self.D_f, self.C_f, self.mask,
                           stats_dict(st, self.p.n_iters) if st is not None else None)

    def autotune(self, left: torch.Tensor, right: torch.Tensor, stream=None) -> dict:
        """Measures the tunable launch shapes on this frame (``sm_autotune``) and records the
        fastest for this size; later solves of the size use them (outputs do not change).
        Returns the choices; D_f, C_f and mask hold the frame's results."""
        check_image(left, "left", self._shape, self.D_f.device)
        check_image(right, "right", self._shape, self.D_f.device)
        L = _lib.load()
        ch = (ctypes.c_int32 * 11)()
        check(L.sm_autotune(left.data_ptr(), right.data_ptr(), self.W, self.H, left.stride(0), self.p,
                            self.ws_ptr, self.ws_bytes, self.D_f.data_ptr(), self.C_f.data_ptr(),
                            self.mask.data_ptr(), ch, _stream(stream)))
        n = self.p.n_iters
        return {"validate_waves": [int(ch[k]) for k in range(min(n, 8))], "raster_blocks": int(ch[8]),
                "match_lanes": int(ch[9]), "census_rows": int(ch[10])}


LAUNCH_SHAPES = {"validate_waves": 0, "raster_blocks": 1, "match_lanes": 2, "census_rows": 3}


def set_launch_shape(kind: str, W: int, H: int, key: int, value: int) -> None:
    """Records (value > 0) or clears (value = 0) a launch-shape choice for W x H frames
    (``sm_set_launch_shape``); kinds and keys as in LAUNCH_SHAPES and the C header."""
    check(_lib.load().sm_set_launch_shape(LAUNCH_SHAPES[kind], int(W), int(H), int(key), int(value)))


def solve(left: torch.Tensor, right: torch.Tensor, params: dict, stats=False) -> SolveResult:
    H, W = left.shape
    s = Solver(W, H, params, device=left.device)
    r = s(left, right, stats=stats)
    return SolveResult(r.D_f.clone(), r.C_f.clone(), r.mask.clone(), r.stats)


class BatchSolver:
    """Many frames (sizes and parameters may differ) solved concurrently by
    ``sm_solve_batch``: ``n_workers`` host workers, each with its own HIP stream and a
    workspace sized for the largest frame it may get."""

    def __init__(self, n_workers: int, max_W: int, max_H: int, params_list, device="cuda"):
        L = _lib.load()
        need = 0
        for prm in params_list:
            need = max(need, L.sm_solve_workspace_bytes(max_W, max_H, make_params(prm)))
        if need == 0:
            raise ValueError("invalid size or parameters")
        self.n_workers = n_workers
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_workers)]
        self.ws = [torch.empty(need + 256, dtype=torch.uint8, device=device) for _ in range(n_workers)]
        ptrs = [t.data_ptr() + ((-t.data_ptr()) % 256) for t in self.ws]
        self._streams = (ctypes.c_void_p * n_workers)(*[s.cuda_stream for s in self.streams])
        self._ws = (ctypes.c_void_p * n_workers)(*ptrs)
        self._ws_bytes = (ctypes.c_size_t * n_workers)(*([need] * n_workers))
        self.ws_bytes = need

    def __call__(self, frames, outputs=None, stats=False, timing=False):
        """frames: list of (left, right, params) with uint8 [H, W] CUDA tensors. Returns a
        list of (D_f, C_f, mask) and, with ``stats``, the summed statistics and the
        per-frame (worker, latency_us)."""
        n = len(frames)
        arr = (_lib.SmFrame * max(n, 1))()
        outs = outputs
        if outs is None:
            outs = []
            for (l, r, prm) in frames:
                H, W = l.shape
                outs.append((torch.empty((H, W), dtype=torch.float32, device=l.device),
                             torch.empty((H, W), dtype=torch.uint8, device=l.device),
                             torch.empty((H, W), dtype=torch.uint8, device=l.device)))
        check_frames(frames, outs)
        for i, ((l, r, prm), (D, C, M)) in enumerate(zip(frames, outs)):
            H, W = l.shape
            f = arr[i]
            f.L, f.R, f.W, f.H, f.stride = l.data_ptr(), r.data_ptr(), W, H, l.stride(0)
            f.p = make_params(prm)
            f.D_f, f.C_f, f.mask = D.data_ptr(), C.data_ptr(), M.data_ptr()
        # inputs were produced on the current stream; the workers' streams wait for it
        cur = torch.cuda.current_stream(self.device)
        for s in self.streams:
            s.wait_stream(cur)
        st = _lib.SmStats()
        st.timing = _lib.timing_flag(timing)
        L = _lib.load()
        check(L.sm_solve_batch(arr, n, self._streams, self._ws, self._ws_bytes, self.n_workers,
                               st if (stats or timing) else None))
        for s in self.streams:
            cur.wait_stream(s)
        if not (stats or timing):
            return outs
        per = [(int(arr[i].worker), float(arr[i].latency_us)) for i in range(n)]
        return outs, stats_dict(st, 8), per


class ManySolver:
    """Many frames (sizes and parameters may differ) solved stage by stage by
    ``sm_solve_many``: one launch per stage over all frames, host triangulations on
    ``n_threads`` workers. The workspace grows to the largest batch seen."""

    def __init__(self, n_threads: int = 16, device="cuda"):
        self.n_threads = n_threads
        self.device = device
        self.ws = None
        self.ws_bytes = 0

    def _frames(self, frames, outs):
        n = len(frames)
        arr = (_lib.SmFrame * max(n, 1))()
        check_frames(frames, outs)
        for i, ((l, r, prm), (D, C, M)) in enumerate(zip(frames, outs)):
            H, W = l.shape
            f = arr[i]
            f.L, f.R, f.W, f.H, f.stride = l.data_ptr(), r.data_ptr(), W, H, l.stride(0)
            f.p = make_params(prm)
            f.D_f, f.C_f, f.mask = D.data_ptr(), C.data_ptr(), M.data_ptr()
        return arr

    def __call__(self, frames, outputs=None, stats=False, timing=False, stream=None):
        """frames: list of (left, right, params) with uint8 [H, W] CUDA tensors. Returns a
        list of (D_f, C_f, mask) and, with ``stats``, the summed statistics."""
        n = len(frames)
        outs = outputs
        if outs is None:
            outs = [(torch.empty(l.shape, dtype=torch.float32, device=l.device),
                     torch.empty(l.shape, dtype=torch.uint8, device=l.device),
                     torch.empty(l.shape, dtype=torch.uint8, device=l.device)) for (l, _, _) in frames]
        arr = self._frames(frames, outs)
        L = _lib.load()
        need = L.sm_solve_many_workspace_bytes(arr, n) if n else 0
        if n and need == 0:
            raise ValueError("invalid frame sizes or parameters: " + L.sm_last_error().decode(errors="replace"))
        if need > self.ws_bytes:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            self.ws_bytes = need
        ptr = self.ws.data_ptr() + ((-self.ws.data_ptr()) % 256) if self.ws is not None else None
        st = _lib.SmStats()
        st.timing = _lib.timing_flag(timing)
        check(L.sm_solve_many(arr, n, ptr, self.ws_bytes, self.n_threads,
                              st if (stats or timing) else None, _stream(stream)))
        if not (stats or timing):
            return outs
        return outs, stats_dict(st, 8)

    def capture(self, frames, outputs=None, stream=None):
        """Solves ``frames`` like ``__call__`` while recording the batch's device work into
        a HIP graph (``sm_solve_many_capture``); returns ``(outputs, ManyGraph)``. The graph
        replays the batch over the same tensors (new image contents may be copied into
        them); every frame must keep its meshes on the device (``host_mesh = 0``). This
        solver's workspace is then fixed to the graph."""
        n = len(frames)
        outs = outputs
        if outs is None:
            outs = [(torch.empty(l.shape, dtype=torch.float32, device=l.device),
                     torch.empty(l.shape, dtype=torch.uint8, device=l.device),
                     torch.empty(l.shape, dtype=torch.uint8, device=l.device)) for (l, _, _) in frames]
        arr = self._frames(frames, outs)
        L = _lib.load()
        need = L.sm_solve_many_workspace_bytes(arr, n) if n else 0
        if n and need == 0:
            raise ValueError("invalid frame sizes or parameters: " + L.sm_last_error().decode(errors="replace"))
        ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)  # owned by the graph
        ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
        handle = ctypes.c_void_p()
        # a capture needs a stream of its own (not the legacy default stream), ordered after
        # the caller's work and before what the caller does next
        cur = torch.cuda.current_stream(self.device) if stream is None else stream
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(cur)
        check(L.sm_solve_many_capture(arr, n, ptr, need, None, _stream(side), ctypes.byref(handle)))
        cur.wait_stream(side)
        return outs, ManyGraph(handle, ws, frames, outs)


class ManyGraph:
    """A captured stage-batched solve (``sm_solve_many_capture``). ``run()`` replays it over
    the tensors it was captured with and returns the summed statistics."""

    def __init__(self, handle, ws, frames, outs):
        self._h = handle
        self._keep = (ws, frames, outs)  # the graph reads and writes these buffers

    def run(self, stats=False, stream=None):
        if self._h is None:
            raise RuntimeError("graph destroyed")
        L = _lib.load()
        st = _lib.SmStats()
        check(L.sm_many_graph_run(self._h, st if stats else None, _stream(stream)))
        return stats_dict(st, 8) if stats else None

    def close(self):
        if self._h is not None:
            _lib.load().sm_many_graph_destroy(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
