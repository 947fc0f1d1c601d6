"""Python binding of the gfx950 coarse-to-fine visual-hull library (libfvv.so).

Argument marshalling only: every step runs in the HIP kernels behind the C ABI
declared in ``include/fvv.h``.  torch supplies device memory and streams.  The
binding has no CPU path: importing it without the built library, or calling it
without a GPU, raises.

Names follow the C ABI: ``pack_silhouettes``, ``carve``, ``label``,
``roi_grids``, ``surface``, ``carve_batched`` (+ ``carve_batched_graph``,
``tune_carve_batched``), ``frame``, ``frame_graph``, ``mesh``,
``soft_forward`` and ``soft_backward``, as methods of :class:`Context` (which owns the library's
device scratch).  The tile autotuner of the batched carve is
:mod:`paper_1903_11785_amd.autotune`; the soft hull's autograd functions are in
:mod:`paper_1903_11785_amd.soft`.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvv.so")
MAX_CAMS = 32
MAX_STEPS = 12
FRAME_STAGE_EVENTS = 7
FRAME_EVENTS = 11
STAGES = ("pack", "coarse_carve", "label", "fine_carve", "edges", "exit_points")
# events FRAME_STAGE_EVENTS + 2 i, + 2 i + 1: start and end of kernel i itself
FRAME_KERNELS = ("fine_carve", "exit_points")

FVV_OK, FVV_EINVAL, FVV_ECAPACITY, FVV_EDEVICE, FVV_ENOMEM = 0, -1, -2, -3, -4
EXIT_BISECTION, EXIT_BRESENHAM = 0, 1


class FvvError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


# ------------------------------------------------------------------ C structs (layout of fvv.h)
class Camera(C.Structure):
    _fields_ = [("P", C.c_float * 12), ("width", C.c_int32), ("height", C.c_int32)]


class GridC(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("h", C.c_float), ("lo", C.c_int32 * 3),
                ("dims", C.c_int32 * 3)]


class Roi(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("count", C.c_uint32),
                ("min_index", C.c_uint32)]


class Job(C.Structure):
    _fields_ = [("grid", GridC), ("cam_base", C.c_int32), ("n_cams", C.c_int32),
                ("width", C.c_int32), ("height", C.c_int32), ("sil_base", C.c_int64),
                ("out_offset", C.c_int64)]


class SoftCamera(C.Structure):
    _fields_ = [("K", C.c_float * 4), ("R0", C.c_float * 9), ("t0", C.c_float * 3),
                ("omega", C.c_float * 3), ("tau", C.c_float * 3)]


class Limits(C.Structure):
    _fields_ = [("max_cams", C.c_int32), ("max_w", C.c_int32), ("max_h", C.c_int32),
                ("max_coarse", C.c_int64), ("max_fine", C.c_int64), ("max_rois", C.c_uint32),
                ("max_points", C.c_uint32), ("max_jobs", C.c_uint32)]


class Tile(C.Structure):
    _fields_ = [("tx", C.c_int32), ("ty", C.c_int32), ("tz", C.c_int32),
                ("persistent_blocks", C.c_int32)]


class FrameParams(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("cams", Camera * MAX_CAMS), ("coarse", GridC),
                ("hc_um", C.c_int64), ("hf_um", C.c_int64), ("t_np", C.c_uint32),
                ("t_nb", C.c_uint32), ("n_steps", C.c_int32), ("coarse_tile", Tile),
                ("fine_tile", Tile), ("exit_estimator", C.c_int32)]


class FrameOut(C.Structure):
    _fields_ = [("d_occ_coarse", C.c_void_p), ("d_labels", C.c_void_p), ("d_rois", C.c_void_p),
                ("d_jobs", C.c_void_p), ("d_occ_fine", C.c_void_p), ("d_keys", C.c_void_p),
                ("d_xyz", C.c_void_p), ("d_point_off", C.c_void_p), ("d_counts", C.c_void_p),
                ("max_rois", C.c_uint32), ("max_fine", C.c_int64), ("max_points", C.c_uint32),
                ("d_tris", C.c_void_p), ("d_tri_off", C.c_void_p), ("max_tris", C.c_uint32)]


ROI_DTYPE = np.dtype([("lo", "<i4", 3), ("hi", "<i4", 3), ("count", "<u4"), ("min_index", "<u4")])
JOB_DTYPE = np.dtype({"names": ["origin", "h", "lo", "dims", "cam_base", "n_cams", "width",
                                "height", "sil_base", "out_offset"],
                      "formats": [("<f4", 3), "<f4", ("<i4", 3), ("<i4", 3), "<i4", "<i4", "<i4",
                                  "<i4", "<i8", "<i8"],
                      "offsets": [0, 12, 16, 28, 40, 44, 48, 52, 56, 64], "itemsize": 72})
CAMERA_DTYPE = np.dtype({"names": ["P", "width", "height"], "formats": [("<f4", 12), "<i4", "<i4"],
                         "offsets": [0, 48, 52], "itemsize": 56})
assert C.sizeof(Job) == JOB_DTYPE.itemsize and C.sizeof(Roi) == ROI_DTYPE.itemsize
assert C.sizeof(Camera) == CAMERA_DTYPE.itemsize


# ------------------------------------------------------------------ library
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads torch's HIP runtime first, which the library then shares)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1903_11785_amd.build.build()")
    L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
    P, i32, u32, i64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_int64
    sigs = {
        "fvv_create": ([C.POINTER(P), C.POINTER(Limits)], i32),
        "fvv_destroy": ([P], None),
        "fvv_status_str": ([i32], C.c_char_p),
        "fvv_check": ([P, P], i32),
        "fvv_pack_silhouettes": ([P, i32, i32, i32, P, P, P], i32),
        "fvv_carve": ([P, i32, C.POINTER(Camera), P, C.POINTER(GridC), C.POINTER(Tile), P, P], i32),
        "fvv_label": ([P, C.POINTER(GridC), P, P, u32, u32, P, u32, P, P], i32),
        "fvv_roi_grids": ([C.POINTER(GridC), i64, i64, C.POINTER(Roi), u32, C.POINTER(GridC)], i32),
        "fvv_surface": ([P, C.POINTER(GridC), P, i32, C.POINTER(Camera), P, i32, P, P, u32, P, P],
                        i32),
        "fvv_surface_noalloc": ([C.POINTER(GridC), P, i32, C.POINTER(Camera), P, i32, P, P, u32,
                                 P, P], i32),
        "fvv_carve_batched": ([P, P, u32, P, P, P, C.POINTER(Tile), P], i32),
        "fvv_frame": ([P, C.POINTER(FrameParams), P, P, C.POINTER(FrameOut), P, P], i32),
        "fvv_frame_graph_create": ([P, C.POINTER(FrameParams), P, P, C.POINTER(FrameOut),
                                    C.POINTER(P)], i32),
        "fvv_carve_batched_graph_create": ([P, P, u32, P, P, P, C.POINTER(Tile), C.POINTER(P)],
                                           i32),
        "fvv_tune_carve_batched": ([P, P, u32, P, P, P, C.POINTER(Tile), u32, i32,
                                    C.POINTER(C.c_float), C.POINTER(u32), P], i32),
        "fvv_mesh": ([P, C.POINTER(GridC), P, P, P, u32, P, u32, P, P], i32),
        "fvv_isovalue": ([P, C.POINTER(GridC), P, i32, C.POINTER(Camera), P, P, P, u32, P, P, P],
                         i32),
        "fvv_visibility": ([P, i32, C.POINTER(Camera), P, P, u32, P, P, u32, C.c_float, P, P, P],
                           i32),
        "fvv_gather_peak": ([P, P, u32, P, i32, C.POINTER(C.c_double), P], i32),
        "fvv_soft_forward": ([P, C.POINTER(GridC), i32, C.POINTER(SoftCamera), i32, i32, P, P, P, P,
                              P], i32),
        "fvv_soft_backward": ([P, C.POINTER(GridC), i32, C.POINTER(SoftCamera), i32, i32, P, P, P,
                               P, P, P, P], i32),
        "fvv_graph_launch": ([P, P], i32),
        "fvv_graph_destroy": ([P], None),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def library():
    """The loaded ctypes library (raises ImportError when not built)."""
    return _load()


def status_str(s: int) -> str:
    return _load().fvv_status_str(int(s)).decode()


def _ok(s: int, what: str):
    if s != FVV_OK:
        raise FvvError(int(s), what)


# ------------------------------------------------------------------ value types
@dataclass
class Grid:
    origin: Tuple[float, float, float]
    h: float
    lo: Tuple[int, int, int]
    dims: Tuple[int, int, int]

    def c(self) -> GridC:
        g = GridC()
        for a in range(3):
            g.origin[a] = float(np.float32(self.origin[a]))
            g.lo[a] = int(self.lo[a])
            g.dims[a] = int(self.dims[a])
        g.h = float(np.float32(self.h))
        return g

    @staticmethod
    def from_c(g: GridC) -> "Grid":
        return Grid(origin=tuple(np.float32(v) for v in g.origin), h=np.float32(g.h),
                    lo=tuple(int(v) for v in g.lo), dims=tuple(int(v) for v in g.dims))

    @property
    def size(self) -> int:
        return int(np.prod(self.dims, dtype=np.int64))

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (int(self.dims[2]), int(self.dims[1]), int(self.dims[0]))


def make_cameras(P: np.ndarray, W: int, H: int):
    P = np.asarray(P, np.float32).reshape(-1, 12)
    arr = (Camera * P.shape[0])()
    for c in range(P.shape[0]):
        for e in range(12):
            arr[c].P[e] = float(P[c, e])
        arr[c].width = int(W)
        arr[c].height = int(H)
    return arr


def tile(tx: int = 64, tz: int = 4, persistent_blocks: int = 0) -> Tile:
    return Tile(tx, 256 // tx, tz, persistent_blocks)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _event_handle(ev) -> int:
    """hipEvent_t of a torch.cuda.Event (created on first use)."""
    import torch
    if ev.cuda_event == 0:                  # torch creates events lazily
        ev.record(torch.cuda.current_stream())
        torch.cuda.current_stream().synchronize()
    return int(ev.cuda_event)


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def roi_grids(coarse: Grid, hc_um: int, hf_um: int, rois: np.ndarray) -> List[Grid]:
    """Host-side fine lattice of each ROI (rows of ROI_DTYPE or int32 [K][8])."""
    rois = np.ascontiguousarray(rois)
    if rois.dtype != ROI_DTYPE:
        rois = np.ascontiguousarray(rois.astype(np.int32).reshape(-1, 8)).view(ROI_DTYPE).reshape(-1)
    n = rois.shape[0]
    out = (GridC * max(n, 1))()
    src = rois.ctypes.data_as(C.POINTER(Roi)) if n else None
    _ok(_load().fvv_roi_grids(C.byref(coarse.c()), int(hc_um), int(hf_um), src, n, out),
        "fvv_roi_grids")
    return [Grid.from_c(out[t]) for t in range(n)]


# ------------------------------------------------------------------ context
NOALLOC_BITMAP_WORDS = 1 << 20


def surface_noalloc(roi: Grid, occ_fine, P: np.ndarray, W: int, H: int, sils, keys, xyz,
                    n_points, n_steps: int = 8, max_points: Optional[int] = None, stream=None):
    """fvv_surface_noalloc: Context.surface without a context, into the
    caller's keys (int32 [max_points]), xyz (float32 [max_points][3]) and
    n_points (int32 [1]); the library uses its static per-GPU scratch."""
    cams = make_cameras(P, W, H)
    if max_points is None:
        max_points = int(keys.numel())
    _ok(_load().fvv_surface_noalloc(C.byref(roi.c()), _ptr(occ_fine), len(cams), cams,
                                    _ptr(sils), int(n_steps), _ptr(keys), _ptr(xyz),
                                    int(max_points), _ptr(n_points), C.c_void_p(_stream(stream))),
        "fvv_surface_noalloc")
    return keys, xyz, n_points


class Context:
    """Owns the library's device scratch (all allocated up front)."""

    def __init__(self, max_cams: int = 32, max_w: int = 3840, max_h: int = 2160,
                 max_coarse: int = 1 << 23, max_fine: int = 1 << 28, max_rois: int = 4096,
                 max_points: int = 1 << 23, max_jobs: int = 4096):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1903_11785_amd needs a ROCm GPU; there is no CPU path")
        self.L = _load()
        self.limits = Limits(max_cams, max_w, max_h, max_coarse, max_fine, max_rois, max_points,
                             max_jobs)
        h = C.c_void_p()
        _ok(self.L.fvv_create(C.byref(h), C.byref(self.limits)), "fvv_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.fvv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, stream=None) -> int:
        """Synchronise and return the sticky device status (FVV_OK / FVV_ECAPACITY)."""
        return int(self.L.fvv_check(self.h, C.c_void_p(_stream(stream))))

    # -------------------------------------------------------------- calls
    def pack_silhouettes(self, masks, out=None, stream=None):
        import torch
        assert masks.is_cuda and masks.dtype == torch.uint8 and masks.is_contiguous()
        N, H, W = masks.shape
        wpr = (W + 31) // 32
        if out is None:
            out = torch.empty((N, H, wpr), dtype=torch.int32, device=masks.device)
        _ok(self.L.fvv_pack_silhouettes(self.h, N, W, H, _ptr(masks), _ptr(out),
                                        C.c_void_p(_stream(stream))), "fvv_pack_silhouettes")
        return out

    def carve(self, P: np.ndarray, W: int, H: int, sils, grid: Grid, tile_: Optional[Tile] = None,
              out=None, stream=None):
        import torch
        cams = make_cameras(P, W, H)
        if out is None:
            out = torch.empty(grid.shape, dtype=torch.uint8, device=sils.device)
        _ok(self.L.fvv_carve(self.h, len(cams), cams, _ptr(sils), C.byref(grid.c()),
                             C.byref(tile_) if tile_ is not None else None, _ptr(out),
                             C.c_void_p(_stream(stream))), "fvv_carve")
        return out

    def label(self, grid: Grid, occ, t_np: int = 8, t_nb: int = 0xFFFFFFFF, max_rois: int = 4096,
              labels=None, rois=None, n_rois=None, stream=None):
        """In place on occ; returns (labels int32, rois int32 [max_rois][8], n_rois int32 [1])."""
        import torch
        dev = occ.device
        if labels is None:
            labels = torch.empty(grid.shape, dtype=torch.int32, device=dev)
        if rois is None:
            rois = torch.zeros((max_rois, 8), dtype=torch.int32, device=dev)
        if n_rois is None:
            n_rois = torch.zeros(1, dtype=torch.int32, device=dev)
        _ok(self.L.fvv_label(self.h, C.byref(grid.c()), _ptr(occ), _ptr(labels), int(t_np),
                             int(t_nb), _ptr(rois), int(max_rois), _ptr(n_rois),
                             C.c_void_p(_stream(stream))), "fvv_label")
        return labels, rois, n_rois

    def surface(self, roi: Grid, occ_fine, P: np.ndarray, W: int, H: int, sils, n_steps: int = 8,
                max_points: int = 1 << 22, keys=None, xyz=None, n_points=None, stream=None):
        import torch
        dev = occ_fine.device
        cams = make_cameras(P, W, H)
        if keys is None:
            keys = torch.empty(max_points, dtype=torch.int32, device=dev)
        if xyz is None:
            xyz = torch.empty((max_points, 3), dtype=torch.float32, device=dev)
        if n_points is None:
            n_points = torch.zeros(1, dtype=torch.int32, device=dev)
        _ok(self.L.fvv_surface(self.h, C.byref(roi.c()), _ptr(occ_fine), len(cams), cams,
                               _ptr(sils), int(n_steps), _ptr(keys), _ptr(xyz), int(max_points),
                               _ptr(n_points), C.c_void_p(_stream(stream))), "fvv_surface")
        return keys, xyz, n_points

    def carve_batched(self, jobs_dev, n_jobs: int, cams_dev, sils, out, tile_: Optional[Tile] = None,
                      stream=None):
        _ok(self.L.fvv_carve_batched(self.h, _ptr(jobs_dev), int(n_jobs), _ptr(cams_dev),
                                     _ptr(sils), _ptr(out),
                                     C.byref(tile_) if tile_ is not None else None,
                                     C.c_void_p(_stream(stream))), "fvv_carve_batched")
        return out

    def carve_batched_graph(self, jobs_dev, n_jobs: int, cams_dev, sils, out,
                            tile_: Optional[Tile] = None) -> "FrameGraph":
        """fvv_carve_batched captured as a HIP graph (launch with .launch(stream))."""
        g = C.c_void_p()
        _ok(self.L.fvv_carve_batched_graph_create(self.h, _ptr(jobs_dev), int(n_jobs),
                                                  _ptr(cams_dev), _ptr(sils), _ptr(out),
                                                  C.byref(tile_) if tile_ is not None else None,
                                                  C.byref(g)), "fvv_carve_batched_graph_create")
        return FrameGraph(self.L, g)

    def tune_carve_batched(self, jobs_dev, n_jobs: int, cams_dev, sils, out,
                           cands: Sequence[Tile], reps: int = 3, stream=None):
        """Time each candidate tile of fvv_carve_batched on this job table;
        returns (index of the fastest, list of ms per call)."""
        arr = (Tile * len(cands))(*cands)
        ms = (C.c_float * len(cands))()
        best = C.c_uint32()
        _ok(self.L.fvv_tune_carve_batched(self.h, _ptr(jobs_dev), int(n_jobs), _ptr(cams_dev),
                                          _ptr(sils), _ptr(out), arr, len(cands), int(reps), ms,
                                          C.byref(best), C.c_void_p(_stream(stream))),
            "fvv_tune_carve_batched")
        return int(best.value), [float(v) for v in ms]

    def mesh(self, grid: Grid, occ, keys, n_keys, max_tris: int = 1 << 22, tris=None,
             n_tris=None, stream=None):
        """Marching-cubes triangles (uint32 [max_tris][3] indices into keys) of
        one lattice; returns (tris, n_tris) device tensors."""
        import torch
        if tris is None:
            tris = torch.empty((max_tris, 3), dtype=torch.int32, device=occ.device)
        if n_tris is None:
            n_tris = torch.zeros(1, dtype=torch.int32, device=occ.device)
        _ok(self.L.fvv_mesh(self.h, C.byref(grid.c()), _ptr(occ), _ptr(keys), _ptr(n_keys),
                            int(keys.numel()), _ptr(tris), int(tris.shape[0]), _ptr(n_tris),
                            C.c_void_p(_stream(stream))), "fvv_mesh")
        return tris, n_tris

    def isovalue(self, grid: Grid, occ, P: np.ndarray, W: int, H: int, sils, keys, n_keys,
                 lam=None, xyz=None, stream=None):
        """The paper's Bresenham isovalue (lambda, and the point there) of the
        first n_keys keys; returns (lam, xyz) device tensors."""
        import torch
        cams = make_cameras(P, W, H)
        m = int(keys.numel())
        if lam is None:
            lam = torch.empty(m, dtype=torch.float32, device=occ.device)
        if xyz is None:
            xyz = torch.empty((m, 3), dtype=torch.float32, device=occ.device)
        _ok(self.L.fvv_isovalue(self.h, C.byref(grid.c()), _ptr(occ), len(cams), cams, _ptr(sils),
                                _ptr(keys), _ptr(n_keys), m, _ptr(lam), _ptr(xyz),
                                C.c_void_p(_stream(stream))), "fvv_isovalue")
        return lam, xyz

    def visibility(self, P: np.ndarray, W: int, H: int, xyz, n_vertices, tris, n_tris,
                   t_v: float, depth=None, vis=None, stream=None):
        """Depth images float [N][H][W] and per-triangle visibility masks (bit c:
        visible in camera c) of the mesh (xyz vertices, tris indices; the
        counts are device int32 tensors of one element)."""
        import torch
        cams = make_cameras(P, W, H)
        if depth is None:
            depth = torch.empty((len(cams), H, W), dtype=torch.float32, device=xyz.device)
        if vis is None:
            vis = torch.empty(tris.shape[0], dtype=torch.int32, device=xyz.device)
        _ok(self.L.fvv_visibility(self.h, len(cams), cams, _ptr(xyz), _ptr(n_vertices),
                                  int(xyz.shape[0]), _ptr(tris), _ptr(n_tris), int(tris.shape[0]),
                                  float(t_v), _ptr(depth), _ptr(vis),
                                  C.c_void_p(_stream(stream))), "fvv_visibility")
        return depth, vis

    def gather_peak(self, table, reps: int = 20, stream=None) -> float:
        """Words per second the GPU serves from the device table (a measurement
        aid for the carve's gather roofline)."""
        import torch
        sink = torch.empty(16384 * 256, dtype=torch.int32, device=table.device)
        out = C.c_double()
        _ok(self.L.fvv_gather_peak(self.h, _ptr(table), int(table.numel()), _ptr(sink), int(reps),
                                   C.byref(out), C.c_void_p(_stream(stream))), "fvv_gather_peak")
        return out.value

    def soft_forward(self, grid: Grid, cams, W: int, H: int, logits, target=None, occ=None,
                     loss=None, stream=None):
        """Soft occupancy (and L2 loss with a target) of `grid`; cams: a
        SoftCamera ctypes array (see soft_cameras)."""
        _ok(self.L.fvv_soft_forward(self.h, C.byref(grid.c()), len(cams), cams, int(W), int(H),
                                    _ptr(logits), _ptr(target), _ptr(occ), _ptr(loss),
                                    C.c_void_p(_stream(stream))), "fvv_soft_forward")

    def soft_backward(self, grid: Grid, cams, W: int, H: int, logits, grad_logits, grad_pose,
                      target=None, grad_occ=None, scale=None, stream=None):
        _ok(self.L.fvv_soft_backward(self.h, C.byref(grid.c()), len(cams), cams, int(W), int(H),
                                     _ptr(logits), _ptr(target), _ptr(grad_occ), _ptr(scale),
                                     _ptr(grad_logits), _ptr(grad_pose),
                                     C.c_void_p(_stream(stream))), "fvv_soft_backward")

    def frame(self, params: FrameParams, sils, out: "FrameBuffers", masks=None, events=None,
              stream=None):
        """The whole path for one frame.  masks (uint8 [N][H][W], optional) are
        packed into sils first.  events: optional list of FRAME_EVENTS
        torch.cuda.Event(enable_timing=True): the first FRAME_STAGE_EVENTS are
        recorded between the stages, the others take the start and end times
        of the FRAME_KERNELS kernels themselves."""
        ev = None
        if events is not None:
            assert len(events) == FRAME_EVENTS
            ev = (C.c_void_p * FRAME_EVENTS)(*[_event_handle(e) for e in events])
        _ok(self.L.fvv_frame(self.h, C.byref(params), _ptr(masks), _ptr(sils), C.byref(out.c), ev,
                             C.c_void_p(_stream(stream))), "fvv_frame")

    def frame_graph(self, params: FrameParams, sils, out: "FrameBuffers", masks=None) -> "FrameGraph":
        g = C.c_void_p()
        _ok(self.L.fvv_frame_graph_create(self.h, C.byref(params), _ptr(masks), _ptr(sils),
                                          C.byref(out.c), C.byref(g)), "fvv_frame_graph_create")
        return FrameGraph(self.L, g)


class FrameGraph:
    def __init__(self, L, g):
        self.L, self.g = L, g

    def launch(self, stream=None):
        _ok(self.L.fvv_graph_launch(self.g, C.c_void_p(_stream(stream))), "fvv_graph_launch")

    def close(self):
        if self.g:
            self.L.fvv_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def frame_params(P: np.ndarray, W: int, H: int, coarse: Grid, hc_um: int, hf_um: int,
                 t_np: int = 8, t_nb: int = 0xFFFFFFFF, n_steps: int = 8,
                 coarse_tile: Optional[Tile] = None, fine_tile: Optional[Tile] = None,
                 exit_estimator: int = 0) -> FrameParams:
    """exit_estimator: EXIT_BISECTION (0) or EXIT_BRESENHAM (1, the paper's
    image-space isovalue)."""
    p = FrameParams()
    cams = make_cameras(P, W, H)
    p.n_cams = len(cams)
    for c in range(len(cams)):
        p.cams[c] = cams[c]
    p.coarse = coarse.c()
    p.hc_um, p.hf_um = int(hc_um), int(hf_um)
    p.t_np, p.t_nb, p.n_steps = int(t_np), int(t_nb), int(n_steps)
    p.coarse_tile = coarse_tile if coarse_tile is not None else tile(64, 1)
    p.fine_tile = fine_tile if fine_tile is not None else tile(64, 4)
    p.exit_estimator = int(exit_estimator)
    return p


class FrameBuffers:
    """Device outputs of one frame (caller-owned torch tensors)."""

    def __init__(self, coarse: Grid, max_rois: int = 256, max_fine: int = 1 << 26,
                 max_points: int = 1 << 22, device: str = "cuda", max_tris: int = 0):
        import torch
        z = lambda shape, dt: torch.zeros(shape, dtype=dt, device=device)
        self.occ_coarse = z(coarse.shape, torch.uint8)
        self.labels = z(coarse.shape, torch.int32)
        self.rois = z((max_rois, 8), torch.int32)
        self.jobs = z((max_rois, JOB_DTYPE.itemsize), torch.uint8)
        self.occ_fine = z(max_fine, torch.uint8)
        self.keys = z(max_points, torch.int32)
        self.xyz = z((max_points, 3), torch.float32)
        self.point_off = z(max_rois + 1, torch.int32)
        self.counts = z(4, torch.int32)
        # marching-cubes triangles of the ROIs (vertex indices into keys / xyz),
        # when max_tris > 0
        self.tris = z((max_tris, 3), torch.int32) if max_tris > 0 else None
        self.tri_off = z(max_rois + 1, torch.int32) if max_tris > 0 else None
        self.max_rois, self.max_fine, self.max_points = max_rois, max_fine, max_points
        self.max_tris = max_tris
        self.c = FrameOut(_ptr(self.occ_coarse), _ptr(self.labels), _ptr(self.rois),
                          _ptr(self.jobs), _ptr(self.occ_fine), _ptr(self.keys), _ptr(self.xyz),
                          _ptr(self.point_off), _ptr(self.counts), max_rois, max_fine, max_points,
                          _ptr(self.tris) if self.tris is not None else None,
                          _ptr(self.tri_off) if self.tri_off is not None else None, max_tris)

    def jobs_host(self, n: int) -> np.ndarray:
        return self.jobs[:n].cpu().numpy().reshape(-1).view(JOB_DTYPE)


def jobs_to_device(jobs: np.ndarray, device="cuda"):
    import torch
    jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
    return torch.from_numpy(jobs.view(np.uint8).reshape(-1, JOB_DTYPE.itemsize).copy()).to(device)


def cameras_to_device(P: np.ndarray, W: int, H: int, device="cuda"):
    import torch
    P = np.asarray(P, np.float32).reshape(-1, 12)
    arr = np.zeros(P.shape[0], CAMERA_DTYPE)
    arr["P"] = P
    arr["width"] = W
    arr["height"] = H
    return torch.from_numpy(arr.view(np.uint8).reshape(-1, CAMERA_DTYPE.itemsize).copy()).to(device)


def frame_major_jobs(boxes: Sequence[Tuple[int, Sequence[int], Sequence[int]]],
                     origins: Sequence[Sequence[float]], hs: Sequence[float], n_cams: int, W: int,
                     H: int) -> Tuple[np.ndarray, int]:
    """Job table of ROIs of several frames whose cameras and silhouettes are
    stored frame-major (frame f's cameras from row f*n_cams of the camera
    table, its silhouettes from word f*n_cams*H*ceil(W/32)), outputs back to
    back in table order.  boxes: (frame, lo, dims) per ROI, lo in global
    lattice indices of the frame's lattice (origins[f], hs[f]).  Returns the
    JOB_DTYPE table and the total output bytes."""
    wpr = (W + 31) // 32
    jobs = np.zeros(len(boxes), JOB_DTYPE)
    off = 0
    for t, (f, lo, dims) in enumerate(boxes):
        jobs[t]["origin"] = origins[f]
        jobs[t]["h"] = hs[f]
        jobs[t]["lo"] = lo
        jobs[t]["dims"] = dims
        jobs[t]["cam_base"] = f * n_cams
        jobs[t]["n_cams"] = n_cams
        jobs[t]["width"], jobs[t]["height"] = W, H
        jobs[t]["sil_base"] = f * n_cams * H * wpr
        jobs[t]["out_offset"] = off
        off += int(np.prod(np.asarray(dims, np.int64)))
    return jobs, off


def soft_cameras(K: np.ndarray, R0: np.ndarray, t0: np.ndarray, omega: np.ndarray,
                 tau: np.ndarray):
    """SoftCamera ctypes array from K [N][4] (fx, fy, cx, cy), R0 [N][3][3],
    t0 [N][3], omega [N][3], tau [N][3] (host arrays)."""
    K, R0, t0 = (np.asarray(a, np.float64) for a in (K, R0, t0))
    omega, tau = (np.asarray(a, np.float64) for a in (omega, tau))
    n = K.shape[0]
    arr = (SoftCamera * n)()
    for c in range(n):
        arr[c].K[:] = [float(v) for v in K[c]]
        arr[c].R0[:] = [float(v) for v in R0[c].reshape(-1)]
        arr[c].t0[:] = [float(v) for v in t0[c]]
        arr[c].omega[:] = [float(v) for v in omega[c]]
        arr[c].tau[:] = [float(v) for v in tau[c]]
    return arr
