"""CPU oracle of the coarse-to-fine visual-hull path (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path never imports it.  It wraps ``fvv_oracle.c`` (plain
C written from the paper's definitions) through ctypes with numpy arrays, and
shares no code with the HIP library.

Functions (paper sections in ``fvv_oracle.c``):
  pack, carve, label, label_bfs, roi_fine, edges, bisect, mesh, point_inside,
  floor_div, and ``frame`` which chains them in the paper's order
  (Sec. II-B-1 sparse hull, II-B-2 labelling + Eq. (1) filter + boxes,
  II-B-3 dense hull per ROI, II-C crossing edges + exit points).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fvv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        i32, i64, f32 = C.c_int32, C.c_int64, C.c_float
        L.orc_floor_div.argtypes = [f32, f32]
        L.orc_floor_div.restype = i64
        L.orc_pack.argtypes = [C.c_int, C.c_int, C.c_int, p, p]
        L.orc_carve.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, f32, p, p, p]
        L.orc_carve.restype = i64
        L.orc_label.argtypes = [p, p, p, C.c_uint32, C.c_uint32, p, i32]
        L.orc_label.restype = i32
        L.orc_label_bfs.argtypes = [p, p, p]
        L.orc_label_bfs.restype = i32
        L.orc_roi_fine.argtypes = [p, p, i64, i64, p, p, p, p]
        L.orc_edges.argtypes = [p, p, p, i64]
        L.orc_edges.restype = i64
        L.orc_mesh.argtypes = [p, p, p, i64, p, i64]
        L.orc_mesh.restype = i64
        L.orc_bisect.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, f32, p, p, p, p, i64,
                                 C.c_int, p, p]
        L.orc_bisect.restype = i64
        L.orc_isovalue.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, f32, p, p, p, p, i64, p,
                                   p]
        L.orc_line_lambda2.argtypes = [p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_line_lambda2.restype = C.c_double
        L.orc_depth.argtypes = [C.c_int, p, C.c_int, C.c_int, p, i64, p, i64, p]
        L.orc_visibility.argtypes = [C.c_int, p, C.c_int, C.c_int, p, i64, p, i64, p, f32, p]
        L.orc_edge_point.argtypes = [p, f32, p, p, p, C.c_uint32, f32, p]
        L.orc_point_inside.argtypes = [C.c_int, p, C.c_int, C.c_int, p, f32, f32, f32]
        L.orc_point_inside.restype = i32
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _i3(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32).reshape(3))


def _f3(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(3))


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> int:
    """Sets the OpenMP threads of later oracle calls; returns the previous count."""
    return int(lib().orc_set_threads(int(n)))


def floor_div(a: float, w: float) -> int:
    return int(lib().orc_floor_div(np.float32(a), np.float32(w)))


def pack(masks: np.ndarray) -> np.ndarray:
    """uint8 [N][H][W] -> uint32 [N][H][ceil(W/32)], bit x&31 of word x>>5."""
    masks = np.ascontiguousarray(masks, dtype=np.uint8)
    N, H, W = masks.shape
    out = np.empty((N, H, (W + 31) // 32), np.uint32)
    lib().orc_pack(N, W, H, _p(masks), _p(out))
    return out


@dataclass
class Lattice:
    origin: np.ndarray            # float32 (3,)
    h: np.float32
    lo: Tuple[int, int, int]      # global index of sample (0,0,0)
    dims: Tuple[int, int, int]

    @property
    def size(self) -> int:
        return int(np.prod(self.dims, dtype=np.int64))


def carve(P: np.ndarray, sils: np.ndarray, W: int, H: int, lat: Lattice) -> Tuple[np.ndarray, int]:
    """Occupancy uint8 [nz][ny][nx] and the number of (voxel, camera) tests."""
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    sils = np.ascontiguousarray(sils, dtype=np.uint32)
    nx, ny, nz = lat.dims
    occ = np.empty((nz, ny, nx), np.uint8)
    T = lib().orc_carve(P.shape[0], _p(P), W, H, _p(sils), _p(_f3(lat.origin)),
                        np.float32(lat.h), _p(_i3(lat.lo)), _p(_i3(lat.dims)), _p(occ))
    return occ, int(T)


def label(occ: np.ndarray, t_np: int = 8, t_nb: int = 0xFFFFFFFF, max_rois: int = 1 << 20
          ) -> Tuple[np.ndarray, np.ndarray, np.ndarray, int]:
    """(filtered occ, labels int32, rois int32 [K][8] = lo3 hi3 count min_index, K)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8).copy()
    nz, ny, nx = occ.shape
    labels = np.empty(occ.shape, np.int32)
    cap = int(min(max_rois, max(occ.size, 1)))
    rois = np.zeros((cap, 8), np.int32)
    K = lib().orc_label(_p(_i3((nx, ny, nz))), _p(occ), _p(labels), t_np, t_nb, _p(rois), cap)
    return occ, labels, rois[:min(K, cap)].copy(), int(K)


def label_bfs(occ: np.ndarray) -> Tuple[np.ndarray, int]:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    nz, ny, nx = occ.shape
    comp = np.empty(occ.shape, np.int32)
    n = lib().orc_label_bfs(_p(_i3((nx, ny, nz))), _p(occ), _p(comp))
    return comp, int(n)


def roi_fine(coarse: Lattice, hc_um: int, hf_um: int, h_fine: np.float32,
             box_lo, box_hi) -> Lattice:
    flo = np.zeros(3, np.int32)
    fn = np.zeros(3, np.int32)
    lib().orc_roi_fine(_p(_i3(coarse.lo)), _p(_i3(coarse.dims)), int(hc_um), int(hf_um),
                       _p(_i3(box_lo)), _p(_i3(box_hi)), _p(flo), _p(fn))
    return Lattice(origin=np.asarray(coarse.origin, np.float32), h=np.float32(h_fine),
                   lo=tuple(int(v) for v in flo), dims=tuple(int(v) for v in fn))


def edges(occ: np.ndarray) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    nz, ny, nx = occ.shape
    dims = _i3((nx, ny, nz))
    E = lib().orc_edges(_p(dims), _p(occ), None, 0)
    keys = np.empty(max(E, 1), np.uint32)
    lib().orc_edges(_p(dims), _p(occ), _p(keys), E)
    return keys[:E].copy()


def mesh(occ: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """Triangles [T][3] (indices into keys) of the isosurface over the cells
    of the lattice occ [nz][ny][nx]; keys: its crossing edges (edges())."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    nz, ny, nx = occ.shape
    dims = _i3((nx, ny, nz))
    T = lib().orc_mesh(_p(dims), _p(occ), _p(keys), keys.size, None, 0)
    if T < 0:
        raise ValueError("a crossing edge is missing from keys")
    tris = np.empty((max(T, 1), 3), np.uint32)
    lib().orc_mesh(_p(dims), _p(occ), _p(keys), keys.size, _p(tris), T)
    return tris[:T].copy()


def bisect(P, sils, W, H, lat: Lattice, occ: np.ndarray, keys: np.ndarray, steps: int = 8,
           count_tests: bool = False):
    """Exit points (xyz, t*) of the crossing edges; with count_tests also the
    number of (point, camera) tests of the index-order early exit."""
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    sils = np.ascontiguousarray(sils, dtype=np.uint32)
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    E = keys.size
    xyz = np.empty((max(E, 1), 3), np.float32)
    t = np.empty(max(E, 1), np.float32)
    T = lib().orc_bisect(P.shape[0], _p(P), W, H, _p(sils), _p(_f3(lat.origin)),
                         np.float32(lat.h), _p(_i3(lat.lo)), _p(_i3(lat.dims)), _p(occ), _p(keys),
                         E, steps, _p(xyz), _p(t))
    if count_tests:
        return xyz[:E].copy(), t[:E].copy(), int(T)
    return xyz[:E].copy(), t[:E].copy()


def isovalue(P, sils, W, H, lat: Lattice, occ: np.ndarray, keys: np.ndarray):
    """The paper's isovalue of every crossing edge (Sec. II-C, Eq. (2)-(3)):
    lambda (float32, the minimum over cameras of the Bresenham image-space
    ratio) and the point at that parameter along the edge from its occupied
    end."""
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    sils = np.ascontiguousarray(sils, dtype=np.uint32)
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    E = keys.size
    lam = np.empty(max(E, 1), np.float32)
    xyz = np.empty((max(E, 1), 3), np.float32)
    lib().orc_isovalue(P.shape[0], _p(P), W, H, _p(sils), _p(_f3(lat.origin)), np.float32(lat.h),
                       _p(_i3(lat.lo)), _p(_i3(lat.dims)), _p(occ), _p(keys), E, _p(lam), _p(xyz))
    return lam[:E].copy(), xyz[:E].copy()


def line_lambda2(sil: np.ndarray, W: int, H: int, p_on, p_off) -> float:
    """lambda_i^2 of Eq. (2) for one camera: the Bresenham line of pixels from
    p_on to p_off over one packed silhouette [H][ceil(W/32)]."""
    sil = np.ascontiguousarray(sil, dtype=np.uint32)
    return float(lib().orc_line_lambda2(_p(sil), W, H, int(p_on[0]), int(p_on[1]), int(p_off[0]),
                                        int(p_off[1])))


def depth(P, W: int, H: int, xyz: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Depth images float32 [N][H][W] of a triangle mesh (Sec. II-D-1, Eq. (4)):
    per pixel the minimum camera-plane distance of the triangles covering it,
    +inf where none does."""
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    tris = np.ascontiguousarray(tris, dtype=np.uint32).reshape(-1, 3)
    out = np.empty((P.shape[0], H, W), np.float32)
    lib().orc_depth(P.shape[0], _p(P), W, H, _p(xyz), xyz.shape[0], _p(tris), tris.shape[0],
                    _p(out))
    return out


def visibility(P, W: int, H: int, xyz: np.ndarray, tris: np.ndarray, depth_images: np.ndarray,
               t_v: float) -> np.ndarray:
    """uint32 [T]: bit c set when triangle m is visible in camera c (Sec.
    II-D-2: in view, and not farther than the depth image by more than t_v)."""
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    tris = np.ascontiguousarray(tris, dtype=np.uint32).reshape(-1, 3)
    D = np.ascontiguousarray(depth_images, dtype=np.float32)
    vis = np.empty(max(tris.shape[0], 1), np.uint32)
    lib().orc_visibility(P.shape[0], _p(P), W, H, _p(xyz), xyz.shape[0], _p(tris), tris.shape[0],
                         _p(D), np.float32(t_v), _p(vis))
    return vis[:tris.shape[0]].copy()


def edge_point(lat: Lattice, occ: np.ndarray, key: int, t: float) -> np.ndarray:
    """The world point (float32 xyz) at parameter t of crossing edge `key` of
    the lattice, from its occupied end (t = 0) toward the other, formed as the
    bisection forms its test points."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    out = np.empty(3, np.float32)
    lib().orc_edge_point(_p(_f3(lat.origin)), np.float32(lat.h), _p(_i3(lat.lo)),
                         _p(_i3(lat.dims)), _p(occ), int(key), np.float32(t), _p(out))
    return out


def point_inside(P, sils, W, H, X: float, Y: float, Z: float) -> bool:
    P = np.ascontiguousarray(P, dtype=np.float32).reshape(-1, 12)
    sils = np.ascontiguousarray(sils, dtype=np.uint32)
    return bool(lib().orc_point_inside(P.shape[0], _p(P), W, H, _p(sils), np.float32(X),
                                       np.float32(Y), np.float32(Z)))


@dataclass
class FrameResult:
    sils: np.ndarray
    coarse: Lattice
    occ_coarse: np.ndarray          # as carved
    occ_filtered: np.ndarray        # after the Eq. (1) filter
    labels: np.ndarray
    rois: np.ndarray                # [K][8]
    fine: List[Lattice] = field(default_factory=list)
    occ_fine: List[np.ndarray] = field(default_factory=list)
    keys: List[np.ndarray] = field(default_factory=list)
    xyz: List[np.ndarray] = field(default_factory=list)
    tstar: List[np.ndarray] = field(default_factory=list)
    tests_coarse: int = 0
    tests_fine: int = 0
    tests_surface: int = 0          # (point, camera) tests of the bisection

    @property
    def fine_voxels(self) -> int:
        return int(sum(l.size for l in self.fine))


def frame(masks: np.ndarray, P: np.ndarray, origin, hc_um: int, hf_um: int,
          coarse_dims, t_np: int = 8, t_nb: int = 0xFFFFFFFF, steps: int = 8,
          surface: bool = True, max_rois: int = 1 << 20) -> FrameResult:
    """The whole path on one frame, step by step in the paper's order."""
    N, H, W = masks.shape
    sils = pack(masks)
    hc = np.float32(float(hc_um) * 1e-6)
    hf = np.float32(float(hf_um) * 1e-6)
    coarse = Lattice(origin=np.asarray(origin, np.float32), h=hc, lo=(0, 0, 0),
                     dims=tuple(int(v) for v in coarse_dims))
    occ, Tc = carve(P, sils, W, H, coarse)
    occ_f, labels, rois, K = label(occ, t_np, t_nb, max_rois)
    res = FrameResult(sils=sils, coarse=coarse, occ_coarse=occ, occ_filtered=occ_f,
                      labels=labels, rois=rois, tests_coarse=Tc)
    for r in rois:
        lat = roi_fine(coarse, hc_um, hf_um, hf, r[0:3], r[3:6])
        of, Tf = carve(P, sils, W, H, lat)
        res.fine.append(lat)
        res.occ_fine.append(of)
        res.tests_fine += Tf
        if surface:
            keys = edges(of)
            xyz, t, Ts = bisect(P, sils, W, H, lat, of, keys, steps, count_tests=True)
            res.tests_surface += Ts
            res.keys.append(keys)
            res.xyz.append(xyz)
            res.tstar.append(t)
    return res
