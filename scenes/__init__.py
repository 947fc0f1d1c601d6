"""Seeded synthetic multi-camera scenes: cameras, ellipsoid unions, silhouettes.

This module produces INPUT DATA only.  It holds none of the reconstruction
method's arithmetic (no voxel projection, no labelling, no isosurface): it
places pinhole cameras, builds objects as unions of ellipsoids, and renders
each camera's binary silhouette analytically in FP64 (a pixel is foreground
iff the ray through its centre hits an ellipsoid in front of the camera).
Both the CPU oracle and the GPU path consume what it returns.

Workloads (the paper's volleyball/judo recordings are private, so seeded
synthetic scenes of the same shape stand in for them; the paper's own setups
are in its experiments section):

* ``tiny``       4 cameras 320x240 (f=300) on a 6 m ring, 2 random ellipsoids in
                 a 4x4x2 m volume, coarse 62.5 mm (64x64x32), fine 20 mm.
* ``volleyball`` 16 cameras 1920x1080 (f in [1800, 2400]) around an 18x9x4 m
                 court at 3-8 m height, 12 players of 5 ellipsoids each,
                 coarse 100 mm (180x90x40), fine 10 mm.
* ``judo``       24 cameras 3840x2160 (f in [3600, 4800]) around a 10x10x3 m mat,
                 2-4 players in touching pairs, 1 % boundary-pixel noise,
                 coarse 40 mm (250x250x75), fine 5 mm.
* ``batched``    the tiny rig, one new scene per frame, 12 uneven ROI boxes
                 (edges 0.6-2.5 m) per frame at 10 mm.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence([cfg, frame,
purpose])))`` with purpose 0 = cameras, 1 = objects, 2 = noise, 3 = ROI boxes.
The court rigs are static (drawn with frame 0 for every frame): the paper's
cameras do not move and are calibrated once.

Conventions (shared by specification with the consumers, not by code):
camera rows are R = [right; down; forward] with world z up, intrinsics
K = [[f, 0, W/2], [0, f, H/2], [0, 0, 1]], P = K [R | -R C] rounded once to
float32; pixel (x, y) covers [x, x+1) x [y, y+1).  Lattices are anchored at
the volume's minimum corner and voxel sizes are integer micrometres.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

CFG_TINY, CFG_VOLLEYBALL, CFG_JUDO, CFG_BATCHED = 1, 2, 3, 4
# the paper's own volleyball shape (its lattice sizes and rig), and the judo
# frame at a fine spacing that fills ~1e8 fine samples
CFG_PAPER_V, CFG_JUDO_FINE = 5, 6
UINT32_MAX = 0xFFFFFFFF


def rng_for(cfg: int, frame: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, frame, purpose])))


# --------------------------------------------------------------------------- cameras
@dataclass
class Camera:
    K: np.ndarray          # 3x3 float64
    R: np.ndarray          # 3x3 float64, rows right/down/forward
    C: np.ndarray          # (3,) float64 centre
    W: int
    H: int

    @property
    def P64(self) -> np.ndarray:
        return self.K @ np.hstack([self.R, (-self.R @ self.C)[:, None]])

    @property
    def P32(self) -> np.ndarray:
        return self.P64.astype(np.float32)


def look_at(C, target, f: float, W: int, H: int) -> Camera:
    C = np.asarray(C, np.float64)
    fwd = np.asarray(target, np.float64) - C
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    K = np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])
    return Camera(K=K, R=R, C=C, W=W, H=H)


def project64(cam: Camera, X: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """FP64 pinhole projection of world points X [..., 3] -> (x, y, depth)."""
    Xc = (X - cam.C) @ cam.R.T
    uvw = Xc @ cam.K.T
    return uvw[..., 0] / uvw[..., 2], uvw[..., 1] / uvw[..., 2], uvw[..., 2]


def _corners(lo, hi) -> np.ndarray:
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])


def _fits_inset(cam: Camera, pts: np.ndarray, inset: float) -> bool:
    x, y, d = project64(cam, pts)
    return bool(np.all(d > 0) and np.all(x >= inset * cam.W) and np.all(x <= (1 - inset) * cam.W)
                and np.all(y >= inset * cam.H) and np.all(y <= (1 - inset) * cam.H))


def ring_camera_min_distance(az: float, height: float, f: float, W: int, H: int,
                             vol_lo, vol_hi, target, inset: float = 0.02) -> Camera:
    """Smallest horizontal distance (FP64 bisection) at which all 8 volume
    corners fall inside the image shrunk by ``inset`` on every side."""
    pts = _corners(vol_lo, vol_hi)
    t = np.asarray(target, float)

    def cam_at(d):
        return look_at([t[0] + d * np.cos(az), t[1] + d * np.sin(az), height], t, f, W, H)

    lo_d, hi_d = 0.5, 1000.0
    assert _fits_inset(cam_at(hi_d), pts, inset)
    for _ in range(80):
        mid = 0.5 * (lo_d + hi_d)
        if _fits_inset(cam_at(mid), pts, inset):
            hi_d = mid
        else:
            lo_d = mid
    return cam_at(hi_d)


# --------------------------------------------------------------------------- objects
@dataclass
class Ellipsoid:
    center: np.ndarray     # (3,)
    Q: np.ndarray          # 3x3 rotation, columns are the principal axes
    axes: np.ndarray       # (3,) semi-axes

    @property
    def M(self) -> np.ndarray:
        return self.Q @ np.diag(1.0 / self.axes ** 2) @ self.Q.T

    def aabb(self) -> Tuple[np.ndarray, np.ndarray]:
        half = np.sqrt(((self.Q * self.axes[None, :]) ** 2).sum(axis=1))
        return self.center - half, self.center + half

    def inside(self, X: np.ndarray, scale: float = 1.0) -> np.ndarray:
        """(X-c)^T M (X-c) <= scale^2 for points X [..., 3]."""
        d = X - self.center
        return np.einsum('...i,ij,...j->...', d, self.M, d) <= scale * scale


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], float)


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], float)


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], float)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def player(rng: np.random.Generator, pos_xy, yaw: float, scale: float, lift: float,
           tilt: float = 0.0) -> List[Ellipsoid]:
    """A standing (or tilted) player as 5 ellipsoids in a local frame
    (x forward, y lateral, z up), then tilted about local y, yawed and placed."""
    s = scale
    parts = [(np.array([0.0, 0.0, 0.45 * s]), np.eye(3), np.array([0.18, 0.12, 0.45]) * s),   # legs
             (np.array([0.0, 0.0, 1.20 * s]), np.eye(3), np.array([0.20, 0.13, 0.32]) * s),   # torso
             (np.array([0.0, 0.0, 1.68 * s]), np.eye(3), np.array([0.10, 0.10, 0.12]) * s)]   # head
    for side in (+1.0, -1.0):                                                            # arms
        a = np.deg2rad(rng.uniform(0.0, 150.0))
        Rx = rot_x(side * a)
        shoulder = np.array([0.0, side * 0.24 * s, 1.45 * s])
        d = Rx @ np.array([0.0, 0.0, -1.0])
        parts.append((shoulder + 0.32 * s * d, Rx, np.array([0.05, 0.05, 0.32]) * s))
    Rt = rot_y(tilt)
    Rw = rot_z(yaw)
    out = []
    for c, Q, ax in parts:
        c2 = Rw @ (Rt @ c)
        out.append(Ellipsoid(center=c2, Q=Rw @ Rt @ Q, axes=ax.copy()))
    # rest on the floor (lowest point at z = 0.02 m) unless lifted by a jump
    zmin = min(e.aabb()[0][2] for e in out)
    dz = 0.02 - zmin + lift
    for e in out:
        e.center = e.center + np.array([pos_xy[0], pos_xy[1], dz])
    return out


# --------------------------------------------------------------------------- rendering
def render_masks(cams: List[Camera], ells: List[Ellipsoid]) -> np.ndarray:
    """uint8 [N][H][W]: 1 iff the ray through pixel centre (x+0.5, y+0.5) hits an
    ellipsoid in front of the camera (FP64 quadratic discriminant)."""
    N, H, W = len(cams), cams[0].H, cams[0].W
    out = np.zeros((N, H, W), np.uint8)
    for ci, cam in enumerate(cams):
        f, cx, cy = cam.K[0, 0], cam.K[0, 2], cam.K[1, 2]
        for e in ells:
            lo, hi = e.aabb()
            x, y, d = project64(cam, _corners(lo, hi))
            if np.any(d <= 0):
                raise ValueError("ellipsoid straddles a camera plane")
            x0 = max(int(np.floor(x.min())) - 2, 0)
            x1 = min(int(np.ceil(x.max())) + 2, W)
            y0 = max(int(np.floor(y.min())) - 2, 0)
            y1 = min(int(np.ceil(y.max())) + 2, H)
            if x0 >= x1 or y0 >= y1:
                continue
            M = e.M
            ev = cam.C - e.center
            cq = ev @ M @ ev - 1.0
            if cq <= 0:
                raise ValueError("camera inside an ellipsoid")
            Mp = cam.R @ M @ cam.R.T
            bp = cam.R @ (M @ ev)
            ux = ((np.arange(x0, x1) + 0.5 - cx) / f)[None, :]
            uy = ((np.arange(y0, y1) + 0.5 - cy) / f)[:, None]
            A = (Mp[0, 0] * ux * ux + Mp[1, 1] * uy * uy + Mp[2, 2]
                 + 2 * Mp[0, 1] * ux * uy + 2 * Mp[0, 2] * ux + 2 * Mp[1, 2] * uy)
            B = bp[0] * ux + bp[1] * uy + bp[2]
            hit = (B * B - A * cq >= 0) & (B < 0)
            out[ci, y0:y1, x0:x1] |= hit.astype(np.uint8)
    return out


def flip_boundary_noise(masks: np.ndarray, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Flip ``frac`` of the boundary pixels (pixels with a 4-neighbour of the
    opposite value) of each camera, chosen uniformly without replacement."""
    out = masks.copy()
    for ci in range(masks.shape[0]):
        m = masks[ci].astype(bool)
        b = np.zeros_like(m)
        b[1:, :] |= m[1:, :] != m[:-1, :]
        b[:-1, :] |= m[:-1, :] != m[1:, :]
        b[:, 1:] |= m[:, 1:] != m[:, :-1]
        b[:, :-1] |= m[:, :-1] != m[:, 1:]
        idx = np.flatnonzero(b)
        k = int(round(frac * idx.size))
        if k:
            pick = rng.choice(idx, size=k, replace=False)
            flat = out[ci].reshape(-1)
            flat[pick] ^= 1
    return out


# --------------------------------------------------------------------------- scenes
@dataclass
class Scene:
    name: str
    cfg: int
    frame: int
    cams: List[Camera]
    masks: np.ndarray                 # uint8 [N][H][W]
    ellipsoids: List[Ellipsoid]
    vol_lo: np.ndarray
    vol_hi: np.ndarray
    origin: np.ndarray                # float32 (3,), the volume's min corner
    hc_um: int                        # coarse voxel size, micrometres
    hf_um: int                        # fine voxel size, micrometres
    coarse_dims: Tuple[int, int, int]
    t_np: int = 8
    t_nb: int = UINT32_MAX
    n_steps: int = 8
    noisy: bool = False
    groups: List[List[int]] = field(default_factory=list)   # ellipsoid indices per object

    @property
    def P32(self) -> np.ndarray:
        return np.stack([c.P32 for c in self.cams]).astype(np.float32)

    @property
    def W(self) -> int:
        return self.cams[0].W

    @property
    def H(self) -> int:
        return self.cams[0].H

    @property
    def hc(self) -> np.float32:
        return um_to_h(self.hc_um)

    @property
    def hf(self) -> np.float32:
        return um_to_h(self.hf_um)


def um_to_h(um: int) -> np.float32:
    """Voxel size in metres as float32: the double um*1e-6 rounded once."""
    return np.float32(float(um) * 1e-6)


def lattice_dims(extent_m: float, h_um: int) -> int:
    """Corner-anchored lattice: samples at 0, h, ..., extent - h."""
    q, r = divmod(int(round(extent_m * 1_000_000)), h_um)
    return q if r == 0 else q + 1


def _bounding_sphere_in_image(cams, e: Ellipsoid) -> bool:
    r = float(e.axes.max())
    for cam in cams:
        x, y, d = project64(cam, e.center[None, :])
        if d[0] <= r:
            return False
        rp = cam.K[0, 0] * r / np.sqrt(d[0] ** 2 - r * r)
        if not (x[0] - rp >= 0 and x[0] + rp < cam.W and y[0] - rp >= 0 and y[0] + rp < cam.H):
            return False
    return True


def tiny_rig(n_cams: int = 4) -> List[Camera]:
    return [look_at([6 * np.cos(2 * np.pi * k / n_cams), 6 * np.sin(2 * np.pi * k / n_cams), 0.0],
                    [0, 0, 0], 300.0, 320, 240) for k in range(n_cams)]


def scene_tiny(seed: int, n_cams: int = 4) -> Scene:
    rng = rng_for(CFG_TINY, seed, 1)
    cams = tiny_rig(n_cams)
    while True:
        ells = []
        for _ in range(2):
            ells.append(Ellipsoid(center=np.array([rng.uniform(-1.4, 1.4), rng.uniform(-1.4, 1.4),
                                                   rng.uniform(-0.4, 0.4)]),
                                  Q=random_rotation(rng), axes=rng.uniform(0.2, 0.5, size=3)))
        if all(_bounding_sphere_in_image(cams, e) for e in ells):
            break
    lo, hi = np.array([-2.0, -2.0, -1.0]), np.array([2.0, 2.0, 1.0])
    return Scene(name="tiny", cfg=CFG_TINY, frame=seed, cams=cams, masks=render_masks(cams, ells),
                 ellipsoids=ells, vol_lo=lo, vol_hi=hi, origin=lo.astype(np.float32),
                 hc_um=62500, hf_um=20000,
                 coarse_dims=(lattice_dims(4, 62500), lattice_dims(4, 62500), lattice_dims(2, 62500)),
                 groups=[[0], [1]])


def _court_rig(cfg: int, frame: int, n: int, W: int, H: int, f_lo: float, f_hi: float,
               vol_lo, vol_hi) -> List[Camera]:
    rng = rng_for(cfg, frame, 0)
    target = 0.5 * (np.asarray(vol_lo, float) + np.asarray(vol_hi, float))
    cams = []
    for k in range(n):
        az = 2 * np.pi * k / n + np.deg2rad(rng.uniform(-5.0, 5.0))
        height = rng.uniform(3.0, 8.0)
        f = rng.uniform(f_lo, f_hi)
        cams.append(ring_camera_min_distance(az, height, f, W, H, vol_lo, vol_hi, target))
    return cams


def _place_players(rng, n_per_half: int, x_rng, y_rng, spacing: float):
    pts = []
    for half in (-1, +1):
        placed = 0
        while placed < n_per_half:
            p = np.array([half * rng.uniform(*x_rng), rng.uniform(*y_rng)])
            if all(np.linalg.norm(p - q) >= spacing for q in pts):
                pts.append(p)
                placed += 1
    return pts


def scene_volleyball(frame: int) -> Scene:
    lo, hi = np.array([-9.0, -4.5, 0.0]), np.array([9.0, 4.5, 4.0])
    cams = _court_rig(CFG_VOLLEYBALL, 0, 16, 1920, 1080, 1800.0, 2400.0, lo, hi)   # static rig
    rng = rng_for(CFG_VOLLEYBALL, frame, 1)
    ells, groups = [], []
    for p in _place_players(rng, 6, (0.8, 8.2), (-3.8, 3.8), 1.0):
        yaw = rng.uniform(0, 2 * np.pi)
        s = rng.uniform(0.9, 1.1)
        lift = rng.uniform(0.2, 0.8) if rng.uniform() < 0.25 else 0.0
        es = player(rng, p, yaw, s, lift)
        groups.append(list(range(len(ells), len(ells) + len(es))))
        ells += es
    return Scene(name="volleyball", cfg=CFG_VOLLEYBALL, frame=frame, cams=cams,
                 masks=render_masks(cams, ells), ellipsoids=ells, vol_lo=lo, vol_hi=hi,
                 origin=lo.astype(np.float32), hc_um=100000, hf_um=10000,
                 coarse_dims=(lattice_dims(18, 100000), lattice_dims(9, 100000), lattice_dims(4, 100000)),
                 groups=groups)


def scene_judo(frame: int) -> Scene:
    lo, hi = np.array([-5.0, -5.0, 0.0]), np.array([5.0, 5.0, 3.0])
    cams = _court_rig(CFG_JUDO, 0, 24, 3840, 2160, 3600.0, 4800.0, lo, hi)   # static rig
    rng = rng_for(CFG_JUDO, frame, 1)
    n_pairs = int(rng.integers(1, 3))          # 2-4 players in touching pairs
    ells, groups = [], []
    centres = []
    while len(centres) < n_pairs:
        c = np.array([rng.uniform(-3.0, 3.0), rng.uniform(-3.0, 3.0)])
        if all(np.linalg.norm(c - q) >= 2.5 for q in centres):
            centres.append(c)
    for c in centres:
        yaw = rng.uniform(0, 2 * np.pi)
        s1, s2 = rng.uniform(0.9, 1.1, size=2)
        gap = rng.uniform(-0.03, 0.01)
        sep = 0.20 * s1 + 0.20 * s2 + gap
        fwd = np.array([np.cos(yaw), np.sin(yaw)])
        for who, (s, off, yw) in enumerate([(s1, -0.5 * sep, yaw), (s2, 0.5 * sep, yaw + np.pi)]):
            tilt = np.deg2rad(rng.uniform(45.0, 90.0)) if rng.uniform() < 0.3 else 0.0
            es = player(rng, c + off * fwd, yw, s, 0.0, tilt=tilt)
            groups.append(list(range(len(ells), len(ells) + len(es))))
            ells += es
    masks = flip_boundary_noise(render_masks(cams, ells), 0.01, rng_for(CFG_JUDO, frame, 2))
    return Scene(name="judo", cfg=CFG_JUDO, frame=frame, cams=cams, masks=masks, ellipsoids=ells,
                 vol_lo=lo, vol_hi=hi, origin=lo.astype(np.float32), hc_um=40000, hf_um=5000,
                 coarse_dims=(lattice_dims(10, 40000), lattice_dims(10, 40000), lattice_dims(3, 40000)),
                 noisy=True, groups=groups)


def scene_paper_volleyball(frame: int) -> Scene:
    """The shape of the paper's volleyball experiment: an 18 x 18 x 9 m volume,
    coarse 50 mm (360 x 360 x 180 samples), fine 20 mm, 10 cameras of 3840 x
    2160 with f about 3000 px, 14 players (7 per half of an 18 x 9 m court
    in the middle of the volume, spacing >= 1 m)."""
    lo, hi = np.array([-9.0, -9.0, 0.0]), np.array([9.0, 9.0, 9.0])
    cams = _court_rig(CFG_PAPER_V, 0, 10, 3840, 2160, 2900.0, 3100.0, lo, hi)   # static rig
    rng = rng_for(CFG_PAPER_V, frame, 1)
    ells, groups = [], []
    for p in _place_players(rng, 7, (0.8, 8.2), (-3.8, 3.8), 1.0):
        yaw = rng.uniform(0, 2 * np.pi)
        s = rng.uniform(0.9, 1.1)
        lift = rng.uniform(0.2, 0.8) if rng.uniform() < 0.25 else 0.0
        es = player(rng, p, yaw, s, lift)
        groups.append(list(range(len(ells), len(ells) + len(es))))
        ells += es
    return Scene(name="paper_volleyball", cfg=CFG_PAPER_V, frame=frame, cams=cams,
                 masks=render_masks(cams, ells), ellipsoids=ells, vol_lo=lo, vol_hi=hi,
                 origin=lo.astype(np.float32), hc_um=50000, hf_um=20000,
                 coarse_dims=(lattice_dims(18, 50000), lattice_dims(18, 50000),
                              lattice_dims(9, 50000)),
                 groups=groups)


def scene_judo_fine(frame: int) -> Scene:
    """The judo frame (rig, players, noise) with 2 mm fine voxels: ~1e8 fine
    samples in its ROIs."""
    sc = scene_judo(frame)
    sc.name, sc.cfg, sc.hf_um = "judo_fine", CFG_JUDO_FINE, 2000
    return sc


def make_scene(cfg: int, frame: int) -> Scene:
    if cfg == CFG_TINY:
        return scene_tiny(frame)
    if cfg == CFG_VOLLEYBALL:
        return scene_volleyball(frame)
    if cfg == CFG_JUDO:
        return scene_judo(frame)
    if cfg == CFG_PAPER_V:
        return scene_paper_volleyball(frame)
    if cfg == CFG_JUDO_FINE:
        return scene_judo_fine(frame)
    raise ValueError(f"no single-frame scene for cfg {cfg}")


# --------------------------------------------------------------------------- batched ROIs
@dataclass
class RoiBox:
    frame: int
    lo: Tuple[int, int, int]          # global fine lattice index of the box's first sample
    dims: Tuple[int, int, int]


def batched_rois(n_frames: int = 64, rois_per_frame: int = 12, hf_um: int = 10000,
                 edge_lo: float = 0.6, edge_hi: float = 2.5) -> Tuple[List[Scene], List[RoiBox]]:
    """The batched workload: one tiny-rig scene per frame and, per frame,
    ``rois_per_frame`` boxes with per-axis edges U[edge_lo, edge_hi] m and
    centres uniform in the tiny volume (not clipped), on the fine lattice
    anchored at the tiny volume's min corner."""
    scenes, boxes = [], []
    for fr in range(n_frames):
        sc = scene_tiny(1000 + fr)
        sc.cfg, sc.frame, sc.hf_um = CFG_BATCHED, fr, hf_um
        scenes.append(sc)
        rng = rng_for(CFG_BATCHED, fr, 3)
        for _ in range(rois_per_frame):
            edge = rng.uniform(edge_lo, edge_hi, size=3)
            centre = rng.uniform(sc.vol_lo, sc.vol_hi)
            n = np.maximum(np.round(edge * 1e6 / hf_um).astype(int), 1)
            c_idx = np.round((centre - sc.vol_lo) * 1e6 / hf_um).astype(int)
            lo = c_idx - n // 2
            boxes.append(RoiBox(frame=fr, lo=tuple(int(v) for v in lo), dims=tuple(int(v) for v in n)))
    return scenes, boxes


# --------------------------------------------------------------------------- soft hull
CFG_SOFT = 5


@dataclass
class SoftScene:
    """Inputs of the differentiable soft hull: a 16-camera tiny ring with
    perturbed poses, silhouette logits and a lattice around one object with
    its true occupancy as the target."""
    cams: List[Camera]                # base poses (the rig as calibrated)
    omega: np.ndarray                 # float32 [N][3], rotation perturbations (radians)
    tau: np.ndarray                   # float32 [N][3], translation perturbations (metres)
    logits: np.ndarray                # float32 [N][H][W]
    origin: np.ndarray                # float32 (3,)
    h: np.float32
    lo: Tuple[int, int, int]
    dims: Tuple[int, int, int]
    target: np.ndarray                # float32 [nz][ny][nx], 1 inside the object
    ellipsoids: List[Ellipsoid]

    @property
    def W(self) -> int:
        return self.cams[0].W

    @property
    def H(self) -> int:
        return self.cams[0].H

    def base_pose(self):
        """fx, fy, cx, cy [N][4], R0 [N][3][3], t0 [N][3] (float64): X_cam = R0 X + t0."""
        K = np.array([[c.K[0, 0], c.K[1, 1], c.K[0, 2], c.K[1, 2]] for c in self.cams])
        R0 = np.stack([c.R for c in self.cams])
        t0 = np.stack([-c.R @ c.C for c in self.cams])
        return K, R0, t0


def _blur3(img: np.ndarray, passes: int) -> np.ndarray:
    """Separable [1, 2, 1]/4 smoothing, edge-replicated, `passes` times."""
    out = img.astype(np.float64)
    for _ in range(passes):
        for ax in (0, 1):
            p = np.pad(out, [(1, 1) if a == ax else (0, 0) for a in range(2)], mode="edge")
            sl = [slice(None)] * 2
            a = p[tuple(sl[:ax] + [slice(0, -2)] + sl[ax + 1:])]
            b = p[tuple(sl[:ax] + [slice(1, -1)] + sl[ax + 1:])]
            c = p[tuple(sl[:ax] + [slice(2, None)] + sl[ax + 1:])]
            out = 0.25 * a + 0.5 * b + 0.25 * c
    return out


def scene_soft(seed: int, n_cams: int = 16, h_um: int = 20000, margin: float = 0.06,
               rot_sigma_deg: float = 0.5, trans_sigma_m: float = 0.01) -> SoftScene:
    """The tiny scene of `seed` seen by an n_cams ring; logits = 6 (2 s - 1) for
    the rendered silhouettes smoothed to s in [0, 1] (two [1,2,1] passes) plus
    N(0, 0.1) noise; poses perturbed by omega ~ N(0, rot_sigma) per axis and
    tau ~ N(0, trans_sigma); the lattice covers object 0's box plus `margin`."""
    sc = scene_tiny(seed)
    cams = tiny_rig(n_cams)
    masks = render_masks(cams, sc.ellipsoids)
    rng = rng_for(CFG_SOFT, seed, 2)
    logits = np.stack([6.0 * (2.0 * _blur3(m, 2) - 1.0) for m in masks])
    logits = (logits + rng.normal(0.0, 0.1, size=logits.shape)).astype(np.float32)
    rng = rng_for(CFG_SOFT, seed, 0)
    omega = rng.normal(0.0, np.deg2rad(rot_sigma_deg), size=(n_cams, 3)).astype(np.float32)
    tau = rng.normal(0.0, trans_sigma_m, size=(n_cams, 3)).astype(np.float32)
    e = sc.ellipsoids[0]
    blo, bhi = e.aabb()
    h = um_to_h(h_um)
    origin = sc.origin
    hd = float(h_um) * 1e-6
    lo = tuple(int(np.floor((blo[a] - margin - origin[a]) / hd)) for a in range(3))
    hi = tuple(int(np.ceil((bhi[a] + margin - origin[a]) / hd)) for a in range(3))
    dims = tuple(hi[a] - lo[a] + 1 for a in range(3))
    g = [origin[a] + (lo[a] + np.arange(dims[a])) * hd for a in range(3)]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    target = e.inside(np.stack([X, Y, Z], -1)).astype(np.float32)
    return SoftScene(cams=cams, omega=omega, tau=tau, logits=logits, origin=origin, h=h, lo=lo,
                     dims=dims, target=target, ellipsoids=sc.ellipsoids)
