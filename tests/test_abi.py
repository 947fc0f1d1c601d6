"""The C ABI on the CPU: the built library loads, exports every function that
include/fvv.h declares, and its one host-only call (the ROI -> fine lattice
mapping of Sec. II-B-3) agrees with the oracle.  No GPU work here."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fvv_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def fvv():
    import paper_1903_11785_amd as fvv
    return fvv


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fvv_carve", "fvv_label", "fvv_surface", "fvv_roi_grids", "fvv_carve_batched",
                 "fvv_frame", "fvv_pack_silhouettes", "fvv_mesh", "fvv_isovalue",
                 "fvv_visibility", "fvv_gather_peak", "fvv_soft_forward", "fvv_soft_backward"):
        assert must in names


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the
    C compiler gives the header's structs (host-only compile of a probe)."""
    import ctypes as C
    import json
    import shutil
    import subprocess
    import paper_1903_11785_amd as fvv
    cxx = "/opt/rocm/bin/amdclang++"
    if not os.path.exists(cxx):
        cxx = shutil.which("hipcc")
    assert cxx, "no HIP host compiler"
    exe = tmp_path / "abi_layout"
    subprocess.check_call([cxx, "-x", "hip", "--cuda-host-only", "-std=c++17",
                           f"-I{os.path.join(ROOT, 'include')}",
                           os.path.join(ROOT, "tests", "abi_layout.cpp"), "-o", str(exe)])
    got = json.loads(subprocess.check_output([str(exe)]).decode())
    structs = {"fvv_camera": fvv.Camera, "fvv_grid": fvv.GridC, "fvv_roi": fvv.Roi,
               "fvv_job": fvv.Job, "fvv_limits": fvv.Limits, "fvv_tile": fvv.Tile,
               "fvv_frame_params": fvv.FrameParams, "fvv_frame_out": fvv.FrameOut,
               "fvv_soft_camera": fvv.SoftCamera}
    checked = 0
    for key, value in got.items():
        if key == "end":
            continue
        if "." in key:
            t, f = key.split(".")
            assert getattr(structs[t], f).offset == value, key
        else:
            assert C.sizeof(structs[key]) == value, key
        checked += 1
    assert checked > 40


def test_library_exports_every_declared_symbol(fvv):
    L = fvv.library()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings(fvv):
    assert fvv.status_str(0) == "ok"
    assert "capacity" in fvv.status_str(-2)


def test_roi_grids_host_call_matches_oracle(fvv):
    rng = np.random.default_rng(11)
    for _ in range(300):
        hc = int(rng.choice([62500, 100000, 40000]))
        hf = int(rng.choice([20000, 10000, 5000]))
        dims = tuple(int(v) for v in rng.integers(2, 100, 3))
        lo = tuple(int(v) for v in rng.integers(-20, 20, 3))
        coarse = fvv.Grid(origin=(-9.0, -4.5, 0.0), h=np.float32(hc * 1e-6), lo=lo, dims=dims)
        k = int(rng.integers(1, 6))
        rows = []
        for _ in range(k):
            blo = [int(rng.integers(0, d)) for d in dims]
            bhi = [int(rng.integers(b, d)) for b, d in zip(blo, dims)]
            rows.append([*blo, *bhi, 1, 0])
        got = fvv.roi_grids(coarse, hc, hf, np.array(rows, np.int32))
        olat = oracle.Lattice(origin=np.float32(coarse.origin), h=np.float32(coarse.h), lo=lo,
                              dims=dims)
        for r, g in zip(rows, got):
            ref = oracle.roi_fine(olat, hc, hf, np.float32(float(hf) * 1e-6), r[0:3], r[3:6])
            assert g.lo == ref.lo and g.dims == ref.dims
            assert np.float32(g.h) == np.float32(ref.h)
            assert np.all(np.float32(g.origin) == np.float32(coarse.origin))


def test_roi_grids_rejects_bad_arguments(fvv):
    coarse = fvv.Grid(origin=(0, 0, 0), h=0.1, lo=(0, 0, 0), dims=(10, 10, 10))
    with pytest.raises(fvv.FvvError):
        fvv.roi_grids(coarse, 0, 10000, np.zeros((1, 8), np.int32))
    with pytest.raises(fvv.FvvError):
        fvv.roi_grids(coarse, 100000, 10000, np.array([[0, 0, 0, 10, 0, 0, 1, 0]], np.int32))


def test_no_cpu_fallback_without_gpu(fvv):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        fvv.Context()
