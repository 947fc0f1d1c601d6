"""The gather-ceiling measurement aid (fvv_gather_peak): its reads stay in the
table and are the ones it states (each lane's sum over its steps, recomputed
on the host for sampled lanes from the same offset sequence), it returns a
finite positive rate, and it rejects invalid arguments."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ITERS = 256       # words per lane and launch, as the kernel states
BLOCK = 256


@pytest.fixture(scope="module")
def fvv():
    import paper_1903_11785_amd as fvv
    return fvv


@pytest.fixture(scope="module")
def ctx(fvv):
    c = fvv.Context(max_coarse=1 << 20, max_fine=1 << 20, max_rois=16, max_points=1 << 16,
                    max_jobs=16)
    yield c
    c.close()


def lane_sum(table, n_words, gid):
    """The sum lane gid takes: per-wave LCG offsets in [0, n_words - 64]."""
    M = 1 << 32
    x = ((gid // 64) * 2654435761 + 12345) % M
    span = n_words - 64 + 1
    acc = 0
    for _ in range(ITERS):
        x = (x * 1664525 + 1013904223) % M
        base = (x * span) >> 32
        acc = (acc + int(table[base + gid % 64])) % M
    return acc


@pytest.mark.parametrize("n_words", [64, 1000, 1 << 20])
def test_reads_and_rate(fvv, ctx, n_words):
    import ctypes as C
    import torch
    rng = np.random.default_rng(n_words)
    tab = rng.integers(0, 1 << 32, n_words, dtype=np.uint64).astype(np.uint32)
    d_tab = torch.from_numpy(tab.view(np.int32)).cuda()
    sink = torch.zeros(16384 * 256, dtype=torch.int32, device="cuda")
    out = C.c_double()
    st = ctx.L.fvv_gather_peak(ctx.h, C.c_void_p(d_tab.data_ptr()), n_words,
                               C.c_void_p(sink.data_ptr()), 3, C.byref(out), None)
    assert st == fvv.FVV_OK
    assert np.isfinite(out.value) and out.value > 1e9
    blocks = min(torch.cuda.get_device_properties(0).multi_processor_count * 64, 16384)
    got = sink.cpu().numpy().view(np.uint32)
    lanes = sorted({0, 1, 63, 64, 777, blocks * BLOCK - 1} |
                   set(rng.integers(0, blocks * BLOCK, 6).tolist()))
    for g in lanes:
        assert int(got[g]) == lane_sum(tab, n_words, g), g
    assert not got[blocks * BLOCK:].any()


def test_invalid_arguments(fvv, ctx):
    import ctypes as C
    import torch
    tab = torch.zeros(128, dtype=torch.int32, device="cuda")
    sink = torch.zeros(16384 * 256, dtype=torch.int32, device="cuda")
    out = C.c_double()
    for n, reps in ((63, 1), (128, 0), (128, 1001)):
        st = ctx.L.fvv_gather_peak(ctx.h, C.c_void_p(tab.data_ptr()), n,
                                   C.c_void_p(sink.data_ptr()), reps, C.byref(out), None)
        assert st == fvv.FVV_EINVAL
    with pytest.raises(fvv.FvvError):
        ctx.gather_peak(tab[:10])
