"""The oracle's OpenMP loops give the same frame on one host thread as on all
of them (occupancies, labels, ROI boxes, edge keys, exit points and test
counts), and set_threads restores the previous count."""
import numpy as np

import oracle
import scenes


def test_frame_is_independent_of_the_thread_count():
    sc = scenes.make_scene(scenes.CFG_TINY, 0)
    args = (sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np, sc.t_nb,
            sc.n_steps)
    many = oracle.frame(*args)
    prev = oracle.set_threads(1)
    try:
        assert oracle.threads() == 1
        one = oracle.frame(*args)
    finally:
        oracle.set_threads(prev)
    assert oracle.threads() == prev
    assert len(many.rois) > 0 and many.fine_voxels > 0
    np.testing.assert_array_equal(one.occ_filtered, many.occ_filtered)
    np.testing.assert_array_equal(one.labels, many.labels)
    np.testing.assert_array_equal(one.rois, many.rois)
    for a, b in zip(one.occ_fine, many.occ_fine):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(one.keys, many.keys):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(one.xyz, many.xyz):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    assert (one.tests_coarse, one.tests_fine, one.tests_surface) == \
        (many.tests_coarse, many.tests_fine, many.tests_surface)
