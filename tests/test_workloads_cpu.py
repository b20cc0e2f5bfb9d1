"""Seeded input generators: the windowed permittivity map used by the
128^3 accuracy rerun is exactly the corresponding window of the full map."""
import numpy as np

from paper_2502_20610_amd import workloads as wl


def test_windowed_paint_matches_full_map():
    shape = (90, 70, 60)
    full = wl.paint_boxes(shape, 120, 4, 30, 2.08, 12.25, np.random.default_rng(9))
    for lo, size in [((0, 0, 0), shape), ((10, 20, 5), (40, 30, 50)), ((89, 69, 59), (1, 1, 1))]:
        win = wl.paint_boxes(shape, 120, 4, 30, 2.08, 12.25, np.random.default_rng(9),
                             window=(lo, size))
        ref = full[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]]
        np.testing.assert_array_equal(win, ref)


def test_c3_centre_crop_recipe():
    w = wl.c3_centre_crop(n=32, nsteps=10)
    assert w.shape == (32, 32, 32) and w.bc == (0, 0, 0)
    assert set(np.unique(w.eps)) <= {np.float32(2.08), np.float32(12.25)}
    assert [(s["i"], s["j"], s["k"], s["comp"]) for s in w.sources] == [(16, 16, 16, wl.EZ)]


def test_graded_shell_profile():
    """Plane-by-plane build equals the broadcast definition: sigma_max times
    the squared relative depth into the shell, zero from `thickness` cells in."""
    shape, th, smax = (23, 17, 30), 5, 0.4
    s = wl.graded_shell(shape, th, smax)
    d = np.minimum.reduce(np.meshgrid(*[np.minimum(np.arange(n), n - 1 - np.arange(n)) for n in shape],
                                      indexing="ij"))
    ref = np.where(d < th, smax * ((th - d) / th) ** 2, 0.0).astype(np.float32)
    np.testing.assert_array_equal(s, ref)
    assert s.dtype == np.float32 and s[0, 8, 15] == np.float32(smax) and s[11, 8, 15] == 0.0
