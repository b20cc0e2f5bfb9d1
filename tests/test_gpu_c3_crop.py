"""Accuracy rerun of the 1024x1024x512 workload on its central 128^3 crop
(same permittivity map, PEC walls, one Ez dipole at the centre, 500 steps).

Both schemes must give the FP32 oracle's values bit for bit, and stay within
1e-5 relative L2 of the FP64 oracle over the six components (the FP32/FP64
gap of the Yee recurrence; the FP64 run uses the unrounded coefficients).
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym
from tests.test_gpu_parity import assert_bitwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crop():
    w = wl.c3_centre_crop()
    f32 = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, w.nsteps, sources=w.sources,
                     dtype=np.float32)
    f64 = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, w.nsteps, sources=w.sources,
                     dtype=np.float64)
    return w, f32, f64


@pytest.mark.parametrize("scheme", ["systolic", "plain"])
def test_c3_crop_bitwise_and_fp64_error(crop, scheme):
    w, f32, f64 = crop
    got = fdtd.run_workload(w, scheme)
    assert_bitwise(got, f32, "%s on the 128^3 crop" % scheme)
    err = ym.rel_l2(got, f64)
    assert 0 < err < 1e-5, err
    # the pulse has spread: a sizeable part of the crop is non-zero
    assert np.count_nonzero(got[2]) > got[2].size // 20
