"""GPU parity of FP16 field storage (binary16 device arrays, FP32 arithmetic)
against the FP16-storage oracle, bit for bit: the systolic scheme rounds the
grid once per band, the plain scheme after every half-step and source.  Also
the ABI conversions (input rounding, exact read-back, scales, re-encoding),
the accuracy bar on the 128^3 crop of the 1024x1024x512 workload, and the
calls that need FP32 storage."""
import numpy as np
import pytest

import oracle
from oracle import f16
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym
from tests.test_gpu_parity import assert_bitwise

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def _sim(w, scheme, band=0, exp2=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, storage="fp16")
    if band:
        sim.set_option(fdtd.OPT_BAND_STEPS, band)
    if exp2 is not None:
        sim.set_field_scale(exp2)
    sim.set_materials(w.eps)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


def _cE(w):
    return f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)


CASES = [
    ((40, 36, 34), (PEC, PEC, PEC), 8, None),
    ((35, 29, 40), (PER, PER, PER), 5, None),
    ((31, 47, 29), (PEC, PER, PEC), 0, (1, -2, 0, 3, -1, 2)),
    ((12, 9, 7), (PEC, PEC, PEC), 3, None),
]


@pytest.mark.parametrize("shape,bc,band,exp2", CASES)
def test_systolic_f16_bitwise(shape, bc, band, exp2):
    w = wl.small_case(shape, bc, seed=sum(shape), nsteps=30,
                      dipoles=[tuple(s // 2 for s in shape), (1, 1, 0)])
    e = exp2 or (0,) * 6
    sim = _sim(w, "systolic", band, exp2)
    calls, bands = [], []
    for n in (17, 13):   # two calls: bands restart at each call
        sim.step(n)
        calls.append(n)
        bands.append(sim.info(fdtd.INFO_SYSTOLIC_BAND))
    ref = f16.run_systolic(w.fields, _cE(w), np.float32(w.dt / w.dx), calls, bands,
                           sources=w.sources, exp2=e)
    assert_bitwise(sim.read_fields(), ref, "fp16 systolic %s %s" % (shape, bc))
    sim.close()


@pytest.mark.parametrize("shape,bc,exp2", [((33, 29, 40), (PEC, PEC, PEC), None),
                                           ((20, 18, 24), (PER, PEC, PER), (2, 0, -1, 1, 1, -3))])
def test_plain_f16_bitwise(shape, bc, exp2):
    w = wl.small_case(shape, bc, seed=7, nsteps=21, dipoles=[tuple(s // 2 for s in shape)])
    e = exp2 or (0,) * 6
    sim = _sim(w, "plain", exp2=exp2)
    sim.step(21)
    ref = f16.run_plain(w.fields, _cE(w), np.float32(w.dt / w.dx), 21, sources=w.sources, exp2=e)
    assert_bitwise(sim.read_fields(), ref, "fp16 plain %s" % (shape,))
    sim.close()


def test_f16_batch_bitwise_and_mixed_storage_refused():
    ws = [wl.small_case(sh, bc, seed=50 + q, nsteps=19, dipoles=[tuple(s // 2 for s in sh)])
          for q, (sh, bc, _, _) in enumerate(CASES[:3])]
    sims = [_sim(w, "systolic", 6) for w in ws]
    fp32 = fdtd.Simulation(ws[0].shape, ws[0].dt, ws[0].dx, ws[0].bc, scheme="systolic")
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([sims[0], fp32], 3)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        fdtd.step_batch(sims, 19)
        for w, s in zip(ws, sims):
            ref = f16.run_systolic(w.fields, _cE(w), np.float32(0.5), [19], [6], sources=w.sources)
            assert_bitwise(s.read_fields(), ref, "fp16 batch member %s" % (w.shape,))
    finally:
        fp32.close()
        for s in sims:
            s.close()


def test_f16_field_io_rounding_scales_and_reencoding():
    import torch
    shape = (8, 9, 10)
    rng = np.random.default_rng(3)
    vals = [(rng.standard_normal(shape) * 10.0 ** rng.integers(-9, 6, shape)).astype(np.float32)
            for _ in range(6)]
    vals[0][1, 2, 3] = 70000.0       # overflows to +inf at scale 1
    vals[4][2, 2, 2] = 3e-8          # rounds to the smallest subnormal
    vals[1][0, 0, 0] = -0.0          # signed zeros survive every conversion
    vals[5][3, 3, 3] = -1e-12        # rounds to -0
    sim = fdtd.Simulation(shape, 0.5, 1.0, (PER, PER, PER), storage="fp16")
    try:
        sim.set_fields(vals)
        got = sim.read_fields()
        for c in range(6):
            np.testing.assert_array_equal(got[c].view(np.uint32), f16.store(vals[c]).view(np.uint32))
        assert np.isposinf(got[0][1, 2, 3]) and got[4][2, 2, 2] == np.float32(2.0 ** -24)
        assert np.signbit(got[1][0, 0, 0]) and np.signbit(got[5][3, 3, 3]) and got[5][3, 3, 3] == 0
        # device input and output take the same path
        dev = [torch.from_numpy(v).cuda() for v in vals]
        out = [torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(6)]
        torch.cuda.synchronize()
        sim.set_fields(dev)
        sim.read_fields(out=out)
        sim.synchronize()
        for c in range(6):
            np.testing.assert_array_equal(out[c].cpu().numpy().view(np.uint32),
                                          f16.store(vals[c]).view(np.uint32))
        # new scales re-encode the stored values
        e = (3, -4, 0, 8, -20, 1)
        sim.set_field_scale(e)
        got = sim.read_fields()
        for c in range(6):
            np.testing.assert_array_equal(got[c].view(np.uint32),
                                          f16.store(f16.store(vals[c]), e[c]).view(np.uint32))
        sim.set_fields(vals)
        got = sim.read_fields()
        for c in range(6):
            np.testing.assert_array_equal(got[c].view(np.uint32), f16.store(vals[c], e[c]).view(np.uint32))
        with pytest.raises(fdtd.FdtdError) as err:
            sim.set_field_scale((0, 0, 0, 31, 0, 0))
        assert err.value.code == fdtd.FDTD_EINVAL
    finally:
        sim.close()


def test_f16_needs_fp32_for_conductivity_and_adjoint():
    w = wl.small_case((20, 20, 20), (PEC, PEC, PEC), seed=11, nsteps=4)
    sim = _sim(w, "plain")
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            sim.set_materials(w.eps, sigma=np.zeros(w.shape, np.float32))
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        with pytest.raises(fdtd.FdtdError) as e:
            sim.adjoint(2, 2, (10, 1, 1), (11, 9, 9), 0.5, (2, 2, 2), (5, 5, 5))
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        assert sim.current_step == 0
    finally:
        sim.close()
    s32 = fdtd.Simulation((8, 8, 8))
    with pytest.raises(fdtd.FdtdError) as e:
        s32.set_field_scale((0,) * 6)
    assert e.value.code == fdtd.FDTD_EINVAL
    s32.close()


def test_c3_crop_f16_accuracy_1000_steps():
    """The 128^3 centre crop of the 1024x1024x512 workload (its permittivity
    map, PEC walls, one dipole), 1000 steps with FP16 storage on the
    systolic scheme: bit-exact with the FP16 oracle, and within 2e-3
    relative L2 of the FP64 oracle run with the same (dequantised)
    coefficients."""
    w = wl.c3_centre_crop(nsteps=1000)
    sim = _sim(w, "systolic")
    sim.step(1000)
    K = sim.info(fdtd.INFO_SYSTOLIC_BAND)
    got = sim.read_fields()
    sim.close()
    cE = _cE(w)
    ref = f16.run_systolic(w.fields_or_zeros(), cE, np.float32(w.dt / w.dx), [1000], [K],
                           sources=w.sources)
    assert_bitwise(got, ref, "fp16 systolic, 128^3 crop")
    f64 = [np.array(x, np.float64) for x in w.fields_or_zeros()]
    oracle.step([c.astype(np.float64) for c in cE], w.dt / w.dx, f64, 1000, sources=w.sources,
                dtype=np.float64)
    err = ym.rel_l2(got, f64)
    assert 0 < err <= 2e-3, err
