"""GPU parity of conductive (lossy) materials: the conductive E half-step of
both schemes (plain, and the systolic tile's 11-wide conductive variant)
against the FP32 lossy oracle, bit for bit; sigma = 0 through the lossy entry
point equals the lossless path; batches of conductive grids; invalid
conductivity is refused.  (The conductive adjoint is covered with the other
adjoint tests.)"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def _sigma(shape, seed, hi=0.3):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.0, hi, shape).astype(np.float32) for _ in range(3)]


def _lossy_ref(w, sig, n):
    return oracle.run(w.fields_or_zeros(), w.eps3(), w.bc, w.dt, w.dx, n, sources=w.sources,
                      dtype=np.float32, sigma=sig)


def _sim(w, sig, device=False, scheme="plain", band=0):
    import torch
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme)
    if band:
        sim.set_option(fdtd.OPT_BAND_STEPS, band)
    if device:
        dev = torch.device("cuda:0")
        sim.set_materials(torch.from_numpy(w.eps).to(dev),
                          sigma=[torch.from_numpy(s).to(dev) for s in sig])
    else:
        sim.set_materials(w.eps, sigma=sig)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PER), (PER, PEC, PER)])
@pytest.mark.parametrize("device", [False, True])
def test_lossy_plain_bitwise(bc, device):
    w = wl.small_case((33, 29, 40), bc, seed=8, nsteps=37, dipoles=[(16, 14, 20)])
    sig = _sigma(w.shape, 9)
    sim = _sim(w, sig, device)
    sim.step(37)
    assert_bitwise(sim.read_fields(), _lossy_ref(w, sig, 37), "lossy %s" % (bc,))
    sim.close()


def test_absorbing_shell_bitwise_and_decay():
    """A PEC box whose outer 6 cells conduct with a quadratic grading (a simple
    absorber around a dielectric core): bit-exact, and the field energy after
    the pulse has passed is far below the lossless run's."""
    n = 48
    w = wl.random_dielectric((n, n, n), (PEC, PEC, PEC), 8, 12, 300, side=(4, 12),
                             dipoles=[(24, 24, 24)])
    d = np.minimum.reduce(np.meshgrid(*[np.minimum(np.arange(n), n - 1 - np.arange(n))] * 3,
                                      indexing="ij"))
    prof = np.where(d < 6, 0.4 * ((6 - d) / 6.0) ** 2, 0.0).astype(np.float32)
    sig = [prof] * 3
    sim = _sim(w, sig)
    sim.step(300)
    got = sim.read_fields()
    sim.close()
    assert_bitwise(got, _lossy_ref(w, sig, 300), "absorber")
    sim = _sim(w, sig, scheme="systolic")
    sim.step(300)
    assert sim.info(fdtd.INFO_TILE_X) == 11
    assert_bitwise(sim.read_fields(), got, "absorber, systolic")
    sim.close()
    ref0 = oracle_f32(w, 300)
    e_lossy = sum(float(np.sum(np.asarray(f, np.float64) ** 2)) for f in got)
    e_lossless = sum(float(np.sum(np.asarray(f, np.float64) ** 2)) for f in ref0)
    assert e_lossy < 0.5 * e_lossless


# (shape, boundaries, band): several 11-wide x tiles with a ragged periodic
# ring tile (35 = 3 * 11 + 2), short axes, several bands per call
SYSTOLIC_CASES = [
    ((33, 29, 40), (PEC, PEC, PEC), 0),
    ((35, 29, 40), (PER, PER, PER), 0),
    ((35, 31, 17), (PER, PEC, PER), 8),
    ((23, 16, 45), (PEC, PER, PEC), 5),
    ((12, 9, 7), (PEC, PEC, PEC), 0),
]


@pytest.mark.parametrize("shape,bc,band", SYSTOLIC_CASES)
def test_lossy_systolic_bitwise(shape, bc, band):
    w = wl.small_case(shape, bc, seed=sum(shape), nsteps=37,
                      dipoles=[tuple(s // 2 for s in shape), (1, 1, 0)])
    sig = _sigma(w.shape, sum(shape) + 1)
    sim = _sim(w, sig, scheme="systolic", band=band)
    sim.step(20)
    sim.step(17)   # a second call continues the same state
    assert sim.info(fdtd.INFO_TILE_X) == 11
    assert_bitwise(sim.read_fields(), _lossy_ref(w, sig, 37), "lossy systolic %s %s" % (shape, bc))
    sim.close()


def test_lossy_batch_and_mixed_batch_refused():
    ws = [wl.small_case(sh, bc, seed=30 + q, nsteps=19, dipoles=[tuple(s // 2 for s in sh)])
          for q, (sh, bc, _) in enumerate(SYSTOLIC_CASES[:4])]
    sigs = [_sigma(w.shape, 40 + q) for q, w in enumerate(ws)]
    sims = [_sim(w, s, scheme="systolic") for w, s in zip(ws, sigs)]
    lossless = fdtd.Simulation(ws[0].shape, ws[0].dt, ws[0].dx, ws[0].bc, scheme="systolic")
    try:
        lossless.set_materials(ws[0].eps)
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([sims[0], lossless], 3)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        assert sims[0].current_step == 0 and lossless.current_step == 0
        fdtd.step_batch(sims, 19)
        for w, sg, s in zip(ws, sigs, sims):
            assert_bitwise(s.read_fields(), _lossy_ref(w, sg, 19), "lossy batch member %s" % (w.shape,))
    finally:
        lossless.close()
        for s in sims:
            s.close()


def test_zero_conductivity_equals_lossless_and_back():
    w = wl.small_case((20, 21, 22), (PEC, PEC, PEC), seed=10, nsteps=25, dipoles=[(10, 10, 10)])
    zero = [np.zeros(w.shape, np.float32)] * 3
    sim = _sim(w, zero)
    sim.step(25)
    assert_bitwise(sim.read_fields(), oracle_f32(w, 25), "sigma = 0")
    # a lossless set_materials makes it lossless (and systolic-capable) again
    sim.set_materials(w.eps)
    sim.set_fields(w.fields)
    sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_SYSTOLIC)
    sim.step(25)
    ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 25, step0=25, sources=w.sources,
                     dtype=np.float32)
    assert_bitwise(sim.read_fields(), ref, "lossless again")
    # and conductive again on the systolic scheme: the launch plan follows
    # the narrower conductive tile
    sig = _sigma(w.shape, 13)
    sim.set_materials(w.eps, sigma=sig)
    sim.step(10)
    assert sim.info(fdtd.INFO_TILE_X) == 11
    ref2 = oracle.run(ref, w.eps3(), w.bc, w.dt, w.dx, 10, step0=50, sources=w.sources,
                      dtype=np.float32, sigma=sig)
    assert_bitwise(sim.read_fields(), ref2, "conductive systolic after lossless")
    sim.close()


def test_negative_conductivity_is_refused():
    w = wl.small_case((20, 20, 20), (PEC, PEC, PEC), seed=11, nsteps=4)
    sig = _sigma(w.shape, 12)
    sim = _sim(w, sig)
    with pytest.raises(fdtd.FdtdError) as e:
        sim.set_materials(w.eps, sigma=[-s for s in sig])
    assert e.value.code == fdtd.FDTD_EINVAL
    sim.close()
