"""GPU parity of conductive (lossy) materials: the plain scheme's conductive
E half-step against the FP32 lossy oracle, bit for bit; sigma = 0 through
the lossy entry point equals the lossless path; the schemes and calls that
do not cover conductivity refuse it."""
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


def _sim(w, sig, device=False):
    import torch
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
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
    ref0 = oracle_f32(w, 300)
    e_lossy = sum(float(np.sum(np.asarray(f, np.float64) ** 2)) for f in got)
    e_lossless = sum(float(np.sum(np.asarray(f, np.float64) ** 2)) for f in ref0)
    assert e_lossy < 0.5 * e_lossless


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
    sim.close()


def test_conductivity_is_refused_where_not_covered():
    w = wl.small_case((20, 20, 20), (PEC, PEC, PEC), seed=11, nsteps=4)
    sig = _sigma(w.shape, 12)
    sim = _sim(w, sig)
    sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_SYSTOLIC)
    with pytest.raises(fdtd.FdtdError) as e:
        sim.step(2)
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    with pytest.raises(fdtd.FdtdError) as e:
        fdtd.step_batch([sim], 2)
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    with pytest.raises(fdtd.FdtdError) as e:
        sim.adjoint(2, 2, (10, 1, 1), (11, 9, 9), 0.5, (2, 2, 2), (5, 5, 5))
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    assert sim.current_step == 0
    with pytest.raises(fdtd.FdtdError) as e:
        sim.set_materials(w.eps, sigma=[-s for s in sig])
    assert e.value.code == fdtd.FDTD_EINVAL
    sim.close()
