"""Pins of the conductive (lossy) oracle step, on the CPU.

- sigma = 0 reduces it to the lossless step bit for bit (FP32 and FP64, with
  sources): ca = 1 and cb = cE exactly.
- The semi-implicit conductivity term obeys an exact discrete energy balance:
  with Q the leapfrog energy of the lossless pins,
  Q^{n+1} - Q^n = -(dt/2) sum sigma (E^{n+1} + E^n)^2 over the live entries.
- A spatially uniform E field in a uniform periodic medium has no curl, so it
  decays by ca = (1 - h)/(1 + h), h = sigma dt / (2 eps), per step, and H stays 0.
- PEC-tangential entries stay +0.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym

PEC, PER = 0, 1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_zero_conductivity_is_the_lossless_step(dtype):
    w = wl.small_case((12, 11, 10), (PEC, PER, PEC), seed=2, nsteps=30, dipoles=[(5, 5, 5)])
    zero = [np.zeros(w.shape, np.float32)] * 3
    a = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 30, sources=w.sources, dtype=dtype)
    b = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 30, sources=w.sources, dtype=dtype,
                   sigma=zero)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PER), (PER, PEC, PER)])
def test_discrete_energy_balance(bc):
    w = wl.small_case((9, 8, 7), bc, seed=3, nsteps=1)
    rng = np.random.default_rng(4)
    sig = [rng.uniform(0.0, 0.2, w.shape).astype(np.float32) for _ in range(3)]
    ca, cb = oracle.coeff_lossy(w.eps3(), sig, w.bc, w.dt, w.dx)
    f = tuple(np.array(x, np.float64) for x in w.fields)
    live = ~ym.pec_frozen_mask(w.shape, w.bc).reshape(3, *w.shape)
    for _ in range(5):
        q0 = ym.leapfrog_energy(f, w.eps3(), w.bc, w.dt)
        e0 = [x.copy() for x in f[:3]]
        oracle.step_lossy(ca, cb, w.dt / w.dx, f, 1, dtype=np.float64)
        q1 = ym.leapfrog_energy(f, w.eps3(), w.bc, w.dt)
        loss = sum(float(np.sum((np.asarray(sig[c], np.float64) * (f[c] + e0[c]) ** 2)[live[c]]))
                   for c in range(3))
        assert q1 - q0 == pytest.approx(-0.5 * w.dt * loss, rel=1e-12, abs=1e-14)
        assert q1 < q0


def test_uniform_field_decays_by_ca():
    shape = (6, 5, 7)
    eps, sigma, dt = 2.5, 0.3, 0.5
    e3 = [np.full(shape, eps, np.float32)] * 3
    s3 = [np.full(shape, sigma, np.float32)] * 3
    f = [np.full(shape, v) for v in (1.0, -2.0, 0.5)] + [np.zeros(shape) for _ in range(3)]
    out = oracle.run(f, e3, (PER, PER, PER), dt, 1.0, 12, dtype=np.float64, sigma=s3)
    h = float(np.float32(sigma)) * dt / (2 * float(np.float32(eps)))
    ca = (1 - h) / (1 + h)
    for c, v in enumerate((1.0, -2.0, 0.5)):
        np.testing.assert_allclose(out[c], v * ca ** 12, rtol=1e-13)
    for c in range(3, 6):
        assert np.all(out[c] == 0)


def test_pec_entries_stay_zero_with_conductivity():
    w = wl.small_case((8, 9, 10), (PEC, PEC, PEC), seed=5, nsteps=20, dipoles=[(4, 4, 4)])
    sig = [np.full(w.shape, 0.1, np.float32)] * 3
    out = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 20, sources=w.sources,
                     dtype=np.float32, sigma=sig)
    frozen = ym.pec_frozen_mask(w.shape, w.bc).reshape(3, *w.shape)
    for c in range(3):
        vals = out[c][frozen[c]]
        assert np.all(vals.view(np.uint32) == 0)
