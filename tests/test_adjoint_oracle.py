"""Pins of the adjoint oracle (oracle/adjoint.py), on the CPU.

- The reverse step is the transpose of the forward step: <M x, y> = <x, M^T y>
  for random x, y, with M the C oracle's FP64 step (independent code) on PEC,
  periodic and mixed grids.
- The adjoint gradient of the monitor objective equals central finite
  differences of the FP64 forward objective, per component, at cells inside,
  on the edge of and next to the design box.
- The objective is the squared transform of the sampled field: for a single
  recorded sample it reduces to a closed form.
- The same three pins for the conductive step: its reverse step is the
  transpose of the C oracle's FP64 conductive step, its gradient (sigma held
  fixed) equals central finite differences, and sigma = 0 gives the lossless
  gradient.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from paper_2502_20610_amd import workloads as wl

PEC, PER = 0, 1


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PER), (PER, PEC, PER)])
def test_reverse_step_is_the_transpose(bc):
    rng = np.random.default_rng(1)
    shape = (8, 7, 9)
    eps = [rng.uniform(1.0, 12.25, shape).astype(np.float32) for _ in range(3)]
    cE = oracle.coeff_E(eps, bc, 0.5, 1.0)
    for trial in range(3):
        x = [rng.standard_normal(shape) for _ in range(6)]
        y = [rng.standard_normal(shape) for _ in range(6)]
        Mx = oracle.step(cE, 0.5, tuple(np.array(a) for a in x), 1, dtype=np.float64)
        lE, lH = adj.adjoint_step(tuple(y[:3]), tuple(y[3:]), cE, 0.5)
        a = sum(float(np.sum(m * b)) for m, b in zip(Mx, y))
        b = sum(float(np.sum(p * q)) for p, q in zip(x, list(lE) + list(lH)))
        assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), (a, b)


def _fd(w, eps3, c, cell, h, spec):
    """Central difference of J in eps_c at one cell (FP64 forward)."""
    def J(d):
        e2 = [np.array(e, np.float64) for e in eps3]
        e2[c][cell] += d
        base = oracle.coeff_E(eps3, w.bc, w.dt, w.dx)
        cE = tuple(np.where(b0 == 0.0, 0.0, w.dt / (e * w.dx)) for b0, e in zip(base, e2))
        F, _, _ = adj.forward_dft(w.fields, cE, w.dt / w.dx, spec["n"], spec["mon_lo"],
                                  spec["mon_hi"], spec["comp"], spec["omega"], w.dt,
                                  sources=w.sources)
        return float(np.sum(np.abs(F) ** 2))
    return (J(h) - J(-h)) / (2 * h)


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PEC, PER)])
def test_gradient_matches_finite_differences(bc):
    w = wl.small_case((12, 11, 10), bc, seed=3, nsteps=60, dipoles=[(3, 4, 5)])
    eps3 = [np.array(w.eps) for _ in range(3)]
    spec = dict(n=60, mon_lo=(7, 2, 2), mon_hi=(8, 9, 8), comp=2, omega=0.4)
    des_lo, des_hi = (3, 3, 3), (6, 6, 6)
    J, g = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, 60, spec["mon_lo"], spec["mon_hi"],
                        2, 0.4, des_lo, des_hi, sources=w.sources)
    assert J > 0
    for c, cell in [(2, (4, 4, 4)), (0, (5, 3, 4)), (1, (3, 5, 5)), (2, (5, 5, 3))]:
        fd = _fd(w, eps3, c, cell, 1e-4, spec)
        got = g[c][tuple(p - l for p, l in zip(cell, des_lo))]
        assert abs(got - fd) <= 1e-6 * abs(fd) + 1e-12, (c, cell, got, fd)


def test_gradient_is_zero_on_pec_tangential_entries():
    w = wl.small_case((10, 9, 8), (PEC, PEC, PEC), seed=4, nsteps=20, dipoles=[(4, 4, 4)])
    eps3 = [np.array(w.eps) for _ in range(3)]
    J, g = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, 20, (5, 1, 1), (6, 8, 7), 2, 0.5,
                        (0, 0, 0), (3, 3, 3), sources=w.sources)
    # Ey and Ez are tangential to the x = 0 wall: their cE is pinned at 0 there
    assert np.all(g[1][0] == 0) and np.all(g[2][0] == 0)
    assert np.any(g[0][0] != 0)


def test_objective_single_sample_closed_form():
    """With one step, F = E_c^1 exp(-i w dt), so J = sum (E_c^1)^2 over the box."""
    w = wl.small_case((9, 8, 7), (PEC, PEC, PEC), seed=5, nsteps=1)
    eps3 = [np.array(w.eps) for _ in range(3)]
    J = adj.objective(w.fields, eps3, w.bc, w.dt, w.dx, 1, (2, 2, 2), (5, 6, 4), 2, 0.7)
    f = oracle.run(w.fields, eps3, w.bc, w.dt, w.dx, 1, dtype=np.float64)
    assert J == pytest.approx(float(np.sum(f[2][2:5, 2:6, 2:4] ** 2)), rel=1e-12)


def _sigma(shape, seed, hi=0.3):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.0, hi, shape).astype(np.float32) for _ in range(3)]


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PER), (PER, PEC, PER)])
def test_conductive_reverse_step_is_the_transpose(bc):
    rng = np.random.default_rng(6)
    shape = (7, 9, 8)
    eps = [rng.uniform(1.0, 12.25, shape).astype(np.float32) for _ in range(3)]
    ca, cb = oracle.coeff_lossy(eps, _sigma(shape, 7, 0.8), bc, 0.5, 1.0)
    assert all(np.any((a != 1.0) & (b != 0.0)) for a, b in zip(ca, cb))
    for trial in range(3):
        x = [rng.standard_normal(shape) for _ in range(6)]
        y = [rng.standard_normal(shape) for _ in range(6)]
        Mx = oracle.step_lossy(ca, cb, 0.5, tuple(np.array(a) for a in x), 1, dtype=np.float64)
        lE, lH = adj.adjoint_step_lossy(tuple(y[:3]), tuple(y[3:]), ca, cb, 0.5)
        a = sum(float(np.sum(m * b)) for m, b in zip(Mx, y))
        b = sum(float(np.sum(p * q)) for p, q in zip(x, list(lE) + list(lH)))
        assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), (a, b)


def _fd_lossy(w, eps3, sig, c, cell, h, spec):
    """Central difference of the conductive J in eps_c at one cell, sigma fixed:
    the coefficients are rebuilt in FP64 from the perturbed permittivity."""
    _, base = oracle.coeff_lossy(eps3, sig, w.bc, w.dt, w.dx)

    def J(d):
        ca, cb = [], []
        for q in range(3):
            e = np.asarray(eps3[q], np.float32).astype(np.float64)
            if q == c:
                e[cell] += d
            hh = np.asarray(sig[q], np.float32).astype(np.float64) * w.dt / (2.0 * e)
            pinned = base[q] == 0.0
            ca.append(np.where(pinned, 1.0, (1.0 - hh) / (1.0 + hh)))
            cb.append(np.where(pinned, 0.0, (w.dt / (e * w.dx)) / (1.0 + hh)))
        F, _, _ = adj.forward_dft(w.fields, tuple(cb), w.dt / w.dx, spec["n"], spec["mon_lo"],
                                  spec["mon_hi"], spec["comp"], spec["omega"], w.dt,
                                  sources=w.sources, ca=tuple(ca))
        return float(np.sum(np.abs(F) ** 2))
    return (J(h) - J(-h)) / (2 * h)


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PEC, PER)])
def test_conductive_gradient_matches_finite_differences(bc):
    w = wl.small_case((12, 11, 10), bc, seed=13, nsteps=60, dipoles=[(3, 4, 5)])
    eps3 = [np.array(w.eps) for _ in range(3)]
    sig = _sigma(w.shape, 14)
    spec = dict(n=60, mon_lo=(7, 2, 2), mon_hi=(8, 9, 8), comp=2, omega=0.4)
    des_lo, des_hi = (3, 3, 3), (6, 6, 6)
    J, g = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, 60, spec["mon_lo"], spec["mon_hi"],
                        2, 0.4, des_lo, des_hi, sources=w.sources, sigma=sig)
    J0 = adj.objective(w.fields, eps3, w.bc, w.dt, w.dx, 60, spec["mon_lo"], spec["mon_hi"],
                       2, 0.4, sources=w.sources)
    assert J > 0 and abs(J - J0) > 1e-2 * J0   # the conductivity changes the objective
    for c, cell in [(2, (4, 4, 4)), (0, (5, 3, 4)), (1, (3, 5, 5)), (2, (5, 5, 3))]:
        fd = _fd_lossy(w, eps3, sig, c, cell, 1e-4, spec)
        got = g[c][tuple(p - l for p, l in zip(cell, des_lo))]
        assert abs(got - fd) <= 1e-6 * abs(fd) + 1e-12, (c, cell, got, fd)


def test_conductive_gradient_with_zero_sigma_is_the_lossless_one():
    w = wl.small_case((10, 9, 8), (PEC, PER, PEC), seed=15, nsteps=30, dipoles=[(4, 4, 4)])
    eps3 = [np.array(w.eps) for _ in range(3)]
    zero = [np.zeros(w.shape, np.float32)] * 3
    args = (w.fields, eps3, w.bc, w.dt, w.dx, 30, (6, 1, 1), (7, 8, 7), 1, 0.5, (1, 2, 2), (5, 6, 5))
    J0, g0 = adj.gradient(*args, sources=w.sources)
    J1, g1 = adj.gradient(*args, sources=w.sources, sigma=zero)
    assert J1 == pytest.approx(J0, rel=1e-14)
    for a, b in zip(g0, g1):
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-14 * np.max(np.abs(a)))
