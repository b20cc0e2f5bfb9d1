"""GPU FP64 reductions of the discrete invariants (fdtd_invariants).

* The device sums and per-cell divergences equal the same quantities computed
  by the test's own numpy/scipy mathematics (tests/yee_math.py) on the
  oracle's state, to 1e-12 relative, for every boundary mix, with
  conductivity, and with FP16 storage (decoded values).
* On lossless GPU runs without sources the leapfrog energy is conserved and
  the per-cell divergences stay put, to FP32 roundoff (the oracle's own FP32
  drift over 200 steps is ~5e-9 for the energy and ~1e-6 of the largest
  divergence); with conductivity the energy decays monotonically.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym

pytestmark = pytest.mark.gpu

BCS = [(0, 0, 0), (1, 1, 0), (1, 1, 1), (0, 1, 0)]


def _eps_eff(coef64, cH):
    """Permittivity the coefficients encode (cH / cE), 0 where cE = 0."""
    return [np.where(c > 0, float(cH) / np.where(c > 0, c, 1.0), 0.0) for c in coef64]


def _expected(fields, eps, bc, cH):
    f = [np.asarray(a, np.float64) for a in fields]
    Q = ym.leapfrog_energy(f, eps, bc, float(cH), 1.0)
    live = [~wl.pec_tangential_mask(f[0].shape, bc, c) for c in range(3)]
    ee = sum(float(np.sum(eps[c][live[c]] * f[c][live[c]] ** 2)) for c in range(3))
    hh = sum(float(np.sum(f[3 + c] ** 2)) for c in range(3))
    inner = ym.interior_mask(f[0].shape, bc)
    de = ym.div_back([np.where(live[c], eps[c] * f[c], 0.0) for c in range(3)]) * inner
    dh = ym.div_fwd(f[3:])
    sums = {"energy": Q, "e_energy": ee, "h_energy": hh,
            "div_e_l1": float(np.abs(de).sum()), "div_e_l2sq": float((de ** 2).sum()),
            "div_h_l1": float(np.abs(dh).sum()), "div_h_l2sq": float((dh ** 2).sum())}
    return sums, de, dh


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


def _sim(w, scheme="systolic", storage="fp32", sigma=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, storage=storage)
    if sigma is None:
        sim.set_materials(w.eps)
    else:
        sim.set_materials(w.eps, sigma=sigma)
    return sim


@pytest.mark.parametrize("bc", BCS)
def test_invariants_match_numpy_on_oracle_state(bc):
    w = wl.small_case((20, 18, 22), bc, seed=41 + bc[0] + 2 * bc[1], nsteps=9, dipoles=[(9, 8, 11)])
    ref = oracle.run(w.fields, w.eps3(), bc, w.dt, w.dx, w.nsteps, sources=w.sources, dtype=np.float32)
    cE = [oracle.round_f32(c).astype(np.float64) for c in oracle.coeff_E(w.eps3(), bc, w.dt, w.dx)]
    eps = _eps_eff(cE, np.float32(w.dt / w.dx))
    with _sim(w) as sim:
        sim.set_fields(ref)
        got, de, dh = sim.invariants(per_cell=True)
    want, de_w, dh_w = _expected(ref, eps, bc, np.float32(w.dt / w.dx))
    for k in fdtd.INVARIANT_NAMES:
        assert _close(got[k], want[k]), (k, got[k], want[k])
    scale_e, scale_h = np.abs(de_w).max(), np.abs(dh_w).max()
    assert np.abs(de - de_w).max() <= 1e-12 * scale_e
    assert np.abs(dh - dh_w).max() <= 1e-12 * scale_h


def test_invariants_are_deterministic_and_device_outputs_agree():
    import torch
    w = wl.small_case((33, 17, 40), (0, 0, 0), seed=5, nsteps=1)
    with _sim(w) as sim:
        sim.set_fields(w.fields)
        a = sim.invariants()
        b = sim.invariants()
        dev = torch.device("cuda:0")
        out = (torch.zeros(7, dtype=torch.float64, device=dev),
               torch.zeros(w.shape, dtype=torch.float64, device=dev),
               torch.zeros(w.shape, dtype=torch.float64, device=dev))
        sim.invariants(device_out=out)
        sim.synchronize()
        _, de, dh = sim.invariants(per_cell=True)
    assert a == b
    assert [a[k] for k in fdtd.INVARIANT_NAMES] == out[0].cpu().tolist()
    assert np.array_equal(out[1].cpu().numpy(), de)
    assert np.array_equal(out[2].cpu().numpy(), dh)


@pytest.mark.parametrize("scheme", ["systolic", "plain"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_energy_and_divergence_conserved_on_gpu_runs(scheme, bc):
    """Source-free lossless runs: Q and the per-cell divergences stay constant
    to FP32 roundoff over 200 steps, and the GPU state after the run gives the
    same invariants as the oracle's state after the same run."""
    w = wl.small_case((40, 36, 34), bc, seed=17, nsteps=200)
    with _sim(w, scheme) as sim:
        sim.set_fields(w.fields)
        q0, de0, dh0 = sim.invariants(per_cell=True)
        sim.step(120)
        sim.step(80)
        q1, de1, dh1 = sim.invariants(per_cell=True)
    assert abs(q1["energy"] - q0["energy"]) <= 1e-7 * q0["energy"]
    assert np.abs(de1 - de0).max() <= 1e-5 * np.abs(de0).max()
    assert np.abs(dh1 - dh0).max() <= 1e-5 * np.abs(dh0).max()
    # the plain Sum(eps E^2 + H^2) is not an invariant: it moves far more
    assert abs((q1["e_energy"] + q1["h_energy"]) - (q0["e_energy"] + q0["h_energy"])) > \
        100 * abs(q1["energy"] - q0["energy"])
    ref = oracle.run(w.fields, w.eps3(), bc, w.dt, w.dx, 200, dtype=np.float32)
    cE = [oracle.round_f32(c).astype(np.float64) for c in oracle.coeff_E(w.eps3(), bc, w.dt, w.dx)]
    want, _, _ = _expected(ref, _eps_eff(cE, np.float32(0.5)), bc, np.float32(0.5))
    assert _close(q1["energy"], want["energy"])


def test_conductive_energy_decays_and_matches_numpy():
    bc = (0, 0, 0)
    w = wl.small_case((32, 30, 28), bc, seed=23, nsteps=60)
    sigma = wl.graded_shell(w.shape, 6, 0.3)
    with _sim(w, "systolic", sigma=sigma) as sim:
        sim.set_fields(w.fields)
        qs = [sim.invariants()["energy"]]
        for _ in range(6):
            sim.step(10)
            qs.append(sim.invariants()["energy"])
        state = sim.read_fields()
    assert all(b < a for a, b in zip(qs, qs[1:])), qs
    ca, cb = oracle.coeff_lossy(w.eps3(), [sigma] * 3, bc, w.dt, w.dx)
    ca32 = [oracle.round_f32(c).astype(np.float64) for c in ca]
    cb32 = [oracle.round_f32(c).astype(np.float64) for c in cb]
    cH = float(np.float32(0.5))
    eps = [np.where(b > 0, cH * (1.0 + a) / (2.0 * np.where(b > 0, b, 1.0)), 0.0) for a, b in zip(ca32, cb32)]
    want, _, _ = _expected(state, eps, bc, cH)
    assert _close(qs[-1], want["energy"])


def test_fp16_storage_invariants_use_decoded_values():
    bc = (1, 1, 0)
    w = wl.small_case((24, 20, 26), bc, seed=29, nsteps=30)
    with _sim(w, "systolic", storage="fp16") as sim:
        sim.set_field_scale([-3] * 6)
        sim.set_fields(w.fields)
        sim.step(30)
        got, de, dh = sim.invariants(per_cell=True)
        state = sim.read_fields()
    cE = [oracle.round_f32(c).astype(np.float16).astype(np.float64)
          for c in oracle.coeff_E(w.eps3(), bc, w.dt, w.dx)]
    want, de_w, dh_w = _expected(state, _eps_eff(cE, np.float32(0.5)), bc, np.float32(0.5))
    for k in fdtd.INVARIANT_NAMES:
        assert _close(got[k], want[k]), (k, got[k], want[k])
    assert np.abs(de - de_w).max() <= 1e-12 * np.abs(de_w).max()


def test_invariants_reject_bad_arguments():
    import ctypes
    lib = fdtd.load_library()
    w = wl.small_case((8, 8, 8), (0, 0, 0), seed=1, nsteps=1)
    with _sim(w) as sim:
        assert lib.fdtd_invariants(sim._h, None, None, None, fdtd.HOST) == fdtd.FDTD_EINVAL
        sums = (ctypes.c_double * 7)()
        assert lib.fdtd_invariants(sim._h, sums, None, None, 5) == fdtd.FDTD_EINVAL
        assert lib.fdtd_invariants(sim._h, sums, None, None, fdtd.HOST) == fdtd.FDTD_OK
