"""GPU adjoint (fdtd_adjoint) against the FP64 adjoint oracle and finite differences.

The GPU run is FP32 (fields, adjoint fields) with FP64 monitor transform and
gradient sums; the oracle is FP64 throughout.  Checks:
- J within 1e-5 and the design-box gradient within 1e-4 (relative L2) of the
  oracle's, with checkpoint intervals that do and do not divide the run;
- per-cell gradients within 1e-3 of central finite differences of the FP64
  objective (the inverse-design accuracy bar), at cells chosen from the
  oracle's gradient;
- the context holds the forward run's final state afterwards (bitwise equal
  to a plain run) and the device-output path equals the host-output path;
- invalid specifications are refused without changing the context;
- the same bars with conductive materials (sigma held fixed): random
  conductivity, a small conductivity that stresses the (1 - ca) factor, and
  an absorbing shell around a dielectric design block.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def _sim(w, scheme="plain"):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme)
    sim.set_materials(w.eps)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _fd(w, c, cell, spec, h=1e-4):
    eps3 = [np.array(w.eps) for _ in range(3)]
    base = oracle.coeff_E(eps3, w.bc, w.dt, w.dx)

    def J(d):
        e2 = [np.array(e, np.float64) for e in eps3]
        e2[c][cell] += d
        cE = tuple(np.where(b0 == 0.0, 0.0, w.dt / (e * w.dx)) for b0, e in zip(base, e2))
        F, _, _ = adj.forward_dft(w.fields_or_zeros(), cE, w.dt / w.dx, spec["n"], spec["mon_lo"],
                                  spec["mon_hi"], spec["comp"], spec["omega"], w.dt,
                                  sources=w.sources)
        return float(np.sum(np.abs(F) ** 2))
    return (J(h) - J(-h)) / (2 * h)


CASES = [
    ("pec", (14, 12, 10), (PEC, PEC, PEC), 80, 25, (4, 3, 3), (8, 7, 6), (10, 1, 1), (11, 11, 9)),
    ("mixed", (12, 13, 11), (PER, PEC, PER), 70, 70, (0, 4, 8), (5, 8, 11), (7, 2, 0), (8, 12, 11)),
    ("ckpt1", (10, 9, 8), (PEC, PEC, PEC), 17, 1, (2, 2, 2), (5, 5, 5), (7, 1, 1), (8, 8, 7)),
]


@pytest.mark.parametrize("name,shape,bc,n,ck,dlo,dhi,mlo,mhi", CASES)
def test_adjoint_matches_oracle(name, shape, bc, n, ck, dlo, dhi, mlo, mhi):
    w = wl.small_case(shape, bc, seed=len(name), nsteps=n, dipoles=[(3, 4, 5)])
    eps3 = [np.array(w.eps) for _ in range(3)]
    J_ref, g_ref = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, n, mlo, mhi, 2, 0.4, dlo, dhi,
                                sources=w.sources)
    sim = _sim(w)
    J, g = sim.adjoint(n, 2, mlo, mhi, 0.4, dlo, dhi, checkpoint_every=ck)
    assert sim.current_step == n
    # the context holds the forward run's final state
    assert_bitwise(sim.read_fields(), oracle_f32(w, n), "state after adjoint")
    sim.close()
    assert abs(J - J_ref) <= 1e-5 * J_ref, (J, J_ref)
    assert _rel(g, np.stack(g_ref)) < 1e-4


def test_adjoint_gradient_matches_finite_differences():
    """A scaled-down inverse-design setup: 64x64x32 PEC box with a dielectric
    design block between a dipole and a monitor plane, 600 steps,
    checkpoints every 200; eight cells checked against FP64 central
    differences."""
    shape = (64, 64, 32)
    w = wl.random_dielectric(shape, (PEC, PEC, PEC), 6, 51, 600, side=(4, 16),
                             dipoles=[(16, 32, 16)])
    dlo, dhi = (24, 24, 14), (40, 40, 18)
    rng = np.random.default_rng(52)
    eps = np.array(w.eps)
    eps[24:40, 24:40, 14:18] = rng.uniform(2.08, 12.25, (16, 16, 4)).astype(np.float32)
    w.eps = eps
    spec = dict(n=600, mon_lo=(48, 24, 8), mon_hi=(49, 40, 24), comp=2, omega=0.36305)
    eps3 = [np.array(w.eps) for _ in range(3)]
    J_ref, g_ref = adj.gradient(w.fields_or_zeros(), eps3, w.bc, w.dt, w.dx, 600, spec["mon_lo"],
                                spec["mon_hi"], 2, spec["omega"], dlo, dhi, sources=w.sources)
    sim = _sim(w)
    J, g = sim.adjoint(600, 2, spec["mon_lo"], spec["mon_hi"], spec["omega"], dlo, dhi,
                       checkpoint_every=200)
    sim.close()
    assert abs(J - J_ref) <= 1e-5 * J_ref
    gr = np.stack(g_ref)
    big = np.argwhere(np.abs(gr) > 1e-2 * np.abs(gr).max())
    pick = big[rng.choice(len(big), 8, replace=False)]
    for c, a, b, k in pick:
        cell = (dlo[0] + a, dlo[1] + b, dlo[2] + k)
        fd = _fd(w, int(c), cell, spec)
        assert abs(g[c, a, b, k] - fd) <= 1e-3 * abs(fd), (c, cell, g[c, a, b, k], fd)


def test_adjoint_device_output_equals_host_output():
    import torch
    w = wl.small_case((12, 10, 9), (PEC, PEC, PEC), seed=9, nsteps=30, dipoles=[(4, 4, 4)])
    args = (30, 2, (8, 1, 1), (9, 9, 8), 0.5, (2, 2, 2), (6, 5, 6))
    sim = _sim(w)
    J1, g1 = sim.adjoint(*args, checkpoint_every=7)
    sim.close()
    sim = _sim(w)
    out = torch.empty((3, 4, 3, 4), dtype=torch.float32, device="cuda:0")
    J2, g2 = sim.adjoint(*args, checkpoint_every=7, out=out)
    sim.close()
    assert J1 == J2
    np.testing.assert_array_equal(g1, g2.cpu().numpy())


@pytest.mark.parametrize("bad", [
    dict(mon_comp=3), dict(mon_lo=(0, 0, 0), mon_hi=(0, 5, 5)), dict(des_hi=(13, 5, 5)),
    dict(nsteps=0), dict(checkpoint_every=-2), dict(isotropic=2),
])
def test_adjoint_rejects_bad_spec(bad):
    w = wl.small_case((12, 10, 9), (PEC, PEC, PEC), seed=9, nsteps=5)
    kw = dict(nsteps=5, mon_comp=2, mon_lo=(8, 1, 1), mon_hi=(9, 9, 8), omega=0.5,
              des_lo=(2, 2, 2), des_hi=(6, 5, 6), checkpoint_every=0)
    kw.update(bad)
    sim = _sim(w)
    with pytest.raises(fdtd.FdtdError) as e:
        sim.adjoint(**kw)
    assert e.value.code == fdtd.FDTD_EINVAL
    assert sim.current_step == 0
    assert_bitwise(sim.read_fields(), w.fields, "unchanged state")
    sim.close()


@pytest.mark.parametrize("lossy", [False, True])
def test_isotropic_gradient_is_the_component_sum(lossy):
    """spec.isotropic = 1 returns one block: the three components' derivatives
    added in FP64 by the library (the design variable of a cell whose single
    permittivity drives all three components), equal to the oracle's sum."""
    w = wl.small_case((14, 12, 10), (PEC, PER, PEC), seed=31, nsteps=40, dipoles=[(3, 4, 5)])
    sigma = wl.graded_shell(w.shape, 3, 0.3) if lossy else None
    args = dict(nsteps=40, mon_comp=2, mon_lo=(11, 1, 1), mon_hi=(12, 11, 9), omega=0.4,
                des_lo=(4, 3, 3), des_hi=(9, 8, 7), checkpoint_every=15)
    res = {}
    for iso in (False, True):
        sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc)
        sim.set_materials(w.eps, sigma=sigma)
        sim.set_fields(w.fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        res[iso] = sim.adjoint(**args, isotropic=iso)
        sim.close()
    (J3, g3), (J1, g1) = res[False], res[True]
    assert J1 == J3
    assert g1.shape == g3.shape[1:]
    s3 = g3.astype(np.float64).sum(axis=0)
    assert np.abs(g1 - s3).max() <= 4e-7 * np.abs(s3).max()
    eps3 = [np.array(w.eps) for _ in range(3)]
    _, g_ref = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, 40, args["mon_lo"], args["mon_hi"], 2,
                            0.4, args["des_lo"], args["des_hi"], sources=w.sources,
                            sigma=None if sigma is None else [sigma] * 3)
    assert _rel(g1, np.sum(np.stack(g_ref), axis=0)) < 1e-4


def test_design_objective_autograd():
    """torch.autograd through design_objective returns the adjoint gradient
    summed over the three components, and matches a finite difference of the
    objective in the isotropic design variable."""
    import torch
    w = wl.small_case((16, 14, 12), (PEC, PEC, PEC), seed=21, nsteps=60, dipoles=[(3, 7, 6)])
    args = dict(nsteps=60, mon_comp=2, mon_lo=(12, 2, 2), mon_hi=(13, 12, 10), omega=0.4,
                des_lo=(6, 4, 4), des_hi=(10, 9, 8), checkpoint_every=20)
    prob = fdtd.DesignProblem(w.eps, w.bc, w.dt, w.dx, w.sources, args)
    x0 = np.array(w.eps[6:10, 4:9, 4:8])
    x = torch.tensor(x0, dtype=torch.float32, requires_grad=True)
    J = fdtd.design_objective(x, prob)
    J.backward()
    J_ref, g_ref = prob.evaluate(x0)
    assert float(J.detach()) == J_ref
    np.testing.assert_allclose(x.grad.numpy(), g_ref, rtol=1e-6)
    # isotropic finite difference (FP64 oracle) at one cell
    eps3 = [np.array(w.eps) for _ in range(3)]
    cell = (8, 6, 5)
    base = oracle.coeff_E(eps3, w.bc, w.dt, w.dx)

    def Jfd(d):
        e = np.array(w.eps, np.float64)
        e[cell] += d
        cE = tuple(np.where(b0 == 0.0, 0.0, w.dt / (e * w.dx)) for b0 in base)
        F, _, _ = adj.forward_dft(w.fields_or_zeros(), cE, w.dt / w.dx, 60, args["mon_lo"],
                                  args["mon_hi"], 2, 0.4, w.dt, sources=w.sources)
        return float(np.sum(np.abs(F) ** 2))
    w.fields = None
    fd = (Jfd(1e-4) - Jfd(-1e-4)) / 2e-4
    got = x.grad.numpy()[cell[0] - 6, cell[1] - 4, cell[2] - 4]
    assert abs(got - fd) <= 1e-3 * abs(fd), (got, fd)


# ---- conductive materials (sigma held fixed, gradient in eps) -------------

def _sigma(shape, seed, lo=0.0, hi=0.3):
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo, hi, shape).astype(np.float32) for _ in range(3)]


def _sim_lossy(w, sig):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    sim.set_materials(w.eps, sigma=sig)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


def _fd_lossy(w, sig, c, cell, spec, h=1e-4):
    """Central difference of the conductive FP64 objective in eps_c at one
    cell, sigma fixed (coefficients rebuilt in FP64 from the perturbed eps)."""
    eps3 = [np.array(w.eps) for _ in range(3)]
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
        F, _, _ = adj.forward_dft(w.fields_or_zeros(), tuple(cb), w.dt / w.dx, spec["n"],
                                  spec["mon_lo"], spec["mon_hi"], spec["comp"], spec["omega"],
                                  w.dt, sources=w.sources, ca=tuple(ca))
        return float(np.sum(np.abs(F) ** 2))
    return (J(h) - J(-h)) / (2 * h)


@pytest.mark.parametrize("name,shape,bc,n,ck,dlo,dhi,mlo,mhi", CASES)
def test_conductive_adjoint_matches_oracle(name, shape, bc, n, ck, dlo, dhi, mlo, mhi):
    w = wl.small_case(shape, bc, seed=len(name) + 40, nsteps=n, dipoles=[(3, 4, 5)])
    sig = _sigma(w.shape, len(name) + 41)
    eps3 = [np.array(w.eps) for _ in range(3)]
    J_ref, g_ref = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, n, mlo, mhi, 2, 0.4, dlo, dhi,
                                sources=w.sources, sigma=sig)
    sim = _sim_lossy(w, sig)
    J, g = sim.adjoint(n, 2, mlo, mhi, 0.4, dlo, dhi, checkpoint_every=ck)
    assert sim.current_step == n
    ref_state = oracle.run(w.fields, eps3, w.bc, w.dt, w.dx, n, sources=w.sources,
                           dtype=np.float32, sigma=sig)
    assert_bitwise(sim.read_fields(), ref_state, "state after conductive adjoint")
    sim.close()
    assert abs(J - J_ref) <= 1e-5 * J_ref, (J, J_ref)
    assert _rel(g, np.stack(g_ref)) < 1e-4


def test_conductive_adjoint_small_sigma():
    """sigma of order 1e-3 (ca within 1e-4 of 1): the (1 - ca) factor of the
    gradient is taken from the FP32 ca, which this case stresses."""
    w = wl.small_case((14, 12, 10), (PEC, PEC, PEC), seed=47, nsteps=80, dipoles=[(3, 4, 5)])
    sig = _sigma(w.shape, 48, 5e-4, 2e-3)
    eps3 = [np.array(w.eps) for _ in range(3)]
    args = (80, 2, (10, 1, 1), (11, 11, 9), 0.4, (4, 3, 3), (8, 7, 6))
    J_ref, g_ref = adj.gradient(w.fields, eps3, w.bc, w.dt, w.dx, 80, args[2], args[3], 2, 0.4,
                                args[5], args[6], sources=w.sources, sigma=sig)
    sim = _sim_lossy(w, sig)
    J, g = sim.adjoint(*args, checkpoint_every=30)
    sim.close()
    assert abs(J - J_ref) <= 1e-5 * J_ref, (J, J_ref)
    assert _rel(g, np.stack(g_ref)) < 1e-4


def test_conductive_adjoint_absorbing_shell_finite_differences():
    """A 48x48x32 PEC box lined with a graded conducting shell (6 cells,
    sigma up to 0.4), a dielectric design block between a dipole and a
    monitor plane, 400 steps: J and the gradient against the FP64 oracle,
    and eight cells against FP64 central differences within 1e-3."""
    shape = (48, 48, 32)
    w = wl.random_dielectric(shape, (PEC, PEC, PEC), 6, 61, 400, side=(4, 12),
                             dipoles=[(14, 24, 16)])
    dlo, dhi = (20, 18, 12), (30, 30, 20)
    rng = np.random.default_rng(62)
    eps = np.array(w.eps)
    eps[20:30, 18:30, 12:20] = rng.uniform(2.08, 12.25, (10, 12, 8)).astype(np.float32)
    w.eps = eps
    shell = wl.graded_shell(shape, thickness=6, sigma_max=0.4)
    # a weakly conducting design block too, so both sums of the gradient matter there
    shell[20:30, 18:30, 12:20] = rng.uniform(0.0, 0.05, (10, 12, 8)).astype(np.float32)
    sig = [shell] * 3
    spec = dict(n=400, mon_lo=(36, 16, 8), mon_hi=(37, 32, 24), comp=2, omega=0.36305)
    eps3 = [np.array(w.eps) for _ in range(3)]
    J_ref, g_ref = adj.gradient(w.fields_or_zeros(), eps3, w.bc, w.dt, w.dx, 400, spec["mon_lo"],
                                spec["mon_hi"], 2, spec["omega"], dlo, dhi, sources=w.sources,
                                sigma=sig)
    sim = _sim_lossy(w, sig)
    J, g = sim.adjoint(400, 2, spec["mon_lo"], spec["mon_hi"], spec["omega"], dlo, dhi,
                       checkpoint_every=150)
    sim.close()
    assert abs(J - J_ref) <= 1e-5 * J_ref
    gr = np.stack(g_ref)
    assert _rel(g, gr) < 1e-4
    big = np.argwhere(np.abs(gr) > 1e-2 * np.abs(gr).max())
    pick = big[rng.choice(len(big), 8, replace=False)]
    for c, a, b, k in pick:
        cell = (dlo[0] + a, dlo[1] + b, dlo[2] + k)
        fd = _fd_lossy(w, sig, int(c), cell, spec)
        assert abs(g[c, a, b, k] - fd) <= 1e-3 * abs(fd), (c, cell, g[c, a, b, k], fd)


def test_conductive_design_objective_autograd():
    import torch
    w = wl.small_case((16, 14, 12), (PEC, PEC, PEC), seed=23, nsteps=60, dipoles=[(3, 7, 6)])
    args = dict(nsteps=60, mon_comp=2, mon_lo=(12, 2, 2), mon_hi=(13, 12, 10), omega=0.4,
                des_lo=(6, 4, 4), des_hi=(10, 9, 8), checkpoint_every=20)
    sig = _sigma(w.shape, 24)[0]
    prob = fdtd.DesignProblem(w.eps, w.bc, w.dt, w.dx, w.sources, args, sigma=sig)
    x0 = np.array(w.eps[6:10, 4:9, 4:8])
    x = torch.tensor(x0, dtype=torch.float32, requires_grad=True)
    J = fdtd.design_objective(x, prob)
    J.backward()
    w.fields = None
    eps3 = [np.array(w.eps) for _ in range(3)]
    J_ref, g_ref = adj.gradient(w.fields_or_zeros(), eps3, w.bc, w.dt, w.dx, 60, args["mon_lo"],
                                args["mon_hi"], 2, 0.4, args["des_lo"], args["des_hi"],
                                sources=w.sources, sigma=[sig] * 3)
    assert abs(float(J.detach()) - J_ref) <= 1e-5 * J_ref
    assert _rel(x.grad.numpy(), np.stack(g_ref).sum(axis=0)) < 1e-4


@pytest.mark.parametrize("lossy", [False, True])
def test_segmenting_does_not_change_the_result(lossy):
    """One segment recorded during the forward run (automatic length), several
    checkpointed segments with a ragged last one, and one-step segments give
    bit-identical J and gradients; the sweep recomputes len - 1 steps of every
    segment but the last."""
    w = wl.small_case((12, 11, 10), (PEC, PER, PEC), seed=71, nsteps=30, dipoles=[(3, 4, 5)])
    sig = _sigma(w.shape, 72) if lossy else None
    args = (30, 1, (8, 1, 1), (9, 10, 9), 0.45, (2, 3, 2), (6, 8, 7))
    res = {}
    for ck, recomputed in [(0, 0), (30, 0), (7, 4 * 6), (1, 0), (13, 2 * 12)]:
        sim = _sim_lossy(w, sig) if lossy else _sim(w)
        res[ck] = sim.adjoint(*args, checkpoint_every=ck)
        assert sim.adjoint_recomputed_steps == recomputed, ck
        assert sim.current_step == 30
        if ck == 7:
            ref = oracle.run(w.fields, [w.eps] * 3, w.bc, w.dt, w.dx, 30, sources=w.sources,
                             dtype=np.float32, sigma=sig)
            assert_bitwise(sim.read_fields(), ref, "state after a segmented adjoint")
        sim.close()
    for ck in (30, 7, 1, 13):
        assert res[ck][0] == res[0][0]
        np.testing.assert_array_equal(res[ck][1], res[0][1])
