"""The inverse-design gradient at its full grid size, against FP64 finite differences.

Workload: 256x256x128 PEC box of eps 2.08 with a 64x64x16 design block of
per-cell eps ~ U[2.08, 12.25], an Ez dipole on its -x side and the objective
sum |DFT Ez|^2 at the source frequency over a 64x64 monitor plane, checkpoint
every 200 steps -- as the workload defines it, except that the run is 1000
steps instead of 4000 (by then the pulse has crossed the design block and the
monitor plane; sixteen FP64 runs of 4000 steps would take minutes).

The GPU gradient (FP32 fields, FP64 transform and sums) must agree with FP64
central differences at eight design cells within 1e-3 relative.  The
differences come from batched FP64 runs in plain torch (tests/torch_yee64.py),
which the first test pins to the C oracle bit for bit.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import torch_yee64 as ty

pytestmark = pytest.mark.gpu


def test_torch_fp64_forward_is_the_oracle():
    w = wl.small_case((12, 10, 9), (0, 0, 0), seed=12, nsteps=25, dipoles=[(4, 5, 3)])
    w.fields = None                                   # zero start, as forward_J assumes
    mon_lo, mon_hi, omega = (9, 1, 1), (10, 9, 8), 0.41
    eps = [np.asarray(w.eps, np.float64)] * 3
    J, f = ty.forward_J([eps], w.bc, w.dt, w.dx, 25, mon_lo, mon_hi, 2, omega, w.sources)
    ref = oracle.run(w.fields_or_zeros(), w.eps3(), w.bc, w.dt, w.dx, 25, sources=w.sources)
    for c in range(6):
        assert np.array_equal(f[c][0].cpu().numpy().view(np.uint64), ref[c].view(np.uint64)), c
    J_ref = adj.objective(w.fields_or_zeros(), w.eps3(), w.bc, w.dt, w.dx, 25, mon_lo, mon_hi, 2,
                          omega, sources=w.sources)
    assert abs(J[0] - J_ref) <= 1e-13 * J_ref


def test_full_size_gradient_matches_fp64_finite_differences():
    nsteps = 1000
    w, a = wl.c5_adjoint(nsteps=nsteps)
    a["checkpoint_every"] = 200
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    try:
        sim.set_materials(w.eps)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        J, g = sim.adjoint(**a)
        # the four earlier segments are recomputed from their checkpoints, each
        # up to the step before its last (whose history is all the sweep needs)
        assert sim.adjoint_recomputed_steps == (nsteps // 200 - 1) * (200 - 1)
    finally:
        sim.close()
    lo, hi = a["des_lo"], a["des_hi"]
    rng = np.random.default_rng(55)
    big = np.argwhere(np.abs(g) > 0.05 * np.abs(g).max())
    pick = big[rng.choice(len(big), 8, replace=False)]
    h = 1e-3
    base = np.asarray(w.eps, np.float64)
    runs = []
    for c, i, j, k in pick:
        for sgn in (1.0, -1.0):
            e3 = [base, base, base]
            e = base.copy()
            e[lo[0] + i, lo[1] + j, lo[2] + k] += sgn * h
            e3 = [e if q == c else base for q in range(3)]
            runs.append(e3)
    Js, _ = ty.forward_J(runs + [[base] * 3], w.bc, w.dt, w.dx, nsteps, a["mon_lo"], a["mon_hi"],
                         a["mon_comp"], a["omega"], w.sources)
    J64 = Js[-1]
    assert abs(J - J64) <= 1e-5 * J64, (J, J64)
    for q, (c, i, j, k) in enumerate(pick):
        fd = (Js[2 * q] - Js[2 * q + 1]) / (2 * h)
        assert abs(g[c, i, j, k] - fd) <= 1e-3 * abs(fd), ((c, i, j, k), g[c, i, j, k], fd)
