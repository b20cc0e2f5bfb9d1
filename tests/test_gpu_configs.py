"""Parity of the workload configurations at their stated sizes, every element.

* 256^3 with periodic x and y and PEC z (40 boxes of eps 12.25 in 2.08, a
  central Ez dipole): the systolic scheme on the 15-wide tile, whose ring
  groups are whole 18 x 18-tile z-layers with a ragged last tile (256 = 17 * 15 + 1), against
  the FP32 oracle after 128 steps -- the workload as defined (zero fields),
  and again from random fields so that every ring seam carries data from the
  first step.
  With the 19-wide tile too (ring groups of 14 x 18 tiles).
* The batched sweep: 64 PEC grids with axes drawn from {64, 80, ..., 192},
  each with its own permittivity map and dipole, in one persistent launch,
  every member against the FP32 oracle after 160 steps (the workload runs
  2000; 160 steps span several bands and every grid's tiles).
Results are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu


def _run(w, scheme, nsteps, opts=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme)
    try:
        for k, v in (opts or {}).items():
            sim.set_option(k, v)
        sim.set_materials(w.eps)
        if w.fields is not None:
            sim.set_fields(w.fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"], s.get("first_step", 0))
        sim.step(nsteps)
        out = sim.read_fields()
        info = (sim.info(fdtd.INFO_SYSTOLIC_BAND), sim.info(fdtd.INFO_SYSTOLIC_GRID))
        return out, info
    finally:
        sim.close()


@pytest.mark.parametrize("noise", [False, True])
def test_periodic_256_cube_systolic_bitwise(noise):
    w = wl.c2_periodic_dielectric(nsteps=128)
    if noise:
        rng = np.random.default_rng(77)
        f = [rng.uniform(-0.1, 0.1, size=w.shape).astype(np.float32) for _ in range(6)]
        w.fields = tuple(wl.zero_pec(f, w.bc))
    got, (band, grid) = _run(w, "systolic", 128, {fdtd.OPT_TILE_X: 15})
    assert band > 0 and grid >= 18 * 18    # a whole ring group is resident
    assert_bitwise(got, oracle_f32(w, 128), "256^3 periodic x/y (noise=%s)" % noise)


def test_periodic_256_cube_wide_tile_bitwise():
    """The 19-wide tile (material indices in registers): a ring group is then
    14 x 18 = 252 tiles, so two groups are resident at once; from random
    fields, against the FP32 oracle after 128 steps."""
    w = wl.c2_periodic_dielectric(nsteps=128)
    rng = np.random.default_rng(78)
    f = [rng.uniform(-0.1, 0.1, size=w.shape).astype(np.float32) for _ in range(6)]
    w.fields = tuple(wl.zero_pec(f, w.bc))
    got, (band, grid) = _run(w, "systolic", 128, {fdtd.OPT_TILE_X: 19})
    assert band > 0 and grid >= 2 * 14 * 18
    assert_bitwise(got, oracle_f32(w, 128), "256^3 periodic x/y, 19-wide tile")


def test_periodic_256_cube_systolic_split_calls_and_band():
    """The same grid over calls of 40 + 24 steps with an explicit 16-step band."""
    w = wl.c2_periodic_dielectric(nsteps=64)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        sim.set_option(fdtd.OPT_BAND_STEPS, 16)
        sim.set_materials(w.eps)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.step(40)
        sim.step(24)
        got = sim.read_fields()
    finally:
        sim.close()
    assert_bitwise(got, oracle_f32(w, 64), "256^3 periodic, 40 + 24 steps")


def test_batched_sweep_64_grids_bitwise():
    nsteps = 160
    ws = wl.c4_batch(64, nsteps)
    sims = []
    try:
        for w in ws:
            s = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
            s.set_materials(w.eps)
            for src in w.sources:
                s.add_source(src["comp"], src["i"], src["j"], src["k"], src["waveform"])
            sims.append(s)
        fdtd.step_batch(sims, nsteps)
        for q, (w, s) in enumerate(zip(ws, sims)):
            assert s.current_step == nsteps
            assert_bitwise(s.read_fields(), oracle_f32(w, nsteps), "batch member %d %s" % (q, w.shape))
    finally:
        for s in sims:
            s.close()
