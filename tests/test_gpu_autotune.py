"""The 11- and 19-wide systolic tiles on lossless grids and the measured choice
of tile width and band length (fdtd_autotune).

* FDTD_OPT_TILE_X = 11 runs the lossless update on the narrow tile: bitwise
  with the FP32 oracle on PEC, periodic and mixed boundaries (ragged periodic
  rings of 11-wide tiles), with material indices and with the arrays.
* FDTD_OPT_TILE_X = 19 (material indices in registers, 20-row y and z faces)
  on the same grids, bitwise; it refuses grids without indices and periodic
  x axes shorter than 20 cells.
* fdtd_autotune leaves the fields and the step count as they were, returns a
  candidate pair, keeps it for a second context of the same key, and the run
  that follows stays bitwise.
* Refusals: the 11-wide tile with FP16 storage, a batch mixing widths.
"""
import numpy as np
import pytest

from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu

PEC, PER = 0, 1


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


if not _gpu_available():
    pytest.skip("no GPU", allow_module_level=True)


def _sim(w, opts=()):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    for k, v in opts:
        sim.set_option(k, v)
    sim.set_materials(w.eps)
    sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


@pytest.mark.parametrize("bc,shape", [((PEC, PEC, PEC), (45, 37, 41)), ((PER, PER, PEC), (40, 34, 31)),
                                      ((PER, PEC, PER), (23, 30, 33)), ((PER, PER, PER), (35, 32, 17))])
@pytest.mark.parametrize("width,ids", [(11, 1), (11, 0), (19, 1)])
def test_tile_widths_bitwise(bc, shape, width, ids):
    w = wl.small_case(shape, bc, seed=71 + shape[0], nsteps=23, dipoles=[tuple(n // 2 for n in shape)])
    sim = _sim(w, [(fdtd.OPT_TILE_X, width), (fdtd.OPT_MATERIAL_IDS, ids), (fdtd.OPT_BAND_STEPS, 8)])
    try:
        sim.step(23)
        assert sim.info(fdtd.INFO_TILE_X) == width
        assert_bitwise(sim.read_fields(), oracle_f32(w), "%d-wide tile %s ids=%d" % (width, bc, ids))
    finally:
        sim.close()


@pytest.mark.parametrize("bc,shape,band", [((PEC, PEC, PEC), (83, 45, 52), 24), ((PER, PER, PEC), (58, 47, 40), 16),
                                           ((PER, PER, PER), (40, 33, 36), 32)])
def test_wide_tile_longer_runs_and_sources(bc, shape, band):
    """The 19-wide tile over 60 steps from random fields, with dipoles on
    tile seams and near the walls, and several bands."""
    dip = [(19, 15, 14), (shape[0] - 2, 1, shape[2] // 2), (38, shape[1] // 2, 29)]
    w = wl.small_case(shape, bc, seed=5 + shape[1], nsteps=60, dipoles=dip)
    sim = _sim(w, [(fdtd.OPT_TILE_X, 19), (fdtd.OPT_BAND_STEPS, band)])
    try:
        sim.step(25)
        sim.step(35)
        assert sim.info(fdtd.INFO_TILE_X) == 19 and sim.info(fdtd.INFO_MATERIALS) > 0
        assert_bitwise(sim.read_fields(), oracle_f32(w, 60), "19-wide tile %s K=%d" % (bc, band))
    finally:
        sim.close()


def test_autotune_restores_state_and_keeps_its_choice():
    w = wl.small_case((52, 47, 44), (PEC, PEC, PEC), seed=5, nsteps=30, dipoles=[(26, 23, 22)])
    sim = _sim(w)
    try:
        sim.step(7)
        before = sim.read_fields()
        tile, band = sim.autotune(23)
        assert tile in (11, 15, 19) and band in (8, 12, 16, 23)
        assert sim.current_step == 7
        assert_bitwise(sim.read_fields(), before, "state after autotune")
        sim.step(23)
        assert sim.info(fdtd.INFO_TILE_X) == tile and sim.info(fdtd.INFO_SYSTOLIC_BAND) == band
        assert_bitwise(sim.read_fields(), oracle_f32(w, 30), "run after autotune")
    finally:
        sim.close()
    other = _sim(w)
    try:
        assert other.autotune(23) == (tile, band)     # kept for the same key
    finally:
        other.close()


def test_autotune_with_the_plain_scheme_as_a_candidate():
    """FDTD_OPT_AUTOTUNE_PLAIN: the plain two-launch scheme is timed too; on a
    small grid it usually wins.  Whichever wins, the context reports it, the
    outputs agree with it, and the run that follows is bitwise.  FP16 storage
    never switches (its schemes round at different places)."""
    w = wl.small_case((32, 32, 32), (PEC, PEC, PEC), seed=8, nsteps=40, dipoles=[(16, 16, 16)])
    sim = _sim(w, [(fdtd.OPT_AUTOTUNE_PLAIN, 1)])
    try:
        tile, band = sim.autotune(40)
        scheme = sim.info(fdtd.INFO_SCHEME)
        assert scheme in (fdtd.SCHEME_PLAIN, fdtd.SCHEME_SYSTOLIC)
        assert (tile, band) == (0, 0) if scheme == fdtd.SCHEME_PLAIN else tile in (11, 15, 19)
        sim.step(40)
        assert_bitwise(sim.read_fields(), oracle_f32(w, 40), "run after autotune (scheme %d)" % scheme)
    finally:
        sim.close()
    h = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic", storage="fp16")
    try:
        h.set_option(fdtd.OPT_AUTOTUNE_PLAIN, 1)
        h.set_materials(w.eps)
        tile, band = h.autotune(16)
        assert h.info(fdtd.INFO_SCHEME) == fdtd.SCHEME_SYSTOLIC and tile in (15, 19)
    finally:
        h.close()


def test_autotune_refusals_and_narrow_tile_refusals():
    w = wl.small_case((24, 24, 24), (PEC, PEC, PEC), seed=2, nsteps=4)
    plain = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            plain.autotune(10)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    finally:
        plain.close()
    h = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic", storage="fp16")
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            h.set_option(fdtd.OPT_TILE_X, 11)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    finally:
        h.close()
    # the 19-wide tile without material indices, and on a periodic x axis of
    # fewer than 20 cells
    for bc, shape, opts in [((PEC, PEC, PEC), (24, 24, 24), [(fdtd.OPT_MATERIAL_IDS, 0)]),
                            ((PER, PEC, PEC), (18, 24, 24), [])]:
        v = wl.small_case(shape, bc, seed=3, nsteps=4)
        s = _sim(v, [(fdtd.OPT_TILE_X, 19)] + opts)
        try:
            with pytest.raises(fdtd.FdtdError) as e:
                s.step(4)
            assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        finally:
            s.close()
    a, b = _sim(w, [(fdtd.OPT_TILE_X, 11)]), _sim(w)
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([a, b], 4)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    finally:
        a.close()
        b.close()
