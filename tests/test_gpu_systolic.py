"""GPU parity of the systolic scheme: bit-identical to the FP32 oracle.

The systolic scheme performs exactly the update equations of the plain
scheme, in an order that respects every dependency, so its FP32 result must
be the same value bit for bit (Section 1: the scheme reorders the work and
leaves the update itself unchanged).  Cases cover several tiles per axis with ragged tails,
band lengths from 1 to more than the step count, sources on tile edges and
corners, grids smaller than one tile, fewer persistent workgroups than
tiles (schedule stress), calls split across bands, scheme switches on a live
context, periodic axes (rings of tiles resident together, ragged last tiles,
sources across the seams), and the refusal of configurations the scheme does
not cover.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def run_sys(w, nsteps=None, **opts):
    o = {}
    if "band" in opts:
        o[fdtd.OPT_BAND_STEPS] = opts["band"]
    if "wg" in opts:
        o[fdtd.OPT_WORKGROUPS] = opts["wg"]
    if opts.get("wx"):
        o[fdtd.OPT_TILE_X] = opts["wx"]
    return fdtd.run_workload(w, "systolic", nsteps=nsteps, options=o)


@pytest.mark.parametrize("shape,nsteps,band,seed", [
    ((16, 16, 16), 5, 16, 1),
    ((40, 36, 34), 20, 16, 2),
    ((31, 47, 29), 23, 7, 3),
    ((64, 20, 50), 17, 1, 4),
    ((9, 5, 13), 11, 4, 5),          # grid smaller than one tile
    ((1, 30, 30), 6, 3, 6),          # one-cell-thick axis
    ((45, 45, 45), 33, 10, 7),
])
@pytest.mark.parametrize("wx", [0, 15])   # the default (19 with material indices) and 15
def test_systolic_bitwise_small(shape, nsteps, band, seed, wx):
    dips = [tuple(s // 2 for s in shape)]
    # sources on tile edges and corners of the initial tiling
    for p in [(15, 15, 15), (14, 1, 29), (1, 16, 1)]:
        if all(1 <= p[a] < shape[a] for a in range(3)):
            dips.append(p)
    dips = [d for d in dips if d[0] >= 1 and d[1] >= 1]
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=seed, nsteps=nsteps, dipoles=dips)
    assert_bitwise(run_sys(w, band=band, wx=wx), oracle_f32(w), "systolic %s wx=%d" % (shape, wx))


@pytest.mark.parametrize("shape,seed", [
    ((30, 1, 30), 41),     # one cell along y: every y row but one holds ghosts
    ((30, 30, 1), 42),     # one cell along z
    ((40, 1, 1), 43),      # a line along x
    ((1, 1, 40), 44),      # a line along z
    ((2, 2, 2), 45),       # fewer cells than lanes on every axis
    ((20, 3, 17), 46),     # thin y beside ragged x and z
])
@pytest.mark.parametrize("wx", [0, 15, 11])
def test_systolic_thin_axes(shape, seed, wx):
    """PEC grids with one to three cells along some axes, over several bands:
    the tile's slots along those axes are ghosts but for a few cells.  (The
    z-directed dipole goes only where Ez is not frozen by the PEC planes x = 0
    and y = 0; the random initial fields drive every case.)"""
    c = tuple(s // 2 for s in shape)
    dips = [c] if c[0] >= 1 and c[1] >= 1 else []
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=seed, nsteps=13, dipoles=dips)
    assert_bitwise(run_sys(w, band=5, wx=wx), oracle_f32(w), "systolic thin %s wx=%d" % (shape, wx))


@pytest.mark.parametrize("wg", [1, 2, 7, 64])
def test_systolic_few_workgroups(wg):
    w = wl.small_case((50, 40, 45), (PEC, PEC, PEC), seed=11, nsteps=19, dipoles=[(25, 20, 22)])
    assert_bitwise(run_sys(w, band=6, wg=wg), oracle_f32(w), "systolic wg=%d" % wg)


def test_systolic_long_call_small_grid():
    """20000 steps in one call on 32^3: tiles drift one cell per step along the
    diagonal, so over the call the tile indices span more than 1300 per axis
    (the schedule keeps one progress counter per ticket, not per tile index)."""
    w = wl.small_case((32, 32, 32), (PEC, PEC, PEC), seed=31, nsteps=20000, dipoles=[(16, 16, 16)])
    assert_bitwise(run_sys(w), oracle_f32(w), "systolic 20000 steps")


def test_systolic_c1_bitwise_and_fp64_bound():
    w = wl.c1_cavity_pulse()
    gpu = run_sys(w)
    assert_bitwise(gpu, oracle_f32(w), "systolic C1")
    f64 = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, w.nsteps, dtype=np.float64)
    assert ym.rel_l2(gpu, f64) < 1e-5


def test_systolic_split_calls_and_scheme_switch():
    w = wl.small_case((48, 44, 40), (PEC, PEC, PEC), seed=13, nsteps=41, dipoles=[(20, 21, 22)])
    ref = oracle_f32(w)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    sim.set_materials(w.eps)
    sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    sim.step(9)
    sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_PLAIN)
    sim.step(5)
    sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_SYSTOLIC)
    sim.set_option(fdtd.OPT_BAND_STEPS, 4)
    sim.step(13)
    sim.step(14)
    assert sim.current_step == 41
    assert_bitwise(sim.read_fields(), ref, "systolic split")
    sim.close()


@pytest.mark.parametrize("shape,bc,nsteps,band,seed", [
    ((31, 47, 29), (PER, PEC, PEC), 23, 7, 21),     # x ring of 3 tiles, ragged width 1
    ((40, 36, 34), (PER, PER, PER), 20, 16, 22),    # every axis periodic: one group of 27
    ((16, 20, 50), (PER, PEC, PER), 17, 5, 23),     # two-tile x ring, ragged z tile of width 5
    ((45, 16, 46), (PEC, PER, PEC), 33, 10, 24),    # y ring with a width-1 tile
    ((64, 64, 30), (PER, PER, PEC), 40, 6, 25),     # the boundary pattern of the C2 workload
    ((30, 30, 30), (PER, PER, PER), 12, 1, 26),     # rings with no ragged tile, band of 1
])
@pytest.mark.parametrize("wx", [0, 15])
def test_systolic_periodic_bitwise(shape, bc, nsteps, band, seed, wx):
    # dipoles at the interior, on tile edges and across the periodic seams
    pts = [tuple(s // 2 for s in shape), (0, 15, 14), (shape[0] - 1, 1, shape[2] - 1), (15, 0, 0)]
    dips = [p for p in pts if all(bc[a] == PER or p[a] >= 1 for a in (0, 1))
            and all(p[a] < shape[a] for a in range(3))]
    w = wl.small_case(shape, bc, seed=seed, nsteps=nsteps, dipoles=dips)
    assert_bitwise(run_sys(w, band=band, wx=wx), oracle_f32(w), "systolic periodic %s %s wx=%d" % (shape, bc, wx))


def test_systolic_periodic_ring_group_needs_resident_grid():
    """A ring group (here 3 x 3 tiles of an x-y periodic grid) must be resident
    at once: a smaller persistent grid is refused (never run, never a silent
    fallback); a grid of exactly one group is bit-exact."""
    w = wl.small_case((40, 40, 20), (PER, PER, PEC), seed=27, nsteps=9, dipoles=[(3, 38, 10)])
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    sim.set_option(fdtd.OPT_WORKGROUPS, 8)
    with pytest.raises(fdtd.FdtdError) as e:
        sim.step(1)
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    assert sim.current_step == 0
    sim.close()
    assert_bitwise(run_sys(w, band=4, wg=9), oracle_f32(w), "systolic periodic wg=9")


def test_systolic_refuses_short_periodic_axis_without_fallback():
    sim = fdtd.Simulation((15, 16, 16), 0.5, 1.0, (PER, PEC, PEC), scheme="systolic")
    with pytest.raises(fdtd.FdtdError) as e:
        sim.step(1)
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    assert sim.current_step == 0
    sim.close()


@pytest.mark.parametrize("shape,bc", [((40, 36, 34), (PEC, PEC, PEC)), ((35, 20, 31), (PER, PEC, PER))])
def test_systolic_fence_synchronisation_variant(monkeypatch, shape, bc):
    """The alternative synchronisation (cached accesses, agent-scope release
    and acquire fences around the progress counters, FDTD_SYSTOLIC_SYNC=fence)
    gives the same bits as the device-scope default."""
    monkeypatch.setenv("FDTD_SYSTOLIC_SYNC", "fence")
    w = wl.small_case(shape, bc, seed=sum(shape), nsteps=19, dipoles=[tuple(s // 2 for s in shape)])
    assert_bitwise(run_sys(w, band=6), oracle_f32(w), "fence variant %s" % (shape,))
