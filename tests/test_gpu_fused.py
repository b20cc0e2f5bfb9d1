"""GPU parity of the fused plain step (one launch per step, ping-pong arrays)
against the FP32 oracle, bit for bit.

The fused kernel owns 7 y rows x 64 z lanes per block and recomputes E' on
one more row and, in lane 63, at the cell after the tile; cases put grid
sizes around those widths (below, equal, one over, several tiles), one-cell-
thick axes, many x chunks, sources on block edges, halo cells and chunk
planes, several sources on one cell, conductive materials, odd step counts
(the two array sets trade places every step) and scheme switches in the
middle of a run.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import BCS, assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def _sim(w, scheme="plain_fused", sigma=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme)
    sim.set_materials(w.eps, sigma=sigma)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"], s.get("first_step", 0))
    return sim


@pytest.mark.parametrize("bc", BCS)
def test_fused_bitwise_8cube_all_boundaries(bc):
    w = wl.small_case((8, 8, 8), bc, seed=3, nsteps=11, dipoles=[(4, 3, 5)])
    sim = _sim(w)
    sim.step(11)
    assert_bitwise(sim.read_fields(), oracle_f32(w, 11), "fused 8^3 %s" % (bc,))
    sim.close()


# (shape, boundaries, steps, dipoles): z widths 62/63/64/126/127/130, y widths
# around 7 and 8, a single x plane, a single y row, many x chunks
CASES = [
    ((37, 29, 70), (PEC, PER, PEC), 13, [(5, 6, 62), (18, 7, 63), (30, 13, 1), (36, 14, 69)]),
    ((20, 15, 127), (PER, PEC, PER), 9, [(1, 1, 63), (19, 14, 126), (10, 8, 64)]),
    ((9, 16, 126), (PEC, PEC, PEC), 12, [(4, 6, 62), (4, 7, 125)]),
    ((12, 7, 63), (PER, PER, PER), 10, [(0, 6, 62), (11, 0, 0)]),
    ((1, 17, 33), (PER, PEC, PEC), 8, [(0, 8, 16)]),
    ((64, 1, 64), (PEC, PER, PER), 8, [(32, 0, 63)]),
    ((96, 80, 200), (PEC, PEC, PEC), 7, [(47, 41, 125), (48, 42, 126), (95, 79, 199)]),
    ((5, 66, 130), (PER, PER, PER), 9, [(2, 65, 129), (2, 63, 62)]),
    ((10, 9, 128), (PEC, PER, PER), 9, [(5, 4, 64), (5, 4, 63), (9, 8, 127), (1, 0, 0)]),
    ((7, 15, 65), (PER, PEC, PEC), 10, [(3, 7, 64), (3, 7, 63), (6, 14, 1)]),
]


@pytest.mark.parametrize("shape,bc,n,dip", CASES)
def test_fused_bitwise_ragged(shape, bc, n, dip):
    w = wl.small_case(shape, bc, seed=sum(shape), nsteps=n, dipoles=dip)
    sim = _sim(w)
    sim.step(n)
    assert_bitwise(sim.read_fields(), oracle_f32(w, n), "fused %s %s" % (shape, bc))
    sim.close()


def test_fused_many_sources_same_cell_and_offsets():
    """Twenty-one sources of every E component (interior cells, staggered
    first steps): two on the same cell and component (table-order sums) at
    the first cell of a z tile, which the previous tile's lane 63 recomputes,
    and one more there on another component and x plane."""
    rng = np.random.default_rng(5)
    shape = (30, 25, 70)
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=6, nsteps=15)
    wave = wl.gaussian_sine(15, 0.5)
    srcs = []
    for q in range(18):
        cell = [int(rng.integers(1, s)) for s in shape]
        srcs.append(wl.dipole(q % 3, *cell, wave * (1 + 0.1 * q), first_step=q % 4))
    srcs.append(wl.dipole(1, 10, 7, 64, wave))
    srcs.append(wl.dipole(1, 10, 7, 64, wave * 0.37, first_step=2))
    srcs.append(wl.dipole(0, 11, 7, 64, wave * 0.5))
    w.sources = srcs
    sim = _sim(w)
    sim.step(15)
    assert_bitwise(sim.read_fields(), oracle_f32(w, 15), "fused, many sources")
    sim.close()


def test_fused_conductive_bitwise():
    w = wl.small_case((33, 29, 70), (PER, PEC, PER), seed=8, nsteps=21, dipoles=[(16, 14, 63)])
    rng = np.random.default_rng(9)
    sig = [rng.uniform(0.0, 0.3, w.shape).astype(np.float32) for _ in range(3)]
    sim = _sim(w, sigma=sig)
    sim.step(21)
    ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 21, sources=w.sources,
                     dtype=np.float32, sigma=sig)
    assert_bitwise(sim.read_fields(), ref, "fused conductive")
    sim.close()


def test_fused_scheme_switches_and_odd_steps():
    """plain 7 -> fused 5 -> systolic 6 -> fused 3 -> plain 2: the state
    carries across the buffer swaps and the other schemes."""
    w = wl.small_case((40, 36, 34), (PEC, PEC, PEC), seed=12, nsteps=23, dipoles=[(20, 18, 17)])
    sim = _sim(w, scheme="plain")
    for scheme, n in (("plain", 7), ("plain_fused", 5), ("systolic", 6), ("plain_fused", 3),
                      ("plain", 2)):
        sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEMES[scheme])
        sim.step(n)
    assert sim.current_step == 23
    assert_bitwise(sim.read_fields(), oracle_f32(w, 23), "fused with switches")
    # fields written between steps land in the current set
    sim.set_fields(w.fields)
    sim.set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_PLAIN_FUSED)
    sim.step(4)
    ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 4, step0=23, sources=w.sources,
                     dtype=np.float32)
    assert_bitwise(sim.read_fields(), ref, "fused after set_fields")
    sim.close()


def test_fused_profile_counts_and_fp16_refused():
    w = wl.small_case((16, 16, 16), (PEC, PEC, PEC), seed=13, nsteps=5)
    sim = _sim(w)
    sim.set_option(fdtd.OPT_PROFILE, 1)
    sim.step(5)
    n, ms = sim.kernel_stats(fdtd.KERNEL_PLAIN_FUSED)
    assert n == 5 and ms > 0
    assert sim.kernel_stats(fdtd.KERNEL_PLAIN_E)[0] == 0
    sim.close()
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain_fused", storage="fp16")
    sim.set_materials(w.eps)
    with pytest.raises(fdtd.FdtdError) as e:
        sim.step(1)
    assert e.value.code == fdtd.FDTD_EUNSUPPORTED
    assert sim.current_step == 0
    sim.close()
