"""CPU checks of the systolic schedule (plan, dependencies, data flow).

The emulator in tests/systolic_emulator.py runs the tile tickets as
interleaved coroutines with the kernel's waits; with every interleaving the
result must be bit-identical to the FP32 oracle, because the scheme performs
exactly the same update equations in an order that respects every
dependency (Section 3: one-directional dependencies along the x-t diagonal).
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import workloads as wl
from tests import systolic_emulator as emu

PEC = 0


def _oracle(w, n):
    return oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, n, sources=w.sources,
                      dtype=np.float32)


def _coeffs(w):
    cE = oracle.coeff_E(w.eps3(), w.bc, w.dt, w.dx)
    return [oracle.round_f32(c) for c in cE], np.float32(w.dt / w.dx)


def test_plan_is_topological_and_covers_the_domain():
    shape, W, K, n = (13, 11, 9), (4, 3, 5), 3, 8
    tickets, ranges, ticket_of = emu.plan(shape, W, K, n)
    for i, (band, a, b, c) in enumerate(tickets):
        for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]:
            j = ticket_of.get((band, a + d[0], b + d[1], c + d[2]))
            assert j is None or j < i
        if band > 0:
            j = ticket_of.get((band - 1, a, b, c))
            assert j is None or j < i
    # at every step of every band, the tiles' B boxes cover each domain cell once
    for band, rg in enumerate(ranges):
        for tau in range(band * K + 1, min(n, (band + 1) * K) + 1):
            cover = np.zeros(shape, int)
            for a in range(rg[0][0], rg[0][1] + 1):
                for b in range(rg[1][0], rg[1][1] + 1):
                    for c in range(rg[2][0], rg[2][1] + 1):
                        lo = [a * W[0] + tau, b * W[1] + tau, c * W[2] + tau]
                        sl = tuple(slice(max(0, l), max(0, min(s, l + w)))
                                   for l, s, w in zip(lo, shape, W))
                        cover[sl] += 1
            assert np.all(cover == 1)


@pytest.mark.parametrize("shape,W,K,nsteps,seed", [
    ((10, 9, 11), (3, 4, 3), 3, 7, 1),
    ((16, 12, 14), (5, 4, 6), 4, 9, 2),
    ((7, 13, 6), (2, 2, 3), 2, 5, 3),
    ((12, 12, 12), (15, 15, 15), 6, 11, 4),   # one tile larger than the grid
])
def test_emulated_schedule_bitwise(shape, W, K, nsteps, seed):
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=seed, nsteps=nsteps,
                      dipoles=[tuple(s // 2 for s in shape), (1, 1, 1)])
    ref = _oracle(w, nsteps)
    cE, cH = _coeffs(w)
    for resident, sched_seed in [(1, 0), (3, 1), (50, 2)]:
        m = emu.Machine(w.fields, cE, cH, shape, W, K, nsteps, sources=w.sources)
        got = m.run(resident=resident, seed=sched_seed)
        for c in range(6):
            np.testing.assert_array_equal(got[c].view(np.uint32), ref[c].view(np.uint32),
                                          err_msg="component %d resident %d" % (c, resident))


@pytest.mark.parametrize("shape,W,bc", [
    ((10, 9, 11), (3, 4, 3), (1, 0, 0)),
    ((10, 9, 11), (3, 4, 3), (0, 1, 1)),
    ((8, 7, 9), (3, 3, 4), (1, 1, 1)),
    ((9, 6, 12), (4, 5, 5), (1, 1, 0)),
])
def test_plan_periodic_groups(shape, W, bc):
    """Periodic axes: every band holds the whole ring of each periodic axis,
    the tiles of one ring group (same PEC coordinates) are consecutive, every
    upwind neighbour outside the group comes earlier, and the boxes (wrapped)
    cover each cell once at every step."""
    K, n = 3, 7
    tickets, ranges, ticket_of = emu.plan(shape, W, K, n, bc)
    L = emu.ring_tiles(shape, W, bc)
    pec = [d for d in range(3) if not bc[d]]
    groups = {}
    for i, (band, a, b, c) in enumerate(tickets):
        g = (band,) + tuple((a, b, c)[d] for d in pec)
        groups.setdefault(g, []).append(i)
        for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]:
            u = emu.wrap_tile((a + d[0], b + d[1], c + d[2]), L)
            j = ticket_of.get((band,) + u)
            if j is None:
                continue
            same = all(u[e] == (a, b, c)[e] for e in pec)
            assert same or j < i
    for g, idx in groups.items():
        assert idx == list(range(idx[0], idx[0] + len(idx)))
        assert len(idx) == int(np.prod([L[d] for d in range(3) if bc[d]]))
    for band, rg in enumerate(ranges):
        for tau in range(band * K + 1, min(n, (band + 1) * K) + 1):
            cover = np.zeros(shape, int)
            for a in range(rg[0][0], rg[0][1] + 1):
                for b in range(rg[1][0], rg[1][1] + 1):
                    for c in range(rg[2][0], rg[2][1] + 1):
                        idx = []
                        for d, t in enumerate((a, b, c)):
                            w = W[d]
                            if bc[d] and t == L[d] - 1:
                                w = shape[d] - W[d] * (L[d] - 1)
                            x = np.arange(t * W[d] + tau, t * W[d] + tau + w)
                            idx.append(x % shape[d] if bc[d] else x[(x >= 0) & (x < shape[d])])
                        cover[np.ix_(*idx)] += 1
            assert np.all(cover == 1)


@pytest.mark.parametrize("shape,W,K,nsteps,bc,seed", [
    ((10, 9, 11), (3, 4, 3), 3, 7, (1, 0, 0), 11),
    ((10, 9, 11), (3, 4, 3), 4, 9, (0, 1, 1), 12),
    ((8, 7, 9), (3, 3, 4), 3, 8, (1, 1, 1), 13),
    ((9, 6, 12), (4, 5, 5), 2, 7, (1, 1, 0), 14),
    ((7, 8, 10), (6, 7, 3), 5, 9, (1, 1, 0), 15),   # two-tile rings, width-1 ragged tiles
])
def test_emulated_schedule_periodic_bitwise(shape, W, K, nsteps, bc, seed):
    dips = [tuple(s // 2 for s in shape), (shape[0] - 1, 1, shape[2] - 1)]
    dips = [d for d in dips if all(bc[a] or d[a] >= 1 for a in range(3))]
    w = wl.small_case(shape, bc, seed=seed, nsteps=nsteps, dipoles=dips)
    ref = _oracle(w, nsteps)
    cE, cH = _coeffs(w)
    L = emu.ring_tiles(shape, W, bc)
    group = int(np.prod([L[d] for d in range(3) if bc[d]]))
    for resident, sched_seed in [(group, 0), (group + 5, 1), (400, 2)]:
        m = emu.Machine(w.fields, cE, cH, shape, W, K, nsteps, sources=w.sources, bc=bc)
        got = m.run(resident=resident, seed=sched_seed)
        for c in range(6):
            np.testing.assert_array_equal(got[c].view(np.uint32), ref[c].view(np.uint32),
                                          err_msg="component %d resident %d" % (c, resident))


def test_emulated_periodic_ring_needs_coresidency():
    """With fewer resident tickets than a ring group the schedule cannot
    progress (the ring's tiles wait on each other in a cycle)."""
    shape, W, bc = (9, 8, 8), (3, 4, 4), (1, 0, 0)
    w = wl.small_case(shape, bc, seed=3, nsteps=4)
    cE, cH = _coeffs(w)
    m = emu.Machine(w.fields, cE, cH, shape, W, 2, 4, bc=bc)
    with pytest.raises(RuntimeError, match="deadlocked"):
        m.run(resident=2, seed=0)


def test_emulator_detects_a_missing_wait(monkeypatch):
    """Sanity of the harness: dropping the wait before the forward-E load
    makes some interleaving read stale data."""
    shape, W, K, n = (10, 10, 10), (3, 3, 3), 3, 6
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=5, nsteps=n)
    ref = _oracle(w, n)
    cE, cH = _coeffs(w)
    orig = emu.Machine.wait

    def no_wait(self, tile, target):
        if target % 2 == 1:      # the E-level waits
            return
        yield from orig(self, tile, target)
    monkeypatch.setattr(emu.Machine, "wait", no_wait)
    differs = False
    for seed in range(6):
        m = emu.Machine(w.fields, cE, cH, shape, W, K, n)
        got = m.run(resident=60, seed=seed)
        if any(not np.array_equal(np.nan_to_num(got[c]), ref[c]) for c in range(6)):
            differs = True
            break
    assert differs


def test_crop_oracle_reproduces_full_runs():
    """The sampled full-size parity check recomputes cells on crops; the crop
    construction must give exactly the full-grid value (walls, edges, corners,
    interior, sources)."""
    from tests.crop_oracle import crop_oracle
    w = wl.random_dielectric((40, 36, 44), (PEC, PEC, PEC), 10, 3, 6, side=(2, 10), noise=0.1,
                             dipoles=[(20, 18, 22)])
    full = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 6, sources=w.sources,
                      dtype=np.float32)
    for p in [(0, 0, 0), (39, 35, 43), (0, 35, 20), (39, 0, 1), (20, 0, 43), (1, 18, 0),
              (39, 18, 22), (20, 35, 22), (20, 18, 43), (13, 7, 7), (20, 18, 22), (21, 18, 21)]:
        ref = crop_oracle(w, p, 6)
        val = np.array([f[p] for f in full], np.float32)
        np.testing.assert_array_equal(ref.view(np.uint32), val.view(np.uint32), err_msg=str(p))


def test_emulator_detects_a_missing_reuse_wait(monkeypatch):
    """Sanity of the harness: a ring slot reused after waiting only for the
    occupant's -z consumer (not the diagonal consumers that take the x- and
    y-face edges) is overwritten early in some interleaving."""
    shape, W, K, n = (12, 12, 12), (3, 3, 3), 4, 8
    w = wl.small_case(shape, (PEC, PEC, PEC), seed=6, nsteps=n)
    ref = _oracle(w, n)
    cE, cH = _coeffs(w)
    def run(seed, only_z):
        m = emu.Machine(w.fields, cE, cH, shape, W, K, n)   # R sized for all consumers
        if only_z:
            monkeypatch.setattr(emu, "DOWN", [(0, 0, -1)])
        got = m.run(resident=200, seed=seed)
        monkeypatch.undo()
        return any(not np.array_equal(np.nan_to_num(got[c]), ref[c]) for c in range(6))
    bad = [s for s in range(8) if run(s, True)]
    assert bad
    assert not run(bad[0], False)


def test_crop_oracle_reproduces_full_fp16_runs():
    """The same crop construction under the FP16-storage systolic schedule
    (rounding of the whole grid every K steps is cell by cell, so a crop sees
    the same rounding)."""
    from oracle import f16
    from tests.crop_oracle import crop_oracle
    w = wl.random_dielectric((40, 36, 44), (PEC, PEC, PEC), 10, 3, 6, side=(2, 10), noise=0.1,
                             dipoles=[(20, 18, 22)])
    cE16 = f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)
    full = f16.run_systolic(w.fields, cE16, np.float32(w.dt / w.dx), [6], [4], sources=w.sources)
    for p in [(0, 0, 0), (39, 35, 43), (0, 35, 20), (20, 18, 22), (21, 18, 21), (13, 7, 7)]:
        ref = crop_oracle(w, p, 6, fp16_band=4)
        val = np.array([f[p] for f in full], np.float32)
        np.testing.assert_array_equal(ref.view(np.uint32), val.view(np.uint32), err_msg=str(p))
