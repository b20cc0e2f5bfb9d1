"""GPU parity of fdtd_step_batch: several independent simulations (different
sizes, boundaries, materials and sources) advanced in one persistent systolic
launch over a shared ticket queue.  Every member must equal the FP32 oracle
bit for bit, exactly as when stepped alone."""
import numpy as np
import pytest

from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise, oracle_f32

pytestmark = pytest.mark.gpu
PEC, PER = 0, 1


def _sim(w, opts=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    for k, v in (opts or {}).items():
        sim.set_option(k, v)
    sim.set_materials(w.eps)
    if w.fields is not None:
        sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


MEMBERS = [
    ((40, 36, 34), (PEC, PEC, PEC), [(20, 18, 17), (15, 15, 15)]),
    ((16, 20, 50), (PER, PEC, PER), [(0, 15, 14), (8, 10, 25)]),
    ((31, 47, 29), (PEC, PEC, PEC), [(14, 1, 28)]),
    ((45, 16, 46), (PEC, PER, PEC), [(22, 0, 23)]),
    ((9, 5, 13), (PEC, PEC, PEC), []),
    ((30, 30, 30), (PER, PER, PER), [(29, 29, 29)]),
]


def _members(nsteps, seed0=100):
    return [wl.small_case(shape, bc, seed=seed0 + q, nsteps=nsteps, dipoles=d)
            for q, (shape, bc, d) in enumerate(MEMBERS)]


@pytest.mark.parametrize("band,wg", [(8, 0), (3, 0), (16, 27)])
def test_batch_bitwise(band, wg):
    ws = _members(21)
    opts = {fdtd.OPT_BAND_STEPS: band}
    if wg:
        opts[fdtd.OPT_WORKGROUPS] = wg
    sims = [_sim(ws[0], opts)] + [_sim(w) for w in ws[1:]]
    try:
        fdtd.step_batch(sims, 21)
        for w, s in zip(ws, sims):
            assert s.current_step == 21
            assert_bitwise(s.read_fields(), oracle_f32(w, 21), "batch member %s" % (w.shape,))
    finally:
        for s in sims:
            s.close()


def test_batch_pec_members_two_workgroups():
    """PEC members only, on a persistent grid of two workgroups with bands of 3
    steps: the face ring holds few slots, so a ticket's slot was last held a
    few tickets earlier, often by another member, and its slot-reuse wait and
    band-start wait take effect on nearly every ticket."""
    pec = [m for m in MEMBERS if m[1] == (PEC, PEC, PEC)]
    ws = [wl.small_case(shape, bc, seed=300 + q, nsteps=17, dipoles=d)
          for q, (shape, bc, d) in enumerate(pec)]
    sims = [_sim(ws[0], {fdtd.OPT_BAND_STEPS: 3, fdtd.OPT_WORKGROUPS: 2})] + [_sim(w) for w in ws[1:]]
    try:
        fdtd.step_batch(sims, 17)
        for w, s in zip(ws, sims):
            assert s.current_step == 17
            assert_bitwise(s.read_fields(), oracle_f32(w, 17), "batch member %s, 2 workgroups" % (w.shape,))
    finally:
        for s in sims:
            s.close()


def test_batch_split_calls_and_mixed_with_solo_steps():
    """Batch calls, solo calls and plain steps interleave on the members'
    own streams; the state stays exact throughout (sources keep their step
    index per member)."""
    ws = _members(40, seed0=200)
    sims = [_sim(w) for w in ws]
    try:
        fdtd.step_batch(sims, 7)
        sims[1].step(5)                      # member 1 ahead by 5 steps
        sims[2].set_option(fdtd.OPT_SCHEME, fdtd.SCHEME_PLAIN)
        sims[2].step(5)                      # member 2 ahead by 5, plain scheme
        fdtd.step_batch(sims[::-1], 13)      # another lead, another order
        fdtd.step_batch(sims, 15)
        steps = [35, 40, 40, 35, 35, 35]
        for w, s, n in zip(ws, sims, steps):
            assert s.current_step == n
            assert_bitwise(s.read_fields(), oracle_f32(w, n), "member %s after %d" % (w.shape, n))
    finally:
        for s in sims:
            s.close()


def test_batch_of_one_equals_step():
    w = wl.small_case((33, 31, 29), (PEC, PEC, PEC), seed=5, nsteps=17, dipoles=[(16, 15, 14)])
    s = _sim(w)
    try:
        fdtd.step_batch([s], 17)
        assert_bitwise(s.read_fields(), oracle_f32(w), "batch of one")
    finally:
        s.close()


def test_batch_error_paths():
    ws = _members(4)
    sims = [_sim(w) for w in ws[:3]]
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([sims[0], sims[1], sims[0]], 3)
        assert e.value.code == fdtd.FDTD_EINVAL
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch(sims, -1)
        assert e.value.code == fdtd.FDTD_EINVAL
        # a 40x40 periodic ring group (9 tiles) cannot be resident on a grid of 4
        w = wl.small_case((40, 40, 20), (PER, PER, PEC), seed=3, nsteps=4)
        ring = _sim(w)
        sims[0].set_option(fdtd.OPT_WORKGROUPS, 4)
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([sims[0], ring], 3)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        ring.close()
        # nothing moved
        for s in sims:
            assert s.current_step == 0
        short = _sim(wl.small_case((15, 20, 20), (PER, PEC, PEC), seed=3, nsteps=4))
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([sims[1], short], 3)
        assert e.value.code == fdtd.FDTD_EUNSUPPORTED
        short.close()
        fdtd.step_batch(sims, 0)
    finally:
        for s in sims:
            s.close()


def test_batch_of_uneven_grids():
    """A scaled-down batched-sweep setup: 12 PEC grids with dimensions drawn
    from {16, 32, ..., 80} per axis, own random permittivity boxes and a
    centred dipole, 60 steps in one launch."""
    rng = np.random.default_rng(4)
    ws = []
    for q in range(12):
        shape = tuple(int(rng.choice(np.arange(16, 81, 16))) for _ in range(3))
        ws.append(wl.random_dielectric(shape, (PEC, PEC, PEC), 6, 400 + q, 60,
                                       side=(2, max(3, min(shape) // 2)), eps_bg=1.0,
                                       dipoles=[tuple(s // 2 for s in shape)]))
    sims = [_sim(w) for w in ws]
    try:
        fdtd.step_batch(sims, 60)
        for w, s in zip(ws, sims):
            assert_bitwise(s.read_fields(), oracle_f32(w, 60), "uneven member %s" % (w.shape,))
    finally:
        for s in sims:
            s.close()
