"""Failure path of the systolic kernel's bounded waits, forced from the host.

A wait on a neighbour's progress counter polls at most FDTD_OPT_SPIN_LIMIT
times.  With a limit of one poll on a grid of thousands of tiles, waits that
need more than that are certain (a downwind tile reaches its first wait a few
polls after its upwind neighbour started loading its box); the waiting
workgroup raises the timeout bit, and every workgroup leaves the ticket loop
(at its next ticket or within 256 polls of any wait).  Every kernel therefore
ends normally: the host then sees FDTD_ETIMEOUT once and FDTD_ESTATE from
every later call, and a fresh context on the same device runs correctly.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _expect(code, fn, *a):
    with pytest.raises(fdtd.FdtdError) as e:
        fn(*a)
    assert e.value.code == code, str(e.value)


def _fresh_run_is_exact():
    w = wl.small_case((34, 31, 36), (0, 0, 0), seed=3, nsteps=12, dipoles=[(17, 15, 18)])
    got = fdtd.run_workload(w, "systolic")
    ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, w.nsteps, sources=w.sources,
                     dtype=np.float32)
    for c in range(6):
        assert np.array_equal(got[c].view(np.uint32), ref[c].view(np.uint32))


def test_expired_wait_drains_the_grid_and_poisons_the_context():
    w = wl.bare_bones(128, nsteps=48)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        sim.set_materials(w.eps)
        sim.set_fields(w.fields)
        sim.synchronize()
        sim.set_option(fdtd.OPT_SPIN_LIMIT, 1)
        sim.step(48)                      # queued; the kernel drains on the first expiry
        _expect(fdtd.FDTD_ETIMEOUT, sim.synchronize)
        _expect(fdtd.FDTD_ESTATE, sim.synchronize)
        _expect(fdtd.FDTD_ESTATE, sim.step, 1)
        _expect(fdtd.FDTD_ESTATE, sim.read_fields)
        _expect(fdtd.FDTD_ESTATE, sim.set_option, fdtd.OPT_SPIN_LIMIT, 1 << 22)
        _expect(fdtd.FDTD_ESTATE, sim.invariants)
    finally:
        sim.close()
    _fresh_run_is_exact()


def test_expired_wait_in_a_batch_is_reported_by_every_member():
    ws = wl.c4_batch(3, 40, dims=(64, 96))
    sims = []
    try:
        for w in ws:
            s = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
            s.set_materials(w.eps)
            sims.append(s)
        for s in sims:
            s.synchronize()
        sims[0].set_option(fdtd.OPT_SPIN_LIMIT, 1)   # launch options are the lead's
        fdtd.step_batch(sims, 40)
        for s in sims:
            _expect(fdtd.FDTD_ETIMEOUT, s.synchronize)
            _expect(fdtd.FDTD_ESTATE, s.step, 1)
    finally:
        for s in sims:
            s.close()
    _fresh_run_is_exact()


def test_pending_bad_permittivity_does_not_stop_a_batch_member():
    """A member's bad-permittivity bit (device input, checked on the device)
    stays its own: the shared launch runs every member, the other members
    report nothing, and that member reports FDTD_EINVAL at its next
    synchronising call."""
    import torch
    ws = [wl.small_case((32, 30, 34), (0, 0, 0), seed=s, nsteps=10, dipoles=[(16, 15, 17)])
          for s in (1, 2)]
    sims = []
    try:
        for q, w in enumerate(ws):
            s = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
            eps = w.eps.copy()
            if q == 1:
                eps[3, 4, 5] = 0.5          # below 1: flagged on the device
            s.set_materials(torch.from_numpy(eps).to("cuda:0"))
            s.set_fields(w.fields)
            for src in w.sources:
                s.add_source(src["comp"], src["i"], src["j"], src["k"], src["waveform"])
            sims.append(s)
        fdtd.step_batch(sims, 10)
        got = sims[0].read_fields()
        ref = oracle.run(ws[0].fields, ws[0].eps3(), ws[0].bc, ws[0].dt, ws[0].dx, 10,
                         sources=ws[0].sources, dtype=np.float32)
        for c in range(6):
            assert np.array_equal(got[c].view(np.uint32), ref[c].view(np.uint32))
        _expect(fdtd.FDTD_EINVAL, sims[1].synchronize)
        sims[1].synchronize()                # reported once, then cleared
        assert sims[1].current_step == 10
    finally:
        for s in sims:
            s.close()
