"""Plain step loops replayed as HIP graphs (FDTD_OPT_GRAPHS).

Calls of 16 steps or more replay a captured graph of 16 steps; the step
number the sources need comes from a device counter the graph advances.
Every replay must give the same bits as one launch per kernel (the graph
off) and as the FP32 oracle: several calls in a row, with the library's own
eager work between them (direct remainder steps, a read-back, new sources,
a field reset), for the two-launch and the fused scheme, with and without
sources, conductive, and with FP16 storage (against the eager launches).
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.test_gpu_parity import assert_bitwise

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


CALLS = [16, 5, 32, 19, 48]   # whole graphs, direct remainders, and both together


def _sim(w, scheme, graphs, storage="fp32", sigma=None):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, storage=storage)
    sim.set_option(fdtd.OPT_GRAPHS, 1 if graphs else 0)
    if sigma is None:
        sim.set_materials(w.eps)
    else:
        sim.set_materials(w.eps, sigma=sigma)
    sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    return sim


def _oracle(w, state, step0, n, sigma=None):
    return oracle.run(state, w.eps3(), w.bc, w.dt, w.dx, n, sources=w.sources, dtype=np.float32,
                      step0=step0, sigma=sigma)


@pytest.mark.parametrize("scheme", ["plain", "plain_fused"])
@pytest.mark.parametrize("with_sources", [True, False])
@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PEC, PER)])
def test_graph_replays_match_eager_and_oracle(scheme, with_sources, bc):
    w = wl.small_case((33, 29, 40), bc, seed=61 + bc[0], nsteps=120,
                      dipoles=[(16, 14, 20), (9, 20, 31)] if with_sources else [])
    g, d = _sim(w, scheme, True), _sim(w, scheme, False)
    try:
        state, step = tuple(np.array(f) for f in w.fields), 0
        for n in CALLS:
            g.step(n)
            d.step(n)
            got, eager = g.read_fields(), d.read_fields()
            state = _oracle(w, state, step, n)
            step += n
            assert_bitwise(got, eager, "%s graph vs eager after %d steps" % (scheme, step))
            assert_bitwise(got, state, "%s graph vs oracle after %d steps" % (scheme, step))
            assert g.current_step == step
    finally:
        g.close()
        d.close()


@pytest.mark.parametrize("scheme", ["plain", "plain_fused"])
def test_graph_recaptured_after_new_sources_and_reset(scheme):
    w = wl.small_case((30, 34, 28), (PEC, PEC, PEC), seed=7, nsteps=80, dipoles=[(15, 17, 14)])
    late = wl.dipole(wl.EY, 10, 9, 8, wl.gaussian_sine(40, 0.5), first_step=32)
    srcs = list(w.sources) + [late]
    sim = _sim(w, scheme, True)
    try:
        sim.step(32)
        sim.add_source(late["comp"], late["i"], late["j"], late["k"], late["waveform"], 32)
        sim.step(32)                       # a new source table: the graph is captured again
        mid = sim.read_fields()
        sim.set_fields(w.fields)           # eager work between replays
        sim.step(16)
        got = sim.read_fields()
    finally:
        sim.close()
    a = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 32, sources=w.sources, dtype=np.float32)
    a = oracle.run(a, w.eps3(), w.bc, w.dt, w.dx, 32, sources=srcs, dtype=np.float32, step0=32)
    assert_bitwise(mid, a, "%s after a new source" % scheme)
    ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 16, sources=srcs, dtype=np.float32, step0=64)
    assert_bitwise(got, ref, "%s after a field reset" % scheme)


def test_graph_conductive_and_fp16():
    w = wl.small_case((28, 31, 26), (PEC, PER, PEC), seed=19, nsteps=40, dipoles=[(14, 15, 13)])
    sig = [np.random.default_rng(2).uniform(0.0, 0.2, w.shape).astype(np.float32) for _ in range(3)]
    for scheme in ("plain", "plain_fused"):
        sim = _sim(w, scheme, True, sigma=sig)
        try:
            sim.step(35)
            got = sim.read_fields()
        finally:
            sim.close()
        ref = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, 35, sources=w.sources, dtype=np.float32,
                         sigma=sig)
        assert_bitwise(got, ref, "%s conductive" % scheme)
    outs = []
    for graphs in (True, False):
        sim = _sim(w, "plain", graphs, storage="fp16")
        try:
            for n in (16, 3, 32):
                sim.step(n)
                outs.append(sim.read_fields())
        finally:
            sim.close()
    for a, b in zip(outs[:3], outs[3:]):
        assert_bitwise(a, b, "FP16 storage, graph vs eager")
