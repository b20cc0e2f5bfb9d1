"""Material indices on the systolic scheme.

Lossless FP32 grids with at most 256 distinct coefficient triples
(cEx, cEy, cEz) -- entry 0, (+0, +0, +0), included -- stream a 4-byte index
per cell instead of the three coefficients.  The triples are found on the
device; the results must stay bit-identical to the FP32 oracle with the
indices on or off (FDTD_OPT_MATERIAL_IDS), at the table's size limit and
just past it (where the per-cell arrays serve), after the materials change,
from device input, and in a batch that mixes the two forms.
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


def _run(w, ids=True, eps=None, steps=None, wx=0):
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        sim.set_option(fdtd.OPT_MATERIAL_IDS, 1 if ids else 0)
        sim.set_option(fdtd.OPT_TILE_X, wx)
        sim.set_materials(w.eps if eps is None else eps)
        if w.fields is not None:
            sim.set_fields(w.fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.step(w.nsteps if steps is None else steps)
        return sim.read_fields(), sim.info(fdtd.INFO_MATERIALS)
    finally:
        sim.close()


def _distinct_triples(w):
    """Distinct (cEx, cEy, cEz) of the workload, the zero entry included."""
    import oracle
    c = [oracle.round_f32(x) for x in oracle.coeff_E(w.eps3(), w.bc, w.dt, w.dx)]
    t = np.stack([x.view(np.uint32).ravel() for x in c], axis=1)
    u = {tuple(r) for r in np.unique(t, axis=0)}
    u.add((0, 0, 0))
    return len(u)


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PEC), (PEC, PER, PER), (PER, PER, PER)])
def test_indices_and_arrays_both_bitwise(bc):
    w = wl.small_case((47, 38, 41), bc, seed=31 + bc[0] + 2 * bc[1], nsteps=21, dipoles=[(23, 19, 20)])
    ref = oracle_f32(w)
    for wx in (0, 15):   # the default (19-wide: indices in registers) and 15-wide
        got, nmat = _run(w, ids=True, wx=wx)
        assert nmat == _distinct_triples(w)
        assert_bitwise(got, ref, "material indices %s wx=%d" % (bc, wx))
    got, _ = _run(w, ids=False)
    assert_bitwise(got, ref, "coefficient arrays %s" % (bc,))


@pytest.mark.parametrize("nvals,expect_ids", [(255, True), (256, False)])
def test_table_limit(nvals, expect_ids):
    """Periodic on every axis (no PEC zeroing): k distinct eps give k + 1
    entries with the zero one, so 255 values fill the table exactly and 256
    do not fit."""
    shape = (36, 32, 34)
    w = wl.small_case(shape, (PER, PER, PER), seed=5, nsteps=16, dipoles=[(18, 16, 17)])
    vals = np.float32(1.0) + np.arange(nvals, dtype=np.float32) * np.float32(0.03125)
    rng = np.random.default_rng(8)
    eps = vals[rng.permutation(np.resize(np.arange(nvals), w.cells))].reshape(shape).astype(np.float32)
    w.eps = eps
    got, nmat = _run(w)
    assert nmat == (256 if expect_ids else 0)
    assert_bitwise(got, oracle_f32(w), "%d materials" % nvals)


def test_materials_change_and_device_input():
    import torch
    w = wl.small_case((40, 33, 37), (PEC, PEC, PER), seed=12, nsteps=18, dipoles=[(20, 16, 18)])
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        assert sim.info(fdtd.INFO_MATERIALS) > 0          # eps = 1 at creation
        many = np.random.default_rng(3).uniform(1.0, 12.0, w.shape).astype(np.float32)
        sim.set_materials(many)
        assert sim.info(fdtd.INFO_MATERIALS) == 0          # per-cell arrays
        sim.set_materials(torch.from_numpy(w.eps).to("cuda:0"))
        assert sim.info(fdtd.INFO_MATERIALS) == _distinct_triples(w)
        sim.set_fields(w.fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.step(w.nsteps)
        assert_bitwise(sim.read_fields(), oracle_f32(w), "device eps after a change")
    finally:
        sim.close()


def test_conductive_contexts_have_no_table():
    w = wl.small_case((20, 20, 20), (PEC, PEC, PEC), seed=2, nsteps=4)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        sim.set_materials(w.eps, sigma=[np.full(w.shape, 0.1, np.float32)] * 3)
        assert sim.info(fdtd.INFO_MATERIALS) == 0
        sim.set_materials(w.eps)
        assert sim.info(fdtd.INFO_MATERIALS) > 0
    finally:
        sim.close()


@pytest.mark.parametrize("bc", [(PEC, PEC, PEC), (PER, PER, PEC)])
def test_fp16_storage_indices_and_rings_both_bitwise(bc):
    """FP16 storage: the table holds the exact FP32 values of the binary16
    coefficients; with indices the x and y faces read them instead of the
    coefficient rings.  Both forms equal the FP16-storage oracle."""
    from oracle import f16
    w = wl.small_case((41, 36, 38), bc, seed=17 + bc[0], nsteps=24, dipoles=[(20, 18, 19)])
    ref = f16.run_systolic(w.fields, f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx), np.float32(w.dt / w.dx),
                           [24], [8], sources=w.sources)
    for ids in (1, 0):
        sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic", storage="fp16")
        try:
            sim.set_option(fdtd.OPT_MATERIAL_IDS, ids)
            sim.set_option(fdtd.OPT_BAND_STEPS, 8)
            sim.set_materials(w.eps)
            assert sim.info(fdtd.INFO_MATERIALS) > 0
            sim.set_fields(w.fields)
            for s in w.sources:
                sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
            sim.step(24)
            got = sim.read_fields()
        finally:
            sim.close()
        assert_bitwise(got, ref, "FP16 storage %s ids=%d" % (bc, ids))


def test_batch_mixing_indices_and_arrays():
    """One member past the table limit: the shared launch streams the arrays
    for every member; all stay bitwise."""
    ws = [wl.small_case((34, 31, 36), (PEC, PEC, PEC), seed=s, nsteps=14, dipoles=[(17, 15, 18)])
          for s in (41, 42)]
    ws[1].eps = np.random.default_rng(4).uniform(1.0, 9.0, ws[1].shape).astype(np.float32)
    sims = []
    try:
        for w in ws:
            s = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
            s.set_materials(w.eps)
            s.set_fields(w.fields)
            for src in w.sources:
                s.add_source(src["comp"], src["i"], src["j"], src["k"], src["waveform"])
            sims.append(s)
        assert sims[0].info(fdtd.INFO_MATERIALS) > 0 and sims[1].info(fdtd.INFO_MATERIALS) == 0
        fdtd.step_batch(sims, 14)
        for q, (w, s) in enumerate(zip(ws, sims)):
            assert_bitwise(s.read_fields(), oracle_f32(w, 14), "batch member %d" % q)
    finally:
        for s in sims:
            s.close()
