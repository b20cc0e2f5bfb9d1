"""fdtd_invariants_noalloc: the allocation-free variant of fdtd_invariants.

Called through the C ABI (ctypes) with device outputs, its sums and per-cell
divergences must equal those of fdtd_invariants on the same state bit for bit
(the same kernels and the same fixed summation order; only the partial-sum
scratch differs).  Two calls in a row, the second on a smaller grid, so that
the second call runs over the scratch the first one left behind; a third call
without per-cell outputs.
"""
import numpy as np
import pytest

from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _gpu_available():
    # (also brings up torch's HIP runtime before the library's first call,
    # as the other GPU tests do at import)
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


if not _gpu_available():
    pytest.skip("no GPU", allow_module_level=True)


def _sim(shape, bc, seed):
    w = wl.small_case(shape, bc, seed=seed, nsteps=6, dipoles=[tuple(n // 2 for n in shape)])
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    sim.set_materials(w.eps)
    sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    sim.step(6)
    return sim


def _check(sim, per_cell):
    import torch
    dev = torch.device("cuda:0")
    n = int(np.prod(sim.shape))
    sums = torch.full((len(fdtd.INVARIANT_NAMES),), float("nan"), dtype=torch.float64, device=dev)
    de = torch.full((n,), float("nan"), dtype=torch.float64, device=dev) if per_cell else None
    dh = torch.full((n,), float("nan"), dtype=torch.float64, device=dev) if per_cell else None
    sim.invariants_noalloc(sums, de, dh)
    sim.synchronize()
    got = sums.cpu().numpy()
    if per_cell:
        ref, rde, rdh = sim.invariants(per_cell=True)
        assert np.array_equal(de.cpu().numpy().reshape(sim.shape).view(np.uint64), rde.view(np.uint64))
        assert np.array_equal(dh.cpu().numpy().reshape(sim.shape).view(np.uint64), rdh.view(np.uint64))
    else:
        ref = sim.invariants()
    want = np.array([ref[k] for k in fdtd.INVARIANT_NAMES])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (got, want)
    assert np.all(np.isfinite(got)) and got[fdtd.INVARIANT_NAMES.index("e_energy")] > 0


def test_noalloc_matches_the_allocating_entry_point_on_two_calls_in_a_row():
    big = _sim((70, 66, 61), (0, 1, 0), seed=21)
    small = _sim((20, 17, 19), (1, 0, 0), seed=22)
    try:
        _check(big, per_cell=True)
        _check(small, per_cell=True)    # smaller input, over the first call's scratch
        _check(big, per_cell=False)
    finally:
        big.close()
        small.close()


def test_noalloc_rejects_a_null_sums_pointer():
    sim = _sim((16, 16, 16), (0, 0, 0), seed=3)
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            sim._check(sim._lib.fdtd_invariants_noalloc(sim._h, None, None, None))
        assert e.value.code == fdtd.FDTD_EINVAL
    finally:
        sim.close()
