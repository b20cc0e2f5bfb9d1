"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

FP32 results must be bit-identical to the FP32 oracle (same operation order,
no contraction, IEEE denormals); the FP32 run must also stay within the 1e-5
relative-L2 bound of the FP64 oracle.  Cases span several tiles with ragged
tails, every boundary combination, sources on and off tile edges, and
degenerate shapes (one-cell-thick axes).
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym

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


def assert_bitwise(gpu, ref, label=""):
    for c, (a, b) in enumerate(zip(gpu, ref)):
        a = np.asarray(a, np.float32)
        b = np.asarray(b, np.float32)
        ua, ub = a.view(np.uint32), b.view(np.uint32)
        bad = np.flatnonzero(ua.ravel() != ub.ravel())
        if bad.size:
            p = np.unravel_index(bad[0], a.shape)
            raise AssertionError("%s component %d: %d/%d entries differ, first at %s: gpu %r "
                                 "oracle %r" % (label, c, bad.size, a.size, p, a[p], b[p]))


def oracle_f32(w, nsteps=None):
    n = w.nsteps if nsteps is None else nsteps
    return oracle.run(w.fields_or_zeros(), w.eps3(), w.bc, w.dt, w.dx, n, sources=w.sources,
                      dtype=np.float32)


BCS = [(a, b, c) for a in (PEC, PER) for b in (PEC, PER) for c in (PEC, PER)]


@pytest.mark.parametrize("bc", BCS)
def test_plain_bitwise_8cube_all_boundaries(bc):
    w = wl.small_case((8, 8, 8), bc, seed=100 + sum(b << i for i, b in enumerate(bc)), nsteps=12,
                      dipoles=[(3, 4, 5)])
    assert_bitwise(fdtd.run_workload(w, "plain"), oracle_f32(w), "plain 8^3 %s" % (bc,))


@pytest.mark.parametrize("shape,bc,seed", [
    ((37, 29, 70), (PEC, PER, PEC), 1),
    ((1, 17, 33), (PER, PEC, PEC), 2),
    ((20, 1, 1), (PEC, PER, PER), 3),
    ((5, 66, 130), (PER, PER, PER), 4),
])
def test_plain_bitwise_ragged(shape, bc, seed):
    dip = [(shape[0] // 2, shape[1] // 2, shape[2] // 2)]
    # keep the dipole off PEC-frozen entries of Ez (i == 0 on PEC x, j == 0 on PEC y)
    if (bc[0] == PEC and dip[0][0] == 0) or (bc[1] == PEC and dip[0][1] == 0):
        dip = []
    w = wl.small_case(shape, bc, seed=seed, nsteps=25, dipoles=dip)
    assert_bitwise(fdtd.run_workload(w, "plain"), oracle_f32(w), "plain %s" % (shape,))


def test_plain_c1_bitwise_and_fp64_bound():
    w = wl.c1_cavity_pulse()
    gpu = fdtd.run_workload(w, "plain")
    assert_bitwise(gpu, oracle_f32(w), "plain C1")
    f64 = oracle.run(w.fields, w.eps3(), w.bc, w.dt, w.dx, w.nsteps, dtype=np.float64)
    assert ym.rel_l2(gpu, f64) < 1e-5


def test_plain_steps_split_across_calls_and_restore():
    """step(a); step(b) == step(a+b); state read back and restored into a new
    context continues bit-identically (checkpoint/resume)."""
    w = wl.small_case((24, 20, 18), (PEC, PEC, PER), seed=9, nsteps=30, dipoles=[(7, 8, 9)])
    ref = oracle_f32(w)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    sim.set_materials(w.eps)
    sim.set_fields(w.fields)
    for s in w.sources:
        sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
    sim.step(11)
    mid = sim.read_fields()
    assert sim.current_step == 11
    sim.close()
    # the restored context starts at step count 0: shift the waveform by 11 samples
    sim3 = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    sim3.set_materials(w.eps)
    sim3.set_fields(mid)
    for s in w.sources:
        sim3.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"][11:])
    sim3.step(19)
    assert_bitwise(sim3.read_fields(), ref, "plain resume")
    sim3.close()


def test_plain_device_pointers_and_profile():
    import torch
    w = wl.small_case((16, 16, 16), (PEC, PEC, PEC), seed=12, nsteps=7)
    ref = oracle_f32(w)
    dev = torch.device("cuda:0")
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain",
                          stream=torch.cuda.current_stream().cuda_stream)
    sim.set_option(fdtd.OPT_PROFILE, 1)
    sim.set_materials(torch.from_numpy(w.eps).to(dev))
    sim.set_fields([torch.from_numpy(f).to(dev) for f in w.fields])
    sim.step(w.nsteps)
    out = [torch.empty(w.shape, dtype=torch.float32, device=dev) for _ in range(6)]
    sim.read_fields(out=out)
    sim.synchronize()
    assert_bitwise([o.cpu().numpy() for o in out], ref, "plain device ptrs")
    n, ms = sim.kernel_stats(fdtd.KERNEL_PLAIN_E)
    assert n == w.nsteps and ms > 0
    sim.close()


def test_error_paths_on_gpu():
    sim = fdtd.Simulation((8, 8, 8), 0.5, 1.0, (PEC, PEC, PEC))
    with pytest.raises(fdtd.FdtdError) as e:
        sim.set_materials(np.full((8, 8, 8), 0.5, np.float32))
    assert e.value.code == fdtd.FDTD_EINVAL
    with pytest.raises(fdtd.FdtdError) as e:
        sim.add_source(wl.EZ, 0, 3, 3, np.ones(4, np.float32))   # Ez frozen on PEC x wall
    assert e.value.code == fdtd.FDTD_EINVAL
    with pytest.raises(fdtd.FdtdError) as e:
        sim.add_source(wl.EZ, 3, 3, 9, np.ones(4, np.float32))
    assert e.value.code == fdtd.FDTD_EINVAL
    with pytest.raises(fdtd.FdtdError) as e:   # design box outside the grid
        sim.adjoint(4, wl.EZ, (1, 1, 1), (2, 2, 2), 0.5, (6, 6, 6), (9, 8, 8))
    assert e.value.code == fdtd.FDTD_EINVAL
    with pytest.raises(fdtd.FdtdError) as e:
        sim.step(-1)
    assert e.value.code == fdtd.FDTD_EINVAL
    sim.step(0)
    assert sim.current_step == 0
    sim.close()
