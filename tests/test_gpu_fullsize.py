"""Parity at the full 1024x1024x512 size, in the launch configuration of the
benchmark, on sampled cells.

After n steps a cell depends only on cells within n of it on each axis (one
cell per axis per step), so each sample is recomputed by the FP32 oracle on a
crop of half-width n+2 around it.  A crop that ends at the grid's upper wall
gets an artificial PEC plane at its own lower end (its tangential E zeroed),
so that its periodic wrap reproduces the wall; that plane is more than n
cells from the sample and cannot reach it.  Crops that start at the lower
wall keep the real wall; interior crops wrap periodically, again more than n
cells from the sample.  Samples cover the interior, every wall, edges,
corners and the three dipoles.  Values are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2502_20610_amd import fdtd
from paper_2502_20610_amd import workloads as wl
from tests.crop_oracle import crop_oracle as _crop_oracle

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


def _samples(w, rng):
    nx, ny, nz = w.shape
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, nz // 2), (nx - 1, 0, 1),
           (nx // 2, 0, nz - 1), (1, ny // 2, 0), (nx - 1, ny // 2, nz // 2),
           (nx // 2, ny - 1, nz // 2), (nx // 2, ny // 2, nz - 1), (nx // 3, ny // 5, 7)]
    for s in w.sources:
        pts.append((s["i"], s["j"], s["k"]))
        pts.append((s["i"] + 1, s["j"], s["k"] - 1))
    for _ in range(8):
        pts.append(tuple(int(rng.integers(0, n)) for n in w.shape))
    # cells on tile edges of the systolic tiling at the first and last step
    pts += [(15 * 20 - 1, 15 * 30, 15 * 10 + 3), (15 * 40 + 8, 15 * 50 - 1, 15 * 20 - 1)]
    return pts


@pytest.mark.parametrize("scheme,band,storage", [("systolic", 4, "fp32"), ("systolic", 16, "fp32"),
                                                 ("systolic", 0, "fp32"), ("plain", 0, "fp32"),
                                                 ("systolic", 0, "fp16")])
def test_fullsize_sampled_bitwise(scheme, band, storage):
    """band 0 = the band the library picks for this grid (the benchmark's
    launch: 64 steps here), over two bands (each sample's crop then spans
    261^3 cells).  With FP16 storage (the benchmark's --storage fp16 launch)
    the crops take the band-end rounding too."""
    import torch
    w = wl.c3_large_dielectric(nsteps=8)
    auto = scheme == "systolic" and band == 0
    nsteps = 8 if scheme == "plain" else (128 if auto else 2 * band)
    pts = _samples(w, np.random.default_rng(5))
    # seeded noise in the dependency cone of every sample, so that no sampled
    # value is trivially zero
    rng = np.random.default_rng(77)
    fields = [np.zeros(w.shape, np.float32) for _ in range(6)]
    r = nsteps + 2
    for p in pts:
        sl = tuple(slice(max(0, p[a] - r), min(w.shape[a], p[a] + r + 1)) for a in range(3))
        for f in fields:
            f[sl] = rng.uniform(-1e-2, 1e-2, size=f[sl].shape).astype(np.float32)
    wl.zero_pec(fields, w.bc)
    w.fields = tuple(fields)
    dev = torch.device("cuda:0")
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, storage=storage)
    try:
        if band:
            sim.set_option(fdtd.OPT_BAND_STEPS, band)
        sim.set_materials(torch.from_numpy(w.eps).to(dev))
        sim.set_fields([torch.from_numpy(f).to(dev) for f in w.fields])
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.step(nsteps)
        used_band = sim.info(fdtd.INFO_SYSTOLIC_BAND)
        if auto:
            assert used_band == 64
        idx = torch.tensor(pts, dtype=torch.long, device=dev)
        got = []
        for c in range(6):
            buf = torch.empty(w.shape, dtype=torch.float32, device=dev)
            sim.read_fields(mask=1 << c, out=[buf] * 6)
            sim.synchronize()
            got.append(buf[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy())
            del buf
        got = np.stack(got, axis=1)
    finally:
        sim.close()
    bad = []
    for n, p in enumerate(pts):
        ref = _crop_oracle(w, p, nsteps, fp16_band=used_band if storage == "fp16" else None)
        if not np.array_equal(ref.view(np.uint32), got[n].view(np.uint32)):
            bad.append((p, got[n], ref))
    assert not bad, "%d/%d samples differ, first %s" % (len(bad), len(pts), bad[0])
    # the check is not vacuous: most sampled cells are non-zero
    assert np.count_nonzero(got) > got.size // 2


def test_max_grid_auto_band_fits_the_rings_and_is_exact():
    """The largest grid the ABI accepts, 1024^3 = 2^30 cells, 128 steps with the
    automatic band: the cost model would take 64-step bands, whose face rings
    would pass the 4 GB of a buffer descriptor's 32-bit offsets, so the launch
    takes the longest band that fits instead.  Sampled cells (walls, corners,
    interior, dipoles) bit for bit against the crop oracle."""
    import torch
    w = wl.c3_large_dielectric(shape=(1024, 1024, 1024), nsteps=128)
    nsteps = 128
    rng = np.random.default_rng(9)
    pts = [(0, 0, 0), (1023, 1023, 1023), (0, 1023, 512), (1023, 0, 1), (512, 511, 1023),
           (700, 3, 300)] + [(s["i"], s["j"], s["k"]) for s in w.sources]
    pts += [tuple(int(rng.integers(0, 1024)) for _ in range(3)) for _ in range(3)]
    dev = torch.device("cuda:0")
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        sim.set_materials(torch.from_numpy(w.eps).to(dev))
        # seeded noise in the dependency cone of every sample (device-side
        # fields; the crop oracle rebuilds each cone from the same host arrays)
        fields = [torch.zeros(w.shape, dtype=torch.float32, device=dev) for _ in range(6)]
        r = nsteps + 2
        host_patches = []
        for p in pts:
            sl = tuple(slice(max(0, p[a] - r), min(1024, p[a] + r + 1)) for a in range(3))
            vals = [rng.uniform(-1e-2, 1e-2, size=tuple(s.stop - s.start for s in sl)).astype(np.float32)
                    for _ in range(6)]
            host_patches.append((sl, vals))
            for f, v in zip(fields, vals):
                f[sl] = torch.from_numpy(v).to(dev)
        torch.cuda.synchronize()
        sim.set_fields(fields)   # PEC-tangential entries are zeroed by the library
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.step(nsteps)
        band = sim.info(fdtd.INFO_SYSTOLIC_BAND)
        slots = sim.info(fdtd.INFO_RING_SLOTS)
        assert band < 64 and slots * band * 6 * 1024 < 2 ** 32, (band, slots)
        idx = torch.tensor(pts, dtype=torch.long, device=dev)
        got = []
        for c in range(6):
            sim.read_fields(mask=1 << c, out=[fields[c]] * 6)
            sim.synchronize()
            got.append(fields[c][idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy())
        got = np.stack(got, axis=1)
        del fields
    finally:
        sim.close()
    # the same initial state on the host, for the crop oracle (patches applied
    # in the same order, later ones overwriting earlier ones)
    host = [np.zeros(w.shape, np.float32) for _ in range(6)]
    for sl, vals in host_patches:
        for f, v in zip(host, vals):
            f[sl] = v
    wl.zero_pec(host, w.bc)
    w.fields = tuple(host)
    bad = []
    for n, p in enumerate(pts):
        ref = _crop_oracle(w, p, nsteps)
        if not np.array_equal(ref.view(np.uint32), got[n].view(np.uint32)):
            bad.append((p, got[n], ref))
    assert not bad, "%d/%d samples differ, first %s" % (len(bad), len(pts), bad[0])
    assert np.count_nonzero(got) > got.size // 2
