"""Seeded synthetic workloads shaped like the paper's FDTD runs.

This module only *draws inputs*: permittivity maps, initial fields, source
waveforms and source positions.  It contains none of the update arithmetic,
so both the CPU oracle and the HIP library consume exactly the same FP32
arrays from it.  It imports nothing else from this package.

The paper's benchmark (Section 4) is a "bare-bones" domain of unstated size
with permittivity/conductivity fields and no sources; its naive sweep (Fig. 1)
grows the domain from a few cells to 2^25.  No public dataset is involved, so
these seeded generators stand in for its workloads:

* dielectric maps: a background permittivity with axis-aligned boxes of a
  higher permittivity; per box, each side is drawn from U{lo..hi}, the corner
  from U{0..n-side} (box fully inside), boxes painted in order (later wins);
  all three components of a cell get the cell's permittivity;
* point dipole sources driven by a Gaussian-modulated sinusoid evaluated in
  FP64 on the host and stored as an FP32 table.

Field order is always (Ex, Ey, Ez, Hx, Hy, Hz); arrays are float32, C order
``[nx, ny, nz]`` with z fastest.  ``bc`` per axis: 0 = PEC, 1 = periodic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PEC, PERIODIC = 0, 1
EX, EY, EZ, HX, HY, HZ = range(6)


@dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]
    bc: Tuple[int, int, int]
    dt: float
    dx: float
    nsteps: int
    eps: np.ndarray                       # float32 [nx,ny,nz], used for all 3 components
    fields: Optional[Tuple[np.ndarray, ...]] = None   # six float32 arrays, None = all zero
    sources: List[dict] = field(default_factory=list)  # comp,i,j,k,waveform(float32),first_step

    @property
    def cells(self) -> int:
        return int(self.shape[0]) * int(self.shape[1]) * int(self.shape[2])

    def eps3(self):
        return (self.eps, self.eps, self.eps)

    def fields_or_zeros(self):
        if self.fields is not None:
            return self.fields
        return tuple(np.zeros(self.shape, np.float32) for _ in range(6))


def pec_tangential_mask(shape, bc, comp: int) -> np.ndarray:
    """Boolean mask of the entries of E component ``comp`` that lie on the
    index-0 plane of a PEC axis to which the component is tangential.  These
    entries are held at +0 (the wall of the closed box)."""
    m = np.zeros(shape, dtype=bool)
    for a in range(3):
        if a != comp and bc[a] == PEC:
            sl = [slice(None)] * 3
            sl[a] = 0
            m[tuple(sl)] = True
    return m


def zero_pec(fields, bc):
    """Set the PEC-tangential E entries of an initial state to +0 (in place)."""
    for c in range(3):
        fields[c][pec_tangential_mask(fields[c].shape, bc, c)] = np.float32(0.0)
    return fields


def paint_boxes(shape, n_boxes: int, side_lo: int, side_hi, eps_bg: float, eps_box,
                rng: np.random.Generator, window=None) -> np.ndarray:
    """Background permittivity with ``n_boxes`` axis-aligned boxes painted in order.

    ``side_hi`` may be an int or a per-axis tuple; ``eps_box`` a float or a
    callable ``rng -> float`` (per-box permittivity).  With ``window`` =
    (lower corner, size) only that window of the map is returned (the same
    random draws, boxes clipped to the window)."""
    wlo, wsz = window if window is not None else ((0, 0, 0), tuple(shape))
    eps = np.full(wsz, np.float32(eps_bg), dtype=np.float32)
    his = side_hi if isinstance(side_hi, (tuple, list)) else (side_hi,) * 3
    for _ in range(n_boxes):
        lo_corner, hi_corner = [], []
        for a in range(3):
            hi = min(int(his[a]), shape[a])
            lo = min(side_lo, hi)
            side = int(rng.integers(lo, hi + 1))
            c0 = int(rng.integers(0, shape[a] - side + 1))
            lo_corner.append(c0)
            hi_corner.append(c0 + side)
        val = eps_box(rng) if callable(eps_box) else eps_box
        sl = tuple(slice(max(lo_corner[a] - wlo[a], 0), max(min(hi_corner[a] - wlo[a], wsz[a]), 0))
                   for a in range(3))
        eps[sl] = np.float32(val)
    return eps


def gaussian_sine(nsamples: int, dt: float, cells_per_period: float = 12.0,
                  eps_bg: float = 2.08, amplitude: float = 1.0) -> np.ndarray:
    """Gaussian-modulated sinusoid, FP64 on the host, returned as FP32.

    w[m] = A sin(w0 (t - t0)) exp(-(t - t0)^2 / (2 tau^2)),  t = m*dt,
    with w0 = 2 pi / (cells_per_period * sqrt(eps_bg)) (that many cells per
    wavelength in the background medium, c = 1, dx = 1), tau = 2 pi / w0 and
    t0 = 4 tau."""
    w0 = 2.0 * math.pi / (cells_per_period * math.sqrt(eps_bg))
    tau = 2.0 * math.pi / w0
    t0 = 4.0 * tau
    t = np.arange(nsamples, dtype=np.float64) * dt
    w = amplitude * np.sin(w0 * (t - t0)) * np.exp(-((t - t0) ** 2) / (2.0 * tau * tau))
    return w.astype(np.float32)


def dipole(comp: int, i: int, j: int, k: int, waveform: np.ndarray, first_step: int = 0) -> dict:
    return {"comp": int(comp), "i": int(i), "j": int(j), "k": int(k),
            "waveform": np.ascontiguousarray(waveform, dtype=np.float32),
            "first_step": int(first_step)}


# ---------------------------------------------------------------------------
# The configurations
# ---------------------------------------------------------------------------

def c1_cavity_pulse(n: int = 64, nsteps: int = 100, seed: int = 1) -> Workload:
    """64^3 vacuum PEC box, Gaussian Ez pulse (sigma = 4 cells) at the centre
    plus seeded U(-1e-3, 1e-3) noise on all six components; 100 steps."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    bc = (PEC, PEC, PEC)
    fields = [rng.uniform(-1e-3, 1e-3, size=shape).astype(np.float32) for _ in range(6)]
    c = n / 2.0
    i = np.arange(n, dtype=np.float64)
    r2 = ((i[:, None, None] - c) ** 2 + (i[None, :, None] - c) ** 2
          + (i[None, None, :] + 0.5 - c) ** 2)
    fields[EZ] = (fields[EZ].astype(np.float64) + np.exp(-r2 / 32.0)).astype(np.float32)
    zero_pec(fields, bc)
    eps = np.ones(shape, np.float32)
    return Workload("c1_pec_vacuum_pulse_%d" % n, shape, bc, 0.5, 1.0, nsteps, eps, tuple(fields))


def random_dielectric(shape, bc, n_boxes: int, seed: int, nsteps: int, side=(8, 64),
                      eps_bg: float = 2.08, eps_box: float = 12.25,
                      dipoles: Sequence[Tuple[int, int, int]] = (), noise: Optional[float] = None,
                      name: str = "random_dielectric") -> Workload:
    """Random-box dielectric (background eps_bg, boxes eps_box), Ez dipoles."""
    rng = np.random.default_rng(seed)
    eps = paint_boxes(shape, n_boxes, side[0], side[1], eps_bg, eps_box, rng)
    fields = None
    if noise is not None:
        f = [rng.uniform(-noise, noise, size=shape).astype(np.float32) for _ in range(6)]
        fields = tuple(zero_pec(f, bc))
    wave = gaussian_sine(nsteps, 0.5, eps_bg=eps_bg)
    sources = [dipole(EZ, *p, wave) for p in dipoles]
    return Workload(name, tuple(shape), tuple(bc), 0.5, 1.0, nsteps, eps, fields, sources)


def c2_periodic_dielectric(n: int = 256, nsteps: int = 1000, seed: int = 2) -> Workload:
    """256^3, periodic x/y, PEC z, 40 boxes of eps 12.25 (sides 8-64) in eps 2.08,
    one Ez dipole at the centre; 1000 steps."""
    c = n // 2
    return random_dielectric((n, n, n), (PERIODIC, PERIODIC, PEC), 40, seed, nsteps,
                             dipoles=[(c, c, c)], name="c2_periodic_xy_dielectric_%d" % n)


def c3_large_dielectric(shape=(1024, 1024, 512), nsteps: int = 500, seed: int = 3,
                        n_boxes: int = 2000) -> Workload:
    """1024x1024x512 PEC box, 2000 boxes of eps 12.25 in eps 2.08, three Ez dipoles
    at seeded interior cells in [16, n-16); 500 steps."""
    rng = np.random.default_rng(seed + 1000)
    dip = [tuple(int(rng.integers(16, s - 16)) for s in shape) for _ in range(3)]
    return random_dielectric(shape, (PEC, PEC, PEC), n_boxes, seed, nsteps, dipoles=dip,
                             name="c3_pec_dielectric_%dx%dx%d" % tuple(shape))


def c3_centre_crop(n: int = 128, nsteps: int = 500, seed: int = 3) -> Workload:
    """Accuracy rerun of the 1024x1024x512 workload: the central n^3 crop of its
    permittivity map, PEC walls, zero fields, one Ez dipole at the crop centre."""
    full_shape = (1024, 1024, 512)
    o = tuple((s - n) // 2 for s in full_shape)
    shape = (n, n, n)
    # the draws of c3_large_dielectric's map, painted on the window only
    eps = paint_boxes(full_shape, 2000, 8, 64, 2.08, 12.25, np.random.default_rng(seed),
                      window=(o, shape))
    fields = tuple(np.zeros(shape, np.float32) for _ in range(6))
    wave = gaussian_sine(nsteps, 0.5)
    return Workload("c3_centre_crop_%d" % n, shape, (PEC, PEC, PEC), 0.5, 1.0, nsteps, eps, fields,
                    [dipole(EZ, n // 2, n // 2, n // 2, wave)])


def c5_adjoint(nsteps: int = 4000, seed: int = 5):
    """Inverse-design gradient setup: 256x256x128 PEC box of eps 2.08 with a
    centred 64x64x16 design block of per-cell eps ~ U[2.08, 12.25] (x 96-159,
    y 96-159, z 56-71), an Ez dipole at (64, 128, 64) on its -x side, and the
    objective sum |DFT Ez|^2 at the source frequency over the 64x64 monitor
    plane x = 192, y 96-159, z 32-95.  Returns (workload, adjoint arguments)."""
    shape = (256, 256, 128)
    rng = np.random.default_rng(seed)
    eps = np.full(shape, np.float32(2.08), dtype=np.float32)
    eps[96:160, 96:160, 56:72] = rng.uniform(2.08, 12.25, (64, 64, 16)).astype(np.float32)
    wave = gaussian_sine(nsteps, 0.5)
    w = Workload("c5_adjoint_256x256x128", shape, (PEC, PEC, PEC), 0.5, 1.0, nsteps, eps, None,
                 [dipole(EZ, 64, 128, 64, wave)])
    omega = 2.0 * math.pi / (12.0 * math.sqrt(2.08))
    args = dict(nsteps=nsteps, mon_comp=EZ, mon_lo=(192, 96, 32), mon_hi=(193, 160, 96),
                omega=omega, des_lo=(96, 96, 56), des_hi=(160, 160, 72), checkpoint_every=0)
    return w, args


def c4_batch(nsims: int = 64, nsteps: int = 2000, seed: int = 4, dims=(64, 192)):
    """Batched sweep: nsims PEC grids, each axis drawn from {64, 80, ..., 192}
    (multiples of 16 in ``dims``);
    per grid a background of eps 1 with 16 boxes of eps ~ U[1, 12.25] (sides 4
    to n/2) and an Ez dipole at the centre (seed + grid index)."""
    out = []
    for q in range(nsims):
        rng = np.random.default_rng(seed + q)
        shape = tuple(int(rng.choice(np.arange(dims[0], dims[1] + 1, 16))) for _ in range(3))
        eps = paint_boxes(shape, 16, 4, tuple(max(4, s // 2) for s in shape), 1.0,
                          lambda r: float(r.uniform(1.0, 12.25)), rng)
        wave = gaussian_sine(nsteps, 0.5, eps_bg=1.0)
        out.append(Workload("c4_member_%d_%dx%dx%d" % ((q,) + shape), shape, (PEC, PEC, PEC), 0.5,
                            1.0, nsteps, eps, None, [dipole(EZ, *(s // 2 for s in shape), wave)]))
    return out


def bare_bones(n, seed: int = 6, nsteps: int = 100, shape=None) -> Workload:
    """Fig. 1-style sweep point: C2-style boxes, fields U(-1, 1), PEC walls, no
    sources (the paper's 'bare-bones' setup has none)."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    n_boxes = max(1, int(round(40 * (shape[0] * shape[1] * shape[2]) / 256 ** 3)))
    return random_dielectric(shape, (PEC, PEC, PEC), n_boxes, seed, nsteps,
                             side=(max(1, min(shape) // 32), max(2, min(shape) // 4)),
                             noise=1.0, name="bare_bones_%dx%dx%d" % shape)


def small_case(shape, bc, seed: int, nsteps: int, n_boxes: int = 6, noise: float = 0.1,
               dipoles: Sequence[Tuple[int, int, int]] = (), eps_box_range=(1.0, 12.25)) -> Workload:
    """Small parity case: random per-box permittivity, random fields, optional dipoles."""
    rng = np.random.default_rng(seed)
    side_hi = tuple(max(1, s // 2) for s in shape)
    eps = paint_boxes(shape, n_boxes, 1, side_hi, 2.08,
                      lambda r: float(r.uniform(*eps_box_range)), rng)
    f = [rng.uniform(-noise, noise, size=shape).astype(np.float32) for _ in range(6)]
    zero_pec(f, bc)
    wave = gaussian_sine(max(nsteps, 1), 0.5)
    sources = [dipole(EZ, *p, wave) for p in dipoles]
    return Workload("small_%dx%dx%d_seed%d" % (tuple(shape) + (seed,)), tuple(shape), tuple(bc),
                    0.5, 1.0, nsteps, eps, tuple(f), sources)


def graded_shell(shape, thickness: int = 16, sigma_max: float = 0.4) -> np.ndarray:
    """Conductivity of a simple absorbing layer: zero inside, growing as the
    square of the depth into a shell of ``thickness`` cells along every wall
    up to ``sigma_max`` at the wall (one FP32 array for all three E
    components).  Built plane by plane, so a full-size grid needs no
    temporaries of its own size."""
    nx, ny, nz = (int(s) for s in shape)
    dist = [np.minimum(np.arange(n), n - 1 - np.arange(n)).astype(np.int32) for n in (nx, ny, nz)]
    dyz = np.minimum(dist[1][:, None], dist[2][None, :])
    ramp = np.where(np.arange(thickness + 1) < thickness,
                    sigma_max * ((thickness - np.arange(thickness + 1)) / thickness) ** 2,
                    0.0).astype(np.float32)
    out = np.empty((nx, ny, nz), np.float32)
    for i in range(nx):
        d = np.minimum(dyz, dist[0][i])
        out[i] = ramp[np.minimum(d, thickness)]
    return out
