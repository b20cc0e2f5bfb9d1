"""FP64 forward Yee runs in plain torch, batched (test infrastructure only).

Finite differences of the full-size inverse-design objective need sixteen
FP64 forward runs of 256x256x128 cells, which the CPU oracle would take many
minutes for.  This module runs them together on the device with elementwise
torch operations: each IEEE double operation is its own kernel, rounded once,
never contracted, and the operations come in the order of the oracle's FP64
step (Section 2, Eq. (1) and its cyclic permutations, sources after the E
half-step, then H from the new E; the monitor transform of the adjoint
oracle).  A GPU test checks the fields against the C oracle bit for bit and
the objective against the adjoint oracle on small grids, so these runs are
the oracle's arithmetic, only placed elsewhere.  Nothing here touches the HIP
library.

Shapes: every field tensor is [B, nx, ny, nz] float64, one row per run.
"""
import math

import numpy as np
import torch


def pec_mask(shape, bc, comp):
    m = np.zeros(shape, bool)
    for a in range(3):
        if a != comp and bc[a] == 0:
            sl = [slice(None)] * 3
            sl[a] = 0
            m[tuple(sl)] = True
    return m


def coefficients(eps_list, bc, dt, dx, device):
    """cE_c = dt / (eps_c dx) in double per run, 0 on PEC-tangential index-0
    planes.  eps_list[b][c]: float64 numpy arrays (run b, component c)."""
    out = []
    for c in range(3):
        rows = []
        for eps in eps_list:
            v = dt / (np.asarray(eps[c], np.float64) * dx)
            v[pec_mask(v.shape, bc, c)] = 0.0
            rows.append(torch.from_numpy(v))
        out.append(torch.stack(rows).to(device))
    return out


def _bwd(a, axis):
    return torch.roll(a, 1, dims=axis + 1)


def _fwd(a, axis):
    return torch.roll(a, -1, dims=axis + 1)


def forward_J(eps_list, bc, dt, dx, nsteps, mon_lo, mon_hi, comp, omega, sources, device="cuda:0"):
    """J_b = sum_r |F_b(r)|^2 for every run b (zero initial fields), with
    F(r) = sum_{n=1..N} E_comp^n(r) exp(-i omega n dt) over the monitor box.
    Returns (J as a float64 numpy array, final fields)."""
    shape = eps_list[0][0].shape
    B = len(eps_list)
    cE = coefficients(eps_list, bc, dt, dx, device)
    cH = dt / dx
    f = [torch.zeros((B,) + tuple(shape), dtype=torch.float64, device=device) for _ in range(6)]
    mb = (slice(None),) + tuple(slice(a, b) for a, b in zip(mon_lo, mon_hi))
    Fr = torch.zeros_like(f[comp][mb])
    Fi = torch.zeros_like(f[comp][mb])
    for n in range(1, nsteps + 1):
        Ex, Ey, Ez, Hx, Hy, Hz = f
        ex = (Ex + cE[0] * (Hz - _bwd(Hz, 1))) - cE[0] * (Hy - _bwd(Hy, 2))
        ey = (Ey + cE[1] * (Hx - _bwd(Hx, 2))) - cE[1] * (Hz - _bwd(Hz, 0))
        ez = (Ez + cE[2] * (Hy - _bwd(Hy, 0))) - cE[2] * (Hx - _bwd(Hx, 1))
        f[0], f[1], f[2] = ex, ey, ez
        s = n - 1
        for q in sources:
            m = s - q.get("first_step", 0)
            if 0 <= m < len(q["waveform"]):
                a = f[q["comp"]]
                a[:, q["i"], q["j"], q["k"]] = a[:, q["i"], q["j"], q["k"]] + float(np.float32(q["waveform"][m]))
        Ex, Ey, Ez = f[0], f[1], f[2]
        hx = (Hx - cH * (_fwd(Ez, 1) - Ez)) + cH * (_fwd(Ey, 2) - Ey)
        hy = (Hy - cH * (_fwd(Ex, 2) - Ex)) + cH * (_fwd(Ez, 0) - Ez)
        hz = (Hz - cH * (_fwd(Ey, 0) - Ey)) + cH * (_fwd(Ex, 1) - Ex)
        f[3], f[4], f[5] = hx, hy, hz
        ph = complex(np.exp(-1j * omega * n * dt))
        x = f[comp][mb]
        Fr = Fr + x * ph.real
        Fi = Fi + x * ph.imag
    J = (Fr * Fr + Fi * Fi).sum(dim=(1, 2, 3))
    return J.cpu().numpy(), f
