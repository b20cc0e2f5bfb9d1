"""CPU oracle for the adjoint (reverse-time) Yee solver -- test infrastructure only.

Only the test suite may import this module; the product library never loads
it.  Everything here is FP64 numpy, written for clarity, not speed.  The
forward steps are the oracle's C update (``oracle.step``); the adjoint steps
are written here from the transposes of the two half-step maps.

Objective (the frequency-domain monitor of the inverse-design setting the
paper motivates in Section 1):

    F(r) = sum_{n=1..N} E_c^n(r) exp(-i w n dt)      for r in the monitor box
    J    = sum_r |F(r)|^2

where E^n is the E field after step n of the run (after the E half-step and
the sources) and c is the monitored E component.

Forward step n as linear maps (sources are an additive term that does not
depend on the permittivity):

    E^n       = E^{n-1} + cE (.) CH(H^{n-1/2})     (E half-step, backward differences)
    H^{n+1/2} = H^{n-1/2} - cH CE(E^n)             (H half-step, forward differences)

with CH the curl of the E update and CE the curl of the H update (both with
periodic index arithmetic; PEC is cE = 0 on the tangential index-0 planes).
Reverse step n, for the adjoint variables lE (of E) and lH (of H):

    lE += dJ/dE^n                                    (monitor samples of step n)
    lE -= cH CE^T(lH)                                (through the H half-step)
    g  += lE (.) CH(H^{n-1/2})                        (dJ/dcE, through the E half-step)
    lH += CH^T(cE (.) lE)

starting from lE = lH = 0 after the last step; g accumulates dJ/dcE.  With
cE = dt / (eps dx), dJ/deps = -g cE / eps (zero where cE is pinned to 0).

With conductivity sigma (the semi-implicit conductive E half-step of the
oracle's lossy step), the E half-step is

    E^n = A (.) E^{n-1} + B (.) CH(H^{n-1/2}),
    A = (1 - h) / (1 + h),  B = (dt / (eps dx)) / (1 + h),  h = sigma dt / (2 eps),

so the reverse step gains the decay of the adjoint E and a second sum:

    lE += dJ/dE^n
    lE -= cH CE^T(lH)
    gB += lE (.) CH(H^{n-1/2});   gA += lE (.) E^{n-1}
    lH += CH^T(B (.) lE)
    lE  = A (.) lE                                  (adjoint of E^{n-1})

and, sigma held fixed, dJ/deps = gA dA/deps + gB dB/deps with
dA/deps = 2 h / (eps (1 + h)^2) and dB/deps = -B / (eps (1 + h)) (zero on the
PEC-pinned entries, where A = 1 and B = 0 do not depend on eps).
"""
from __future__ import annotations

import numpy as np

import oracle

EX, EY, EZ = 0, 1, 2


def _bwd(a, axis):
    """a[i] - a[i-1] (periodic index)."""
    return a - np.roll(a, 1, axis=axis)


def _fwd(a, axis):
    """a[i+1] - a[i] (periodic index)."""
    return np.roll(a, -1, axis=axis) - a


def _bwd_T(b, axis):
    """Transpose of _bwd: (a[i] - a[i-1])^T b = b[i] - b[i+1]."""
    return b - np.roll(b, -1, axis=axis)


def _fwd_T(b, axis):
    """Transpose of _fwd: (a[i+1] - a[i])^T b = b[i-1] - b[i]."""
    return np.roll(b, 1, axis=axis) - b


def curl_h(H):
    """CH(H): the differences of the E half-step (x, y, z components)."""
    Hx, Hy, Hz = H
    return (_bwd(Hz, 1) - _bwd(Hy, 2), _bwd(Hx, 2) - _bwd(Hz, 0), _bwd(Hy, 0) - _bwd(Hx, 1))


def curl_h_T(L):
    """CH^T(L): maps an E-shaped adjoint to an H-shaped one."""
    Lx, Ly, Lz = L
    # CH_x = bwd_y(Hz) - bwd_z(Hy); CH_y = bwd_z(Hx) - bwd_x(Hz); CH_z = bwd_x(Hy) - bwd_y(Hx)
    hx = _bwd_T(Ly, 2) - _bwd_T(Lz, 1)
    hy = _bwd_T(Lz, 0) - _bwd_T(Lx, 2)
    hz = _bwd_T(Lx, 1) - _bwd_T(Ly, 0)
    return (hx, hy, hz)


def curl_e_T(L):
    """CE^T(L): maps an H-shaped adjoint to an E-shaped one."""
    Lx, Ly, Lz = L
    # CE_x = fwd_y(Ez) - fwd_z(Ey); CE_y = fwd_z(Ex) - fwd_x(Ez); CE_z = fwd_x(Ey) - fwd_y(Ex)
    ex = _fwd_T(Ly, 2) - _fwd_T(Lz, 1)
    ey = _fwd_T(Lz, 0) - _fwd_T(Lx, 2)
    ez = _fwd_T(Lx, 1) - _fwd_T(Ly, 0)
    return (ex, ey, ez)


def adjoint_step(lE, lH, cE, cH):
    """Transpose of one source-free forward step (E half-step, then H half-step):
    given the adjoints of (E^n, H^{n+1/2}) return those of (E^{n-1}, H^{n-1/2})."""
    t = curl_e_T(lH)
    lE = tuple(e - cH * d for e, d in zip(lE, t))
    u = curl_h_T(tuple(c * e for c, e in zip(cE, lE)))
    lH = tuple(h + d for h, d in zip(lH, u))
    return lE, lH


def adjoint_step_lossy(lE, lH, ca, cb, cH):
    """Transpose of one source-free conductive forward step (E half-step with
    decay ca and curl coefficient cb, then the H half-step)."""
    t = curl_e_T(lH)
    lE = tuple(e - cH * d for e, d in zip(lE, t))
    u = curl_h_T(tuple(b * e for b, e in zip(cb, lE)))
    lH = tuple(h + d for h, d in zip(lH, u))
    lE = tuple(a * e for a, e in zip(ca, lE))
    return lE, lH


def _box(lo, hi):
    return tuple(slice(a, b) for a, b in zip(lo, hi))


def forward_dft(fields, cE, cH, nsteps, mon_lo, mon_hi, comp, omega, dt, step0=0, sources=(),
                keep_h=None, ca=None):
    """Run nsteps FP64 steps (one oracle call per step) from a copy of ``fields``.

    With ``ca`` given the step is the conductive one, ``cE`` then being its
    curl coefficient cb.  Returns (F, final fields, kept), F being the complex
    monitor transform; if ``keep_h`` is a box (lo, hi), kept[n-1] holds
    CH(H^{n-1/2}) over that box, followed by E^{n-1} there when ``ca`` is
    given."""
    f = tuple(np.array(a, dtype=np.float64, order="C", copy=True) for a in fields)
    mb = _box(mon_lo, mon_hi)
    F = np.zeros(f[comp][mb].shape, np.complex128)
    kept = []
    for n in range(1, nsteps + 1):
        if keep_h is not None:
            kb = _box(*keep_h)
            rec = [c[kb].copy() for c in curl_h(f[3:])]
            if ca is not None:
                rec += [e[kb].copy() for e in f[:3]]
            kept.append(tuple(rec))
        if ca is None:
            oracle.step(cE, cH, f, 1, step0=step0 + n - 1, sources=sources, dtype=np.float64)
        else:
            oracle.step_lossy(ca, cE, cH, f, 1, step0=step0 + n - 1, sources=sources,
                              dtype=np.float64)
        F += f[comp][mb] * np.exp(-1j * omega * n * dt)
    return F, f, kept


def _coefficients(eps, bc, dt, dx, sigma):
    """(ca or None, curl coefficient) of the forward step, FP64."""
    if sigma is None:
        return None, oracle.coeff_E(eps, bc, dt, dx)
    return oracle.coeff_lossy(eps, sigma, bc, dt, dx)


def objective(fields, eps, bc, dt, dx, nsteps, mon_lo, mon_hi, comp, omega, step0=0, sources=(),
              sigma=None):
    """J = sum |F|^2 of an FP64 forward run (conductive when ``sigma`` is given)."""
    ca, cE = _coefficients(eps, bc, dt, dx, sigma)
    F, _, _ = forward_dft(fields, cE, dt / dx, nsteps, mon_lo, mon_hi, comp, omega, dt,
                          step0, sources, ca=ca)
    return float(np.sum(np.abs(F) ** 2))


def gradient(fields, eps, bc, dt, dx, nsteps, mon_lo, mon_hi, comp, omega, des_lo, des_hi,
             step0=0, sources=(), sigma=None):
    """(J, dJ/deps_c over the design box for c = x, y, z) by the adjoint method,
    FP64; with ``sigma`` (three conductivity arrays, held fixed) the forward
    run is the conductive one."""
    ca, cE = _coefficients(eps, bc, dt, dx, sigma)
    lossy = ca is not None
    cH = dt / dx
    shape = fields[0].shape
    F, _, _ = forward_dft(fields, cE, cH, nsteps, mon_lo, mon_hi, comp, omega, dt, step0, sources,
                          ca=ca)
    J = float(np.sum(np.abs(F) ** 2))
    # CH(H^{n-1/2}) (and E^{n-1} when conductive) is needed over the whole grid
    # by the reverse sweep's gradient terms, but only its design-box part is kept
    db = _box(des_lo, des_hi)
    _, _, kept = forward_dft(fields, cE, cH, nsteps, mon_lo, mon_hi, comp, omega, dt, step0,
                             sources, keep_h=(des_lo, des_hi), ca=ca)
    mb = _box(mon_lo, mon_hi)
    lE = tuple(np.zeros(shape) for _ in range(3))
    lH = tuple(np.zeros(shape) for _ in range(3))
    g = [np.zeros(kept[0][0].shape) for _ in range(3)]    # dJ/dcE, or dJ/dB
    gA = [np.zeros(kept[0][0].shape) for _ in range(3)]   # dJ/dA (conductive)
    for n in range(nsteps, 0, -1):
        # dJ/dE_c^n(r) = 2 Re(conj(F(r)) exp(-i w n dt)) on the monitor box
        lE = tuple(np.array(a) for a in lE)
        lE[comp][mb] += 2.0 * np.real(np.conj(F) * np.exp(-1j * omega * n * dt))
        t = curl_e_T(lH)
        lE = tuple(e - cH * d for e, d in zip(lE, t))
        for c in range(3):
            g[c] += lE[c][db] * kept[n - 1][c]
            if lossy:
                gA[c] += lE[c][db] * kept[n - 1][3 + c]
        u = curl_h_T(tuple(cc * e for cc, e in zip(cE, lE)))
        lH = tuple(h + d for h, d in zip(lH, u))
        if lossy:
            lE = tuple(a * e for a, e in zip(ca, lE))
    grad = []
    for c in range(3):
        ce = cE[c][db]
        e = np.asarray(eps[c], np.float32).astype(np.float64)[db]
        if not lossy:
            grad.append(np.where(ce != 0.0, -g[c] * ce / e, 0.0))
            continue
        sg = np.asarray(sigma[c], np.float32).astype(np.float64)[db]
        h = sg * dt / (2.0 * e)
        dA = 2.0 * h / (e * (1.0 + h) ** 2)
        dB = -ce / (e * (1.0 + h))
        grad.append(np.where(ce != 0.0, gA[c] * dA + g[c] * dB, 0.0))
    return J, tuple(grad)
