"""Independent mathematics used to pin the oracle (test code only).

Nothing here calls the oracle's stencil code.  The discrete curl operators
are assembled from 1D periodic difference matrices with Kronecker products
(the textbook construction of the Yee curl on a staggered grid); divergences
and the leapfrog energy are written against those operators or with numpy
shifts.  Arrays are C-ordered [nx, ny, nz] (z fastest), so a flat index is
(i*ny + j)*nz + k.
"""
import numpy as np
import scipy.sparse as sp

PEC, PERIODIC = 0, 1


def _dback(n):
    """(D f)[i] = f[i] - f[i-1 mod n]  (backward difference, periodic)."""
    I = sp.identity(n, format="csr")
    P = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) - 1) % n)), shape=(n, n))
    return (I - P).tocsr()


def _dfwd(n):
    """(D f)[i] = f[i+1 mod n] - f[i]  (forward difference, periodic)."""
    I = sp.identity(n, format="csr")
    P = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
    return (P - I).tocsr()


def axis_ops(shape, d1):
    nx, ny, nz = shape
    Ix, Iy, Iz = (sp.identity(n, format="csr") for n in shape)
    Dx = sp.kron(sp.kron(d1(nx), Iy), Iz).tocsr()
    Dy = sp.kron(sp.kron(Ix, d1(ny)), Iz).tocsr()
    Dz = sp.kron(sp.kron(Ix, Iy), d1(nz)).tocsr()
    return Dx, Dy, Dz


def curl(shape, d1):
    """Block curl [[0,-Dz,Dy],[Dz,0,-Dx],[-Dy,Dx,0]] built from difference d1."""
    Dx, Dy, Dz = axis_ops(shape, d1)
    Z = sp.csr_matrix(Dx.shape)
    return sp.bmat([[Z, -Dz, Dy], [Dz, Z, -Dx], [-Dy, Dx, Z]]).tocsr()


def curl_h(shape):
    """Curl applied to H in the E update (backward differences)."""
    return curl(shape, _dback)


def curl_e(shape):
    """Curl applied to E in the H update (forward differences)."""
    return curl(shape, _dfwd)


def pec_frozen_mask(shape, bc):
    """Flat boolean mask (length 3N) of E entries frozen at +0 by PEC walls."""
    masks = []
    for c in range(3):
        m = np.zeros(shape, dtype=bool)
        for a in range(3):
            if a != c and bc[a] == PEC:
                sl = [slice(None)] * 3
                sl[a] = 0
                m[tuple(sl)] = True
        masks.append(m.ravel())
    return np.concatenate(masks)


def div_back(F):
    """Backward-difference divergence of a 3-component field (periodic shifts)."""
    return ((F[0] - np.roll(F[0], 1, axis=0)) + (F[1] - np.roll(F[1], 1, axis=1))
            + (F[2] - np.roll(F[2], 1, axis=2)))


def div_fwd(F):
    """Forward-difference divergence of a 3-component field (periodic shifts)."""
    return ((np.roll(F[0], -1, axis=0) - F[0]) + (np.roll(F[1], -1, axis=1) - F[1])
            + (np.roll(F[2], -1, axis=2) - F[2]))


def interior_mask(shape, bc):
    """Cells whose index is >= 1 along every PEC axis."""
    m = np.ones(shape, dtype=bool)
    for a in range(3):
        if bc[a] == PEC:
            sl = [slice(None)] * 3
            sl[a] = 0
            m[tuple(sl)] = False
    return m


def leapfrog_energy(fields, eps, bc, dt, dx=1.0):
    """Q = sum eps|E|^2 + sum |H|^2 + (dt/dx) * E . (C_h H), over non-frozen E.

    With E update E += (dt/(eps dx)) C_h H and H update H -= (dt/dx) C_e E and
    C_e = C_h^T, this is <eps E^n, E^n> + <H^{n+1/2}, H^{n-1/2}>, which the
    leapfrog conserves exactly in exact arithmetic."""
    shape = fields[0].shape
    E = np.concatenate([f.astype(np.float64).ravel() for f in fields[:3]])
    H = np.concatenate([f.astype(np.float64).ravel() for f in fields[3:]])
    ep = np.concatenate([np.asarray(e, np.float64).ravel() for e in eps])
    live = ~pec_frozen_mask(shape, bc)
    CH = curl_h(shape) @ H
    return float(np.sum(ep[live] * E[live] ** 2) + np.sum(H * H)
                 + (dt / dx) * np.sum(E[live] * CH[live]))


def rel_l2(a_fields, b_fields):
    num = sum(float(np.sum((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
              for a, b in zip(a_fields, b_fields))
    den = sum(float(np.sum(np.asarray(b, np.float64) ** 2)) for b in b_fields)
    return (num / den) ** 0.5
