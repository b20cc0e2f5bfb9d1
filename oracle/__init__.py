"""CPU oracle for the 3D Yee FDTD leapfrog update -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library (the HIP path) never
loads it and shares no code with it.

The arithmetic lives in ``yee_oracle.c`` (plain C, compiled with
``-ffp-contract=off``; see that file's header for the update equations and
the passages of the paper they follow).  This module only compiles it and
marshals numpy arrays through ctypes.

Functions
---------
coeff_E(eps, bc, dt, dx)           -> (cEx, cEy, cEz) in float64
coeff_lossy(eps, sigma, bc, dt, dx) -> ((caX, caY, caZ), (cbX, cbY, cbZ)) in float64
step(cE, cH, fields, nsteps, ...)  -> advances six fields in place (f64 or f32)
step_lossy(ca, cb, cH, fields, ...) -> the same with conductivity
half_E(cE, fields), half_H(cH, fields) -> one FP32 half-step in place (no sources)
run(fields, eps, bc, dt, dx, ...)  -> convenience: coefficients + steps (sigma optional)

Field tuples are always ordered (Ex, Ey, Ez, Hx, Hy, Hz); arrays are C-ordered
``[nx, ny, nz]`` (z fastest).  ``bc[a]`` is 0 for PEC and 1 for periodic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "yee_oracle.c")
_LIB = os.path.join(_HERE, "_yee_oracle.so")
_lib = None

PEC, PERIODIC = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle shared library in-tree (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Source(ctypes.Structure):
    _fields_ = [("comp", ctypes.c_int32), ("i", ctypes.c_int32), ("j", ctypes.c_int32),
                ("k", ctypes.c_int32), ("w", ctypes.POINTER(ctypes.c_float)),
                ("len", ctypes.c_int64), ("first_step", ctypes.c_int64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_coeff_E.argtypes = [ctypes.c_int] * 3 + [i32p, ctypes.c_double, ctypes.c_double,
                                                            ctypes.c_int, fp, dp]
        lib.oracle_coeff_E.restype = None
        for name, P, S in (("oracle_step_f64", dp, ctypes.c_double),
                           ("oracle_step_f32", fp, ctypes.c_float)):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int] * 3 + [P, P, P, S] + [P] * 6 + [
                ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Source), ctypes.c_int]
            f.restype = None
        lib.oracle_coeff_lossy.argtypes = [ctypes.c_int] * 3 + [i32p, ctypes.c_double,
                                                                 ctypes.c_double, ctypes.c_int, fp,
                                                                 fp, dp, dp]
        lib.oracle_coeff_lossy.restype = None
        for name, P, S in (("oracle_step_lossy_f64", dp, ctypes.c_double),
                           ("oracle_step_lossy_f32", fp, ctypes.c_float)):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int] * 3 + [P] * 6 + [S] + [P] * 6 + [
                ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Source), ctypes.c_int]
            f.restype = None
        lib.oracle_half_E_f32.argtypes = [ctypes.c_int] * 3 + [fp] * 9
        lib.oracle_half_E_f32.restype = None
        lib.oracle_half_H_f32.argtypes = [ctypes.c_int] * 3 + [ctypes.c_float] + [fp] * 6
        lib.oracle_half_H_f32.restype = None
        lib.oracle_round_f32.argtypes = [dp, fp, ctypes.c_int64]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP thread count the oracle runs with."""
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count for later oracle calls."""
    _load().oracle_set_threads(int(n))


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def coeff_E(eps: Sequence[np.ndarray], bc: Sequence[int], dt: float, dx: float):
    """cE_c = dt/(eps_c*dx) in float64, zero on PEC-tangential index-0 planes."""
    lib = _load()
    nx, ny, nz = eps[0].shape
    bcarr = (ctypes.c_int32 * 3)(*[int(b) for b in bc])
    out = []
    for c in range(3):
        e = np.ascontiguousarray(eps[c], dtype=np.float32)
        o = np.empty((nx, ny, nz), dtype=np.float64)
        lib.oracle_coeff_E(nx, ny, nz, bcarr, float(dt), float(dx), c, _ptr(e, ctypes.c_float),
                           _ptr(o, ctypes.c_double))
        out.append(o)
    return tuple(out)


def coeff_lossy(eps: Sequence[np.ndarray], sigma: Sequence[np.ndarray], bc: Sequence[int],
                dt: float, dx: float):
    """(ca, cb) per component in float64 for conductivity sigma: see yee_oracle.c."""
    lib = _load()
    nx, ny, nz = eps[0].shape
    bcarr = (ctypes.c_int32 * 3)(*[int(b) for b in bc])
    ca, cb = [], []
    for c in range(3):
        e = np.ascontiguousarray(eps[c], dtype=np.float32)
        g = np.ascontiguousarray(sigma[c], dtype=np.float32)
        a = np.empty((nx, ny, nz), dtype=np.float64)
        b = np.empty((nx, ny, nz), dtype=np.float64)
        lib.oracle_coeff_lossy(nx, ny, nz, bcarr, float(dt), float(dx), c,
                               _ptr(e, ctypes.c_float), _ptr(g, ctypes.c_float),
                               _ptr(a, ctypes.c_double), _ptr(b, ctypes.c_double))
        ca.append(a)
        cb.append(b)
    return tuple(ca), tuple(cb)


def round_f32(a: np.ndarray) -> np.ndarray:
    """Round an FP64 array to FP32 (done in the C oracle, round-to-nearest-even)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    o = np.empty(a.shape, dtype=np.float32)
    lib.oracle_round_f32(_ptr(a, ctypes.c_double), _ptr(o, ctypes.c_float), a.size)
    return o


def _sources(sources):
    keep = []
    arr = (_Source * max(1, len(sources)))()
    for q, s in enumerate(sources):
        w = np.ascontiguousarray(s["waveform"], dtype=np.float32)
        keep.append(w)
        arr[q] = _Source(int(s["comp"]), int(s["i"]), int(s["j"]), int(s["k"]),
                         _ptr(w, ctypes.c_float), int(w.size), int(s.get("first_step", 0)))
    return arr, keep


def step(cE, cH, fields, nsteps: int, step0: int = 0, sources=(), dtype=np.float64):
    """Advance ``fields`` (six arrays of ``dtype``) in place by ``nsteps`` Yee steps.

    ``cE`` are three coefficient arrays and ``cH`` a scalar, both used exactly as
    given (in ``dtype``).  ``step0`` is the step count at entry; it selects the
    waveform samples of the sources.
    """
    lib = _load()
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        fn, ct = lib.oracle_step_f64, ctypes.c_double
    elif dtype == np.float32:
        fn, ct = lib.oracle_step_f32, ctypes.c_float
    else:
        raise TypeError("oracle supports float64 and float32 only")
    nx, ny, nz = fields[0].shape
    for a in list(cE) + list(fields):
        if a.dtype != dtype or a.shape != (nx, ny, nz) or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("coefficient and field arrays must be C-contiguous %s of shape %s"
                             % (dtype, (nx, ny, nz)))
    src, keep = _sources(list(sources))
    fn(nx, ny, nz, *[_ptr(c, ct) for c in cE], ct(cH), *[_ptr(f, ct) for f in fields],
       int(nsteps), int(step0), src, len(sources))
    del keep
    return fields


def step_lossy(ca, cb, cH, fields, nsteps: int, step0: int = 0, sources=(), dtype=np.float64):
    """Like :func:`step`, with the conductive E half-step E = (ca E + cb d1) - cb d2."""
    lib = _load()
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        fn, ct = lib.oracle_step_lossy_f64, ctypes.c_double
    elif dtype == np.float32:
        fn, ct = lib.oracle_step_lossy_f32, ctypes.c_float
    else:
        raise TypeError("oracle supports float64 and float32 only")
    nx, ny, nz = fields[0].shape
    for a in list(ca) + list(cb) + list(fields):
        if a.dtype != dtype or a.shape != (nx, ny, nz) or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("coefficient and field arrays must be C-contiguous %s of shape %s"
                             % (dtype, (nx, ny, nz)))
    src, keep = _sources(list(sources))
    fn(nx, ny, nz, *[_ptr(c, ct) for c in ca], *[_ptr(c, ct) for c in cb], ct(cH),
       *[_ptr(f, ct) for f in fields], int(nsteps), int(step0), src, len(sources))
    del keep
    return fields


def _check32(arrays, shape):
    for a in arrays:
        if a.dtype != np.float32 or a.shape != shape or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous float32 of shape %s" % (shape,))


def half_E(cE, fields):
    """One FP32 E half-step in place (the first half of :func:`step`, no sources)."""
    lib = _load()
    nx, ny, nz = fields[0].shape
    _check32(list(cE) + list(fields), (nx, ny, nz))
    fp = ctypes.c_float
    lib.oracle_half_E_f32(nx, ny, nz, *[_ptr(c, fp) for c in cE], *[_ptr(f, fp) for f in fields])
    return fields


def half_H(cH, fields):
    """One FP32 H half-step in place (the second half of :func:`step`)."""
    lib = _load()
    nx, ny, nz = fields[0].shape
    _check32(list(fields), (nx, ny, nz))
    fp = ctypes.c_float
    lib.oracle_half_H_f32(nx, ny, nz, ctypes.c_float(cH), *[_ptr(f, fp) for f in fields])
    return fields


def run(fields, eps, bc, dt: float, dx: float, nsteps: int, step0: int = 0, sources=(),
        dtype=np.float64, sigma=None):
    """Copy ``fields``, build the coefficients from ``eps`` (and the
    conductivity ``sigma``, three arrays, if given) and run ``nsteps``.

    The FP32 variant rounds the FP64 coefficients (and cH = dt/dx) to float,
    as the structural fields of the GPU path are FP32.
    """
    cH = float(dt) / float(dx)
    f32 = np.dtype(dtype) == np.float32
    if f32:
        cH = np.float32(cH)
    out = tuple(np.array(f, dtype=dtype, order="C", copy=True) for f in fields)
    if sigma is not None:
        ca, cb = coeff_lossy(eps, sigma, bc, dt, dx)
        if f32:
            ca = tuple(round_f32(c) for c in ca)
            cb = tuple(round_f32(c) for c in cb)
        return step_lossy(ca, cb, cH, out, nsteps, step0=step0, sources=sources, dtype=dtype)
    cE = coeff_E(eps, bc, dt, dx)
    if f32:
        cE = tuple(round_f32(c) for c in cE)
    return step(cE, cH, out, nsteps, step0=step0, sources=sources, dtype=dtype)
