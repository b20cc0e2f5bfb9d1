"""FP16 field storage (Section 4 stores the field values as 16-bit floats) --
test infrastructure only, like the rest of this package.

The paper states the storage format, not where the rounding happens; that
follows from where each scheme keeps values between steps.  The readings
implemented here (FP32 arithmetic throughout, exactly as the FP32 oracle):

- a stored value of field component c is binary16(v * 2^-e_c), rounded to
  nearest even, and reads back as binary16 * 2^e_c (a power-of-two scale, so
  only the binary16 rounding is inexact);
- cE is stored as binary16 of its FP32 value (the dequantised coefficients
  define the simulated materials; accuracy is judged against an FP64 run with
  the same coefficients);
- plain scheme: the arrays are the only state between kernels, so E is
  rounded after the E half-step, a source cell again after each source is
  added, and H after the H half-step;
- systolic scheme: tiles keep their state in FP32 for a band of K steps and
  exchange faces in FP32, so the grid is rounded once per band (bands are
  counted from the start of each call; the last band of a call may be
  shorter).

The binary16 conversion is numpy's (IEEE round to nearest even, with
subnormals and overflow to infinity); the tests pin it against the format's
definition.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import coeff_E, half_E, half_H, round_f32, step

F32 = np.float32


def quantize(v, e: int = 0) -> np.ndarray:
    """binary16 storage of FP32 values under the scale 2^e."""
    with np.errstate(over="ignore"):
        return (np.asarray(v, np.float32) * F32(2.0 ** -e)).astype(np.float16)


def dequantize(h, e: int = 0) -> np.ndarray:
    return np.asarray(h, np.float16).astype(np.float32) * F32(2.0 ** e)


def store(v, e: int = 0) -> np.ndarray:
    """The FP32 value a stored FP32 value reads back as."""
    return dequantize(quantize(v, e), e)


def coeff_E16(eps: Sequence[np.ndarray], bc, dt: float, dx: float):
    """cE as the FP16-storage path holds it: binary16 of the FP32 coefficient,
    returned dequantised (float32)."""
    return tuple(store(round_f32(c)) for c in coeff_E(eps, bc, dt, dx))


def _store_all(fields, exp2):
    for c in range(6):
        fields[c][...] = store(fields[c], exp2[c])


def run_systolic(fields, cE16, cH: float, calls: Sequence[int], bands: Sequence[int], step0: int = 0,
                 sources=(), exp2=(0,) * 6):
    """Systolic scheme with FP16 storage: the input rounded once, then for
    each call of n steps (band length K of that call) runs of K FP32 steps,
    each followed by the rounding of the whole grid."""
    f = [store(np.asarray(x, np.float32), e).copy() for x, e in zip(fields, exp2)]
    s = step0
    for n, K in zip(calls, bands):
        done = 0
        while done < n:
            k = min(K, n - done)
            step(cE16, F32(cH), f, k, step0=s, sources=sources, dtype=np.float32)
            _store_all(f, exp2)
            s += k
            done += k
    return tuple(f)


def run_plain(fields, cE16, cH: float, nsteps: int, step0: int = 0, sources=(), exp2=(0,) * 6):
    """Plain scheme with FP16 storage: E rounded after the E half-step, each
    source cell after its source is added (in table order), H after the H
    half-step."""
    f = [store(np.asarray(x, np.float32), e).copy() for x, e in zip(fields, exp2)]
    for s in range(step0, step0 + nsteps):
        half_E(cE16, f)
        for c in range(3):
            f[c][...] = store(f[c], exp2[c])
        for src in sources:
            m = s - src.get("first_step", 0)
            w = np.asarray(src["waveform"], np.float32)
            if m < 0 or m >= w.size:
                continue
            c, p = src["comp"], (src["i"], src["j"], src["k"])
            f[c][p] = store(F32(f[c][p]) + w[m], exp2[c])
        half_H(F32(cH), f)
        for c in range(3, 6):
            f[c][...] = store(f[c], exp2[c])
    return tuple(f)
