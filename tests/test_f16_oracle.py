"""Pins of the FP16-storage oracle (oracle/f16.py) against what the binary16
format and the mathematics fix, independent of the oracle's own code:

- the conversion is the IEEE binary16 round-to-nearest-even of the format's
  definition (nearest of all finite binary16 values, ties to the even
  significand, overflow to infinity from the midpoint above 65504 on);
- power-of-two scales are exact: scaling a linear run's inputs by 2^k with
  the storage exponents raised by k scales every stored value by 2^k;
- one band covering the whole call reduces to the FP32 oracle rounded at the
  ends, and splitting a call into calls of whole bands changes nothing;
- the accuracy bar (relative L2 <= 2e-3 against FP64 after 1000 steps, the
  FP64 run using the same dequantised coefficients) holds for the systolic
  rounding schedule and fails for the plain one (rounding every half-step),
  and both errors follow the random-walk growth of independent roundings.
"""
import bisect
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import f16
from paper_2502_20610_amd import workloads as wl
from tests import yee_math as ym

PEC, PER = 0, 1
# every finite non-negative binary16 value, in increasing order
_POS16 = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float64)


def _nearest16(x: float) -> float:
    """Round-to-nearest-even onto binary16 from the format's definition."""
    if x != x:
        return x
    s = -1.0 if np.signbit(x) else 1.0
    a = abs(x)
    if a >= 65520.0:            # 65504 + half an ulp (2^5 / 2): overflows
        return s * np.inf
    if a > 65504.0:             # below the midpoint: the largest finite value
        return s * 65504.0
    i = bisect.bisect_left(_POS16.tolist(), a)
    if i < len(_POS16) and _POS16[i] == a:
        return s * a
    lo, hi = _POS16[i - 1], _POS16[i]
    dl, dh = Fraction(a) - Fraction(lo), Fraction(hi) - Fraction(a)
    if dl < dh:
        r = lo
    elif dh < dl:
        r = hi
    else:                        # tie: the even significand (even bit pattern)
        r = lo if (i - 1) % 2 == 0 else hi
    return s * r


def test_binary16_rounding_matches_the_definition():
    rng = np.random.default_rng(1)
    vals = list(rng.standard_normal(400) * 10.0 ** rng.integers(-9, 6, 400))
    vals += [1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2.0 ** -25, 3 * 2.0 ** -25, 2.0 ** -26,
             65504.0, 65519.0, 65520.0, 1e6, 6.103515625e-05, 6.0e-05, 5.96e-08, 2.9e-08,
             -0.0, 0.0, -1.0 - 2.0 ** -11, 0.1, 1.0 / 3.0]
    x32 = np.asarray(vals, np.float32)
    got = f16.quantize(x32).astype(np.float64)
    for x, g in zip(x32.astype(np.float64), got):
        ref = _nearest16(float(x))
        assert (g == ref and np.signbit(g) == np.signbit(ref)) or (np.isnan(g) and np.isnan(ref)), (x, g, ref)


def test_power_of_two_scales_are_exact():
    rng = np.random.default_rng(2)
    v = (rng.standard_normal(1000) * 3.0).astype(np.float32)
    for e, k in [(0, 5), (-3, 7), (4, -6)]:
        a = f16.store(v * np.float32(2.0 ** k), e + k)
        b = f16.store(v, e) * np.float32(2.0 ** k)
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def _case(shape, bc, seed, n):
    w = wl.small_case(shape, bc, seed=seed, nsteps=n, noise=1.0)
    cE = f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)
    return w, cE, np.float32(w.dt / w.dx)


def test_scaled_storage_scales_the_run_exactly():
    """No sources: the Yee step is linear, so inputs times 2^k with every
    storage exponent raised by k give every stored value times 2^k, bit for
    bit (a scale missed on a load or a store would break this)."""
    w, cE, cH = _case((12, 10, 9), (PEC, PER, PEC), 3, 30)
    k = 6
    base = f16.run_systolic(w.fields, cE, cH, [30], [7], exp2=(0,) * 6)
    scaled = f16.run_systolic([f * np.float32(2.0 ** k) for f in w.fields], cE, cH, [30], [7],
                              exp2=(k,) * 6)
    for a, b in zip(scaled, base):
        np.testing.assert_array_equal(a.view(np.uint32), (b * np.float32(2.0 ** k)).view(np.uint32))
    pb = f16.run_plain(w.fields, cE, cH, 12, exp2=(0, 1, 2, 3, 4, 5))
    ps = f16.run_plain([f * np.float32(2.0 ** k) for f in w.fields], cE, cH, 12,
                       exp2=tuple(k + e for e in (0, 1, 2, 3, 4, 5)))
    for a, b in zip(ps, pb):
        np.testing.assert_array_equal(a.view(np.uint32), (b * np.float32(2.0 ** k)).view(np.uint32))


def test_one_band_is_the_fp32_run_rounded_and_bands_split_freely():
    w = wl.small_case((11, 13, 10), (PEC, PEC, PEC), seed=4, nsteps=24, dipoles=[(5, 6, 5)])
    cE = f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)
    cH = np.float32(w.dt / w.dx)
    one = f16.run_systolic(w.fields, cE, cH, [24], [64], sources=w.sources)
    ref = [f16.store(f) for f in w.fields]
    oracle.step(cE, cH, ref, 24, sources=w.sources, dtype=np.float32)
    for a, b in zip(one, ref):
        np.testing.assert_array_equal(a.view(np.uint32), f16.store(b).view(np.uint32))
    whole = f16.run_systolic(w.fields, cE, cH, [24], [8], sources=w.sources)
    split = f16.run_systolic(w.fields, cE, cH, [8, 16], [8, 8], sources=w.sources)
    for a, b in zip(whole, split):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    # every stored value is a binary16 value
    for a in whole:
        np.testing.assert_array_equal(f16.store(a), a)


def test_plain_rounds_after_each_half_step_and_source():
    w = wl.small_case((9, 8, 7), (PEC, PEC, PEC), seed=5, nsteps=3, dipoles=[(4, 4, 3)])
    cE = f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)
    got = f16.run_plain(w.fields, cE, np.float32(0.5), 3, sources=w.sources)
    for a in got:
        np.testing.assert_array_equal(f16.store(a), a)
    # one step by hand: E half-step, round, source, round, H half-step, round
    f = [f16.store(x).copy() for x in w.fields]
    oracle.half_E(cE, f)
    f[:3] = [f16.store(x) for x in f[:3]]
    s = w.sources[0]
    f[2][4, 4, 3] = f16.store(np.float32(f[2][4, 4, 3]) + np.float32(s["waveform"][0]))
    oracle.half_H(np.float32(0.5), f)
    f[3:] = [f16.store(x) for x in f[3:]]
    one = f16.run_plain(w.fields, cE, np.float32(0.5), 1, sources=w.sources)
    for a, b in zip(one, f):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.fixture(scope="module")
def dielectric_box():
    """32^3 dielectric PEC box with a dipole (the shape of the paper's
    workloads at a size the FP64 oracle runs in seconds), 1000 steps."""
    w = wl.random_dielectric((32, 32, 32), (PEC, PEC, PEC), 6, 31, 1000, side=(4, 12),
                             dipoles=[(16, 16, 16)])
    cE16 = f16.coeff_E16(w.eps3(), w.bc, w.dt, w.dx)
    x0 = w.fields_or_zeros()
    ref = {}
    for n in (250, 1000):
        f = [np.array(x, np.float64) for x in x0]
        oracle.step([c.astype(np.float64) for c in cE16], w.dt / w.dx, f, n, sources=w.sources,
                    dtype=np.float64)
        ref[n] = f
    return w, cE16, x0, ref


def test_accuracy_bar_and_random_walk_growth(dielectric_box):
    w, cE16, x0, ref = dielectric_box
    cH = np.float32(w.dt / w.dx)
    err = {}
    for n in (250, 1000):
        sy = f16.run_systolic(x0, cE16, cH, [n], [48], sources=w.sources)
        pl = f16.run_plain(x0, cE16, cH, n, sources=w.sources)
        err[n] = (ym.rel_l2(sy, ref[n]), ym.rel_l2(pl, ref[n]))
    # the bar: systolic schedule within 2e-3 after 1000 steps, plain not
    assert err[1000][0] <= 2e-3, err
    assert err[1000][1] > 2e-3, err
    # rounding every ~0.5 step against every 48 steps: the errors scale
    # roughly as the square root of the number of roundings (factor ~10)
    assert 4 < err[1000][1] / err[1000][0] < 25, err
    # and grow with the run
    assert err[1000][0] > err[250][0] and err[1000][1] > err[250][1], err
