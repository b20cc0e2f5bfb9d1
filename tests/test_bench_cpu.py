"""Host-side logic of bench.py: the algorithmic byte count, the counter-summary
lookup and the single-GPU contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_systolic_bytes_per_update():
    # x and y faces: E, H in and out (48 B) + the coefficient read (12 B);
    # z face: E, H and the coefficient in and out (72 B); band: 60 B / K
    assert bench.systolic_bytes_per_update((15, 15, 15), 32) == pytest.approx(
        (2 * 225 * 60 + 225 * 72) / 3375 + 60 / 32)          # 12.8 + 1.875
    assert bench.systolic_bytes_per_update((31, 15, 15), 64) == pytest.approx(
        ((225 + 465) * 60 + 465 * 72) / 6975 + 60 / 64)
    # conductive: 11-wide tile along x, ca read with cE and carried on the z ring
    assert bench.systolic_bytes_per_update((11, 15, 15), 16, True) == pytest.approx(
        ((225 + 165) * 72 + 165 * 96) / (11 * 15 * 15) + 72 / 16)
    # FP16 storage: all faces through the rings in FP32 (72 B per face cell),
    # the band's state in binary16 (E, H out and in, cE in: 30 B)
    assert bench.systolic_bytes_per_update((15, 15, 15), 48, fp16=True) == pytest.approx(
        3 * 225 * 72 / 3375 + 30 / 48)
    # the headline launch (15^3 tile, 64-step bands): 12.8 + 0.9375
    assert bench.systolic_bytes_per_update((15, 15, 15), 64) == pytest.approx(13.7375)
    # the plain two-launch scheme moves 84 B per update, the fused step 60 B
    # (E, H and cE in, E and H out)
    assert bench.PLAIN_BYTES_PER_UPDATE == 84
    assert bench.PLAIN_FUSED_BYTES_PER_UPDATE == 60


def test_systolic_algorithmic_bytes_follow_the_face_and_band_formula():
    """(in + out) A/V + (out + in)/K with in = E, H and the coefficients (36 B
    in FP32), out = E and H (24 B): 12 + 60/K at the 15^3 tile."""
    assert bench.systolic_alg_bytes_per_update((15, 15, 15), 20) == pytest.approx(12.0 + 3.0)
    assert bench.systolic_alg_bytes_per_update((15, 15, 15), 64) == pytest.approx(12.0 + 60 / 64)
    # material indices: a cell's coefficients enter as its 4-byte index (in = 28 B)
    assert bench.systolic_alg_bytes_per_update((15, 15, 15), 20, materials=True) == pytest.approx(
        52 * 0.2 + 52 / 20)
    # this design with indices: x and y faces read the index, the z face keeps the values
    assert bench.systolic_bytes_per_update((15, 15, 15), 20, materials=True) == pytest.approx(
        (2 * 225 * 52 + 225 * 72) / 3375 + 52 / 20)
    # the 19-wide tile: A = 225 + 285 + 285, V = 4275; its z face carries the
    # index (4 B) instead of the three coefficient values
    assert bench.systolic_alg_bytes_per_update((19, 15, 15), 20, materials=True) == pytest.approx(
        52 * 795 / 4275 + 52 / 20)
    assert bench.systolic_bytes_per_update((19, 15, 15), 20, materials=True) == pytest.approx(
        (510 * 52 + 285 * 56) / 4275 + 52 / 20)
    # the paper's 31x15x15 block: A = 225 + 465 + 465
    assert bench.systolic_alg_bytes_per_update((31, 15, 15), 64) == pytest.approx(
        60 * 1155 / 6975 + 60 / 64)
    # conductive: ca travels with cE (in = 48 B)
    assert bench.systolic_alg_bytes_per_update((11, 15, 15), 16, True) == pytest.approx(
        72 * (225 + 165 + 165) / (11 * 15 * 15) + 72 / 16)
    # FP16 storage halves every stored element
    assert bench.systolic_alg_bytes_per_update((15, 15, 15), 48, fp16=True) == pytest.approx(
        30 * 0.2 + 30 / 48)
    # never more than the design's own exchange
    for k in (8, 20, 64):
        assert bench.systolic_alg_bytes_per_update((15, 15, 15), k) < \
            bench.systolic_bytes_per_update((15, 15, 15), k)


def test_counter_traffic_needs_matching_source_and_launch():
    launch = {"workload": "c3_pec_dielectric_1024x1024x512", "steps": 128, "band": 32,
              "cells": 1024 * 1024 * 512}
    src = "paper_2502_20610_amd/csrc/systolic.hip"
    t = bench.counter_traffic("systolic_kernel", src, launch)
    if t is not None:   # the committed summary matches this source
        assert t > 0
    assert bench.counter_traffic("systolic_kernel", src, dict(launch, steps=7)) is None
    assert bench.counter_traffic("systolic_kernel", src, dict(launch, band=16)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
