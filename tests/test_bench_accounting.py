"""CPU checks of the bench's accounting: the transform count behind the
I_3 flop figure (20 complex P x P transforms per node pair, 18 per lone
node, 18 per node unpaired), the convergence metric of the validation
study, and the refusal of more than one GPU."""
import math
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_i3_transform_and_flop_counts():
    assert bench.i3_transforms(32, 64, True) == 32 * 32 * 20
    assert bench.i3_transforms(32, 64, False) == 32 * 64 * 18
    assert bench.i3_transforms(6, 5, True) == 6 * (2 * 20 + 18)  # two pairs and the middle node
    n = 128 * 128
    assert math.isclose(bench.i3_flops(256, 64, 32, 64, True), 256 * 20480 * 5.0 * n * math.log2(n))
    # the slab launch in float32: 6.01e12 flop
    assert math.isclose(bench.i3_flops(256, 64, 32, 64, True), 6.013e12, rel_tol=1e-3)


def test_i3_algorithmic_count_and_io():
    """The method's own count: 36 unpacked transforms per (j, m) (4 shifts,
    16 convolutions of two transforms), 2.16e13 flop for the slab launch;
    the kernel's minimum traffic: 21 P x P fields per cell."""
    n = 128 * 128
    assert math.isclose(bench.i3_flops_algorithmic(256, 64, 32, 64), 256 * 36 * 32 * 64 * 5.0 * n * math.log2(n))
    assert math.isclose(bench.i3_flops_algorithmic(256, 64, 32, 64), 2.164e13, rel_tol=1e-3)
    # pairing and packing save 36 * 2 / 20 = 3.6x against the method's count
    assert math.isclose(bench.i3_flops_algorithmic(1, 64, 32, 64) / bench.i3_flops(1, 64, 32, 64, True), 3.6)
    assert bench.i3_io_bytes(256, 64, 32, 4) == 256 * 21 * 128 * 128 * 4


def _fake_components(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4, N, N))


def test_convergence_metric():
    c = _fake_components(16, 0)
    assert bench.rel_l1(c, c) == 0.0
    # scaling the error scales the metric linearly; four components add
    d = 1e-3 * _fake_components(16, 1)
    e1, e2 = bench.rel_l1(c + d, c), bench.rel_l1(c + 2 * d, c)
    assert math.isclose(e2, 2 * e1, rel_tol=1e-12)
    # a component that vanishes in the reference is skipped
    z = c.copy()
    z[0] = 0.0
    y = z.copy()
    y[0] = 1e-18
    assert bench.rel_l1(y, z) == 0.0
    # a coarser grid compared with a finer one: common frequencies match
    # exactly for a band-limited field, so only the reference's extra
    # coefficients count (none here)
    N, M = 8, 16
    x = np.arange(M) - M // 2
    f = np.cos(2 * np.pi * 2 * x / M)[:, None] * np.ones(M)[None, :]
    fine = np.stack([f] * 4)
    xc = np.arange(N) - N // 2
    fc = np.cos(2 * np.pi * 2 * xc / N)[:, None] * np.ones(N)[None, :]
    coarse = np.stack([fc] * 4)
    assert bench.rel_l1(coarse, fine) < 1e-14


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
