"""Host-side logic that needs no GPU: launch shapes and the seeded inputs.

* ``tuning.launch_for`` always returns a workgroup of 256 or 512 threads (the
  sizes the bulk kernels are instantiated for), row-wide 2-row tiles on 128-
  and 256-wide lattices, the widest of 256, 128, 64, 32 and 16 that divides nx
  otherwise, and graph replay only for lattices of at most 2^22 nodes;
* the workload generators are deterministic in their seed, and the benchmark's
  256 x 256 x 128 spreading lattice has the fluid and solid counts its JSON
  line reports;
* ``bench.py`` refuses a run on more than one GPU before it touches a device.
"""
import os
import subprocess
import sys

import numpy as np

from paper_2607_25444_amd import tuning, workloads as W


def test_launch_for_sizes_and_shapes():
    for nx in list(range(8, 600, 4)) + [96, 100, 192, 513]:
        bx, by, bz, graph, phase = tuning.launch_for((nx, 64, 64))
        assert bx * by * bz in (256, 512), (nx, bx, by, bz)
        assert phase == 0
        if nx in (128, 256):
            assert (bx, by, bz) == (nx, 2, 1)
        else:
            div = [b for b in (256, 128, 64, 32, 16) if nx % b == 0]
            if div:
                assert bx == div[0], (nx, bx)
    assert tuning.launch_for((512, 512, 512))[:3] == (256, 2, 1)
    assert tuning.launch_for((192, 192, 768))[:3] == (64, 8, 1)
    assert tuning.launch_for((96, 96, 96))[:3] == (32, 4, 2)
    assert tuning.launch_for((128, 128, 256))[3] == 1  # 2^22 nodes
    assert tuning.launch_for((128, 128, 257))[3] == 0


def test_workloads_are_seeded():
    a, b = W.sessile((24, 20, 16), 5.0, 60.0), W.sessile((24, 20, 16), 5.0, 60.0)
    for k in ("solid", "theta", "phi0"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
    s0, s0b, s1 = W.spreading_256(0), W.spreading_256(0), W.spreading_256(1)
    np.testing.assert_array_equal(s0.phi0, s0b.phi0)
    np.testing.assert_array_equal(s0.theta, s0b.theta)
    assert not np.array_equal(s0.phi0, s1.phi0) or not np.array_equal(s0.theta, s1.theta)


def test_spreading_256_counts():
    w = W.spreading_256(0)
    assert w.shape == (256, 256, 128) and w.N == 256 * 256 * 128
    assert int((w.solid == 0).sum()) == 8257536
    assert int((w.solid != 0).sum()) == 131072
    fl = w.solid == 0
    assert np.all((w.phi0[fl] >= 0.0) & (w.phi0[fl] <= 1.0))


def test_bench_refuses_more_than_one_gpu():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    bench = os.path.join(root, "bench.py")
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, bench, *argv], capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, **env))
        assert r.returncode == 2, r.stderr
        assert "one GPU" in r.stderr
        assert r.stdout == ""
