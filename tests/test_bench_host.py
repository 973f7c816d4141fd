"""Host logic of bench.py that needs no GPU: the one-GPU refusal and the choice of the
bundles on which the mixed and FP64 runs are compared."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _grid(side):
    """Row-major grid indices as stand-in directions: theta[0] = column, theta[1] = row."""
    j = np.arange(side * side)
    return np.stack([j % side, j // side]).astype(float)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr


def test_nfw_default_band_is_the_halo_core():
    th, c0, c1, stride = bench.central_band(_grid(256), 7168, 7168)
    rows = th[1]
    assert (c0, c1, stride) == (114 * 256, 142 * 256 - 1, 1)
    assert rows.min() == 114 and rows.max() == 141 and th.shape[1] == 7168
    assert np.any((th[0] == 128) & (th[1] == 128))          # the centre bundle


def test_strided_sample_spans_the_band():
    th, c0, c1, stride = bench.central_band(_grid(512), 28672, 504)
    assert stride == 56 and th.shape[1] == 504
    assert th[1].min() == 228 and th[1].max() == 283         # 56 rows centred on row 256
    assert np.all(np.diff(th[1] * 512 + th[0]) == 56)


def test_band_larger_than_the_grid_takes_the_whole_grid():
    th, c0, c1, stride = bench.central_band(_grid(128), 28672, 1024)
    assert (c0, c1, stride) == (0, 128 * 128 - 1, 16)
    assert th.shape[1] == 1024 and th[1].min() == 0 and th[1].max() == 127
