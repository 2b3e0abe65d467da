"""Host helpers of bench.py: the exact lattice-voxel count of the swept balls
(the paper's metric normalises by (4/3) pi R^3; the exact count is reported
beside it)."""
import itertools

import numpy as np
import pytest

import bench


def _brute(R, N):
    neg, pos = (N // 2, N // 2 - 1) if N % 2 == 0 else ((N - 1) // 2, (N - 1) // 2)
    rsq = int(np.floor(float(R) * float(R)))
    rng = range(-neg, pos + 1)
    return sum(1 for i, j, k in itertools.product(rng, rng, rng) if i * i + j * j + k * k <= rsq)


@pytest.mark.parametrize("R,count", [(15.0, 14147), (20.0, 33401), (30.0, 113081)])
def test_ball_lattice_counts(R, count):
    assert bench.lattice_voxels(np.array([R], np.float32), 250) == count


@pytest.mark.parametrize("N", [7, 8, 19, 20])
def test_lattice_counts_clipped_by_the_periodic_extent(N):
    radii = np.array([0.0, 1.0, 2.5, 3.9, 6.0, 11.5, 40.0], np.float32)
    assert bench.lattice_voxels(radii, N) == sum(_brute(r, N) for r in radii)
    assert bench.lattice_voxels(np.array([], np.float32), N) == 0


def test_kernel_hash_ignores_comments_only():
    """The profiles' kernel hash covers what the compiler sees: comments and
    whitespace do not change it, code and string literals do."""
    import bench
    a = "int f(int x) { return x + 1; } // one\n/* two */"
    b = "int  f(int x)\n{\n  // other words\n  return x + 1;   /* c */\n}"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(a.replace("+ 1", "+ 2"))
    assert bench._code_only('s = "// not a comment";') == 's="// not a comment";'
