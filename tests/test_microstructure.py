"""Seeded input generators: the block-drawn Boolean model equals the
one-draw-at-a-time definition (same SplitMix64 sequence, same voxel test)."""
import math

import numpy as np
import pytest

from microstructure import SplitMix64, _stamp_spheres, boolean_spheres


def _boolean_scalar(shape, radius, fraction, seed):
    nz, ny, nx = shape
    rng = SplitMix64(seed)
    theta = -math.log(1.0 - fraction) / (4.0 * math.pi * radius ** 3 / 3.0)
    count = rng.poisson(theta * nx * ny * nz)
    centers = np.array([[rng.uniform() * nx, rng.uniform() * ny, rng.uniform() * nz] for _ in range(count)])
    return _stamp_spheres(shape, centers.reshape(-1, 3), [radius] * count), centers, rng.state


@pytest.mark.parametrize("shape,r,f,seed", [((32, 32, 32), 3.0, 0.2, 11), ((24, 32, 48), 3.0, 0.3, 12),
                                           ((48, 48, 48), 7.3, 0.4, 5), ((16, 16, 16), 2.5, 0.25, 40),
                                           ((12, 8, 16), 4.0, 0.3, 3)])
def test_block_drawn_boolean_model_equals_the_scalar_definition(shape, r, f, seed):
    ph, info = boolean_spheres(shape, r, f, seed)
    ref, centers, _ = _boolean_scalar(shape, r, f, seed)
    assert info.n_spheres == len(centers)
    assert np.array_equal(info.centers.reshape(-1, 3), centers.reshape(-1, 3))
    assert np.array_equal(ph, ref)


def test_uniform_array_and_poisson_fast_consume_the_same_sequence():
    a, b = SplitMix64(123), SplitMix64(123)
    assert np.array_equal(a.uniform_array(1000), np.array([b.uniform() for _ in range(1000)]))
    for mean in (0.5, 7.0, 300.0, 5000.0):
        assert a.poisson_fast(mean) == b.poisson(mean)
        assert a.state == b.state


@pytest.mark.parametrize("shape,n,seed", [((16, 12, 20), 30, 4), ((24, 24, 24), 64, 9), ((8, 32, 16), 5, 1)])
def test_kd_tree_voronoi_equals_the_brute_force_labelling(shape, n, seed):
    from microstructure import voronoi_cells, voronoi_cells_fast

    a, sa, pa = voronoi_cells(shape, n, 3, seed)
    b, sb, pb = voronoi_cells_fast(shape, n, 3, seed, workers=1)
    assert np.array_equal(sa, sb) and np.array_equal(pa, pb)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,n,seed", [((16, 12, 20), 30, 4), ((12, 8, 16), 7, 2)])
def test_torch_voronoi_equals_the_brute_force_labelling(shape, n, seed):
    torch = pytest.importorskip("torch")
    from microstructure import voronoi_cells, voronoi_cells_torch

    a, sa, pa = voronoi_cells(shape, n, 3, seed)
    b, sb, pb = voronoi_cells_torch(shape, n, 3, seed, device="cpu", rows=5)
    assert np.array_equal(sa, sb) and np.array_equal(pa, pb)
    assert np.array_equal(a, b.numpy())
