"""P15: the soft density prior of the initialisation (Sec. 3.3, Eq. 1) and
the nearest-point distance it is fed with, pinned against the closed form
at its special points and against geometry with known distances.  The
generator's copy (``synth.driving.soft_prior``) is held to the same values.
"""
import math

import numpy as np
import pytest

from oracle import prior as PR
from synth import driving as DRV

S = 0.2                      # minimum voxel size of the driving scenes


def _both():
    return [lambda d, s: PR.soft_prior(d, s),
            lambda d, s: DRV.soft_prior(d, s, -2.0)]


@pytest.mark.parametrize("f", _both())
def test_prior_special_points(f):
    # d = 0: v_close = -2 (the paper's value)
    assert f(0.0, S) == -2.0
    # d = s: v_far + (v_close - v_far) e^-2 = -10 + 8 e^-2
    assert abs(f(S, S) - (-10.0 + 8.0 * math.exp(-2.0))) < 1e-14
    # d = s / 2: -10 + 8 e^-1/2
    assert abs(f(S / 2, S) - (-10.0 + 8.0 * math.exp(-0.5))) < 1e-14
    # far away: v_far = -10
    assert f(10.0, S) == -10.0
    assert abs(f(1.0, S) + 10.0) < 1e-19 + 8.0 * math.exp(-50.0)


@pytest.mark.parametrize("f", _both())
def test_prior_monotone_between_bounds(f):
    d = np.linspace(0.0, 1.0, 1001)
    v = f(d, S)
    assert np.all(np.diff(v) <= 0.0)
    assert np.all((v <= -2.0) & (v >= -10.0))
    # symmetric in the sign of d (it enters squared) and scale-free in d/s
    assert np.allclose(f(-d, S), v, atol=0, rtol=0)
    assert np.allclose(f(3 * d, 3 * S), v, atol=1e-14)


def test_prior_opaque_variant_matches_closed_form():
    # the opaque (trained-like) variant replaces v_close by +10
    d = np.array([0.0, 0.1, 0.2, 0.5])
    ref = np.array([-10.0 + 20.0 * math.exp(-2.0 * x * x / S ** 2) for x in d])
    assert np.allclose(DRV.soft_prior(d, S, 10.0), ref, atol=1e-14, rtol=0)
    assert np.allclose(PR.soft_prior(d, S, v_close=10.0), ref, atol=1e-14,
                       rtol=0)


def test_nearest_distance_known_geometry():
    # points on the integer lattice {0..4}^3: a query's distance is that to
    # the nearest lattice point inside the cube, known in closed form
    g = np.stack(np.meshgrid(*[np.arange(5.0)] * 3, indexing="ij"), -1)
    pts = g.reshape(-1, 3)
    q = np.array([[0.5, 0.5, 0.5], [2.0, 2.0, 2.0], [2.1, 3.0, 1.0],
                  [-1.0, 0.0, 0.0], [5.0, 5.0, 5.0], [0.25, 4.5, 2.0]])
    ref = np.array([math.sqrt(0.75), 0.0, 0.1, 1.0, math.sqrt(3.0),
                    math.sqrt(0.25 ** 2 + 0.5 ** 2)])
    assert np.allclose(PR.nearest_distance_bruteforce(pts, q), ref,
                       atol=1e-15)


def test_nearest_distance_matches_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    pts = rng.uniform(-3, 3, (500, 3))
    q = rng.uniform(-4, 4, (200, 3))
    d_ref, _ = cKDTree(pts).query(q, k=1)
    assert np.allclose(PR.nearest_distance_bruteforce(pts, q), d_ref,
                       atol=1e-14)
