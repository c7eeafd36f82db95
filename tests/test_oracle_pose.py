"""Pins of the oracle's actor pose (Sec. 3.2, reading R17: yaw about world
+z and translation, each linear in t between keyframes, active on the
closed range of the track) against hand-computed values."""
import math

import numpy as np
import pytest

from oracle import geometry as G

TRACK = dict(t=np.array([0.0, 1.0, 3.0]),
             yaw=np.array([0.0, math.pi / 2, math.pi / 2]),
             trans=np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0],
                             [2.0, 4.0, 1.0]]))

S = math.sqrt(0.5)


@pytest.mark.parametrize("t, R, p", [
    # at the first keyframe
    (0.0, [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [0, 0, 0]),
    # half way to the second key: yaw pi/4, p half of (2, 0, 0)
    (0.5, [[S, -S, 0], [S, S, 0], [0, 0, 1]], [1, 0, 0]),
    # a quarter of the way: yaw pi/8
    (0.25, [[math.cos(math.pi / 8), -math.sin(math.pi / 8), 0],
            [math.sin(math.pi / 8), math.cos(math.pi / 8), 0], [0, 0, 1]],
     [0.5, 0, 0]),
    # exactly at the middle keyframe
    (1.0, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], [2, 0, 0]),
    # second interval (length 2): t = 2 is half way, yaw constant
    (2.0, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], [2, 2, 0.5]),
    (2.5, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], [2, 3, 0.75]),
    # the last keyframe is still active
    (3.0, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], [2, 4, 1]),
])
def test_pose_hand_computed(t, R, p):
    act, Rg, pg = G.pose_at(TRACK, t)
    assert act
    assert np.allclose(Rg, np.array(R, float), atol=1e-15, rtol=0)
    assert np.allclose(pg, np.array(p, float), atol=1e-15, rtol=0)


@pytest.mark.parametrize("t", [-1e-9, -0.5, 3.0 + 1e-9, 10.0])
def test_pose_outside_range_inactive(t):
    act, _, _ = G.pose_at(TRACK, t)
    assert not act


def test_pose_maps_local_to_world():
    # x_world = R x_local + p: the actor's local +x axis points along world
    # +y once yawed by pi/2 (counter-clockwise about +z)
    act, R, p = G.pose_at(TRACK, 1.0)
    xw = R @ np.array([1.0, 0.0, 0.0]) + p
    assert np.allclose(xw, [2.0, 1.0, 0.0], atol=1e-15)
    # a point on the +z axis only moves with the translation
    assert np.allclose(R @ np.array([0, 0, 5.0]) + p, [2, 0, 5], atol=1e-15)


def test_single_key_track_active_only_at_its_time():
    tr = dict(t=np.array([2.0]), yaw=np.array([math.pi]),
              trans=np.array([[1.0, 2.0, 3.0]]))
    act, R, p = G.pose_at(tr, 2.0)
    assert act
    assert np.allclose(R, [[-1, 0, 0], [0, -1, 0], [0, 0, 1]], atol=1e-15)
    assert np.allclose(p, [1, 2, 3])
    assert not G.pose_at(tr, 2.0 + 1e-12)[0]
    assert not G.pose_at(tr, 2.0 - 1e-12)[0]


def test_pose_is_rigid_and_continuous():
    rng = np.random.default_rng(3)
    tr = dict(t=np.cumsum(rng.uniform(0.1, 1.0, 6)),
              yaw=rng.uniform(-3, 3, 6), trans=rng.normal(size=(6, 3)))
    for k in range(1, 5):
        tk = tr["t"][k]
        _, Ra, pa = G.pose_at(tr, tk - 1e-10)
        _, Rb, pb = G.pose_at(tr, tk)
        assert np.allclose(Ra, Rb, atol=1e-8) and np.allclose(pa, pb, atol=1e-8)
    for t in np.linspace(tr["t"][0], tr["t"][-1], 17):
        _, R, _ = G.pose_at(tr, t)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
