"""Soft density prior of Sec. 3.3 (Eq. 1), used to pin the generators.

Each grid corner at distance d from its nearest LiDAR point gets
v = v_far + (v_close - v_far) exp(-2 d^2 / s^2), s the minimum voxel size;
the paper sets v_close = -2 and v_far = -10.
"""
import numpy as np

V_CLOSE = -2.0
V_FAR = -10.0


def soft_prior(d, s, v_close=V_CLOSE, v_far=V_FAR):
    d = np.asarray(d, np.float64)
    return v_far + (v_close - v_far) * np.exp(-2.0 * d * d / (s * s))


def nearest_distance_bruteforce(points, queries):
    """Exact nearest-point distance by brute force (small inputs only)."""
    points = np.asarray(points, np.float64)
    out = np.empty(len(queries))
    for i, q in enumerate(np.asarray(queries, np.float64)):
        out[i] = np.sqrt(((points - q) ** 2).sum(1).min())
    return out
