"""Geometry in FP64: voxel boxes, camera rays, ray-box slabs, actor poses.

Sec. 3.1: a leaf at level l with integer cell ijk inside a root cube
(min corner w, side s) occupies [w + ijk*h, w + (ijk+1)*h], h = s / 2^l.
Sec. 3.2: an actor's pose T_t^i maps its local frame to the world,
x_world = R x_local + p; rays are taken to the local frame by the inverse.
"""
import numpy as np


def voxel_boxes(o):
    """All leaves of octree ``o``: (vmin f64[N,3], h f64[N])."""
    h = o["root_size"] / np.exp2(o["level"].astype(np.float64))
    vmin = o["root_min"][None, :] + o["ijk"].T.astype(np.float64) * h[:, None]
    return vmin, h


def camera_ray(view, px, py):
    """Ray through the centre of image pixel (px, py) (reading: pinhole,
    OpenCV axes, unit direction, tau = Euclidean distance)."""
    dcam = np.array([(px + 0.5 - view["cx"]) / view["fx"],
                     (py + 0.5 - view["cy"]) / view["fy"], 1.0])
    R = view["c2w"][:, :3]
    d = R @ dcam
    return view["c2w"][:, 3].copy(), d / np.linalg.norm(d)


def slab(o, d, bmin, bmax):
    """Exact ray/AABB interval [t_enter, t_exit] for the line o + t d.

    Returns (t_enter, t_exit, ax_enter, ax_exit); an empty interval has
    t_exit < t_enter.  Axes with d == 0 constrain only by containment."""
    lo, hi = -np.inf, np.inf
    ax_lo, ax_hi = -1, -1
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < bmin[a] or o[a] > bmax[a]:
                return np.inf, -np.inf, -1, -1
            continue
        t0 = (bmin[a] - o[a]) / d[a]
        t1 = (bmax[a] - o[a]) / d[a]
        if t0 > t1:
            t0, t1 = t1, t0
        if t0 > lo:
            lo, ax_lo = t0, a
        if t1 < hi:
            hi, ax_hi = t1, a
    return lo, hi, ax_lo, ax_hi


def slab_many(o, d, vmin, vmax):
    """Vectorised ``slab`` over boxes: (t0, t1, ax0, ax1) arrays."""
    n = vmin.shape[0]
    lo = np.full(n, -np.inf)
    hi = np.full(n, np.inf)
    ax_lo = np.full(n, -1, np.int64)
    ax_hi = np.full(n, -1, np.int64)
    for a in range(3):
        if d[a] == 0.0:
            out = (o[a] < vmin[:, a]) | (o[a] > vmax[:, a])
            lo = np.where(out, np.inf, lo)
            hi = np.where(out, -np.inf, hi)
            continue
        t0 = (vmin[:, a] - o[a]) / d[a]
        t1 = (vmax[:, a] - o[a]) / d[a]
        tn, tf = np.minimum(t0, t1), np.maximum(t0, t1)
        up = tn > lo
        lo = np.where(up, tn, lo)
        ax_lo = np.where(up, a, ax_lo)
        dn = tf < hi
        hi = np.where(dn, tf, hi)
        ax_hi = np.where(dn, a, ax_hi)
    return lo, hi, ax_lo, ax_hi


def yaw_matrix(yaw):
    c, s = np.cos(yaw), np.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def pose_at(track, t):
    """Reading of Sec. 3.2 for the synthetic tracks: yaw about world +z and
    translation, each linear in t between keyframes; the actor is active
    iff t lies in [t_first, t_last].  Returns (active, R, p)."""
    ts = np.asarray(track["t"], np.float64)
    if t < ts[0] or t > ts[-1]:
        return False, np.eye(3), np.zeros(3)
    k = int(np.searchsorted(ts, t, side="right") - 1)
    k = min(max(k, 0), len(ts) - 1)
    if k == len(ts) - 1:
        yaw, p = track["yaw"][k], np.asarray(track["trans"][k], np.float64)
    else:
        f = (t - ts[k]) / (ts[k + 1] - ts[k])
        yaw = track["yaw"][k] + f * (track["yaw"][k + 1] - track["yaw"][k])
        p0 = np.asarray(track["trans"][k], np.float64)
        p1 = np.asarray(track["trans"][k + 1], np.float64)
        p = p0 + f * (p1 - p0)
    return True, yaw_matrix(yaw), np.array(p, np.float64)


def octree_poses(scene, view, pose_override=None):
    """Per octree: (active, R, p).  Octree 0 is the world-frame background
    (identity).  ``pose_override`` (list of (R, p) per actor) replaces the
    track, for pose gradients and finite differences."""
    out = [(True, np.eye(3), np.zeros(3))]
    for i in range(1, len(scene["octrees"])):
        if pose_override is not None and pose_override[i - 1] is not None:
            R, p = pose_override[i - 1]
            out.append((True, np.asarray(R, np.float64),
                        np.asarray(p, np.float64)))
        else:
            out.append(pose_at(scene["tracks"][i], view["t"]))
    return out


def actor_box(o):
    """The actor's interval box in its local frame: the box given with the
    octree, else its root cube (reading of Sec. 3.3 'Assets' / Sec. 3.4)."""
    if "box_min" in o:
        return o["box_min"], o["box_max"]
    lo = o["root_min"]
    return lo, lo + o["root_size"]
