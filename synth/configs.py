"""Seeded workloads: the small parity scene and camera helpers.

``make_config(1)`` is the plain forward workload: one static octree of 4096
leaves (levels 3-6) in a 1 m cube centred at the origin, built from the 512
level-3 cells by exactly 512 random subdivisions; one raw density per shared
grid corner drawn N(0,1); SH degree 0 with the DC coefficient drawn
U(-1.75, 1.75) per channel (so the rendered colour spans roughly (0,1));
one 128x96 pinhole camera with a 60 degree horizontal field of view placed
2.5 m from the centre, black background, no actors.

The driving-shaped workloads (1M-8M leaves, box cars on lanes) live in
``synth.driving``.
"""
import numpy as np

from .octree import full_grid, random_subdivide, dedup_corners, make_octree


def look_at_c2w(eye, target, up=(0.0, 0.0, 1.0)):
    """Camera-to-world 3x4 with OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r = r / np.linalg.norm(r)
    dn = np.cross(f, r)
    c2w = np.zeros((3, 4))
    c2w[:, 0], c2w[:, 1], c2w[:, 2], c2w[:, 3] = r, dn, f, eye
    return c2w


def make_view(W, H, fov_h_deg, c2w, t=0.0, window=None):
    """Pinhole view; principal point at the image centre, fx = fy."""
    fx = (W / 2.0) / np.tan(np.deg2rad(fov_h_deg) / 2.0)
    x0, y0, w, h = window if window is not None else (0, 0, W, H)
    return dict(fx=float(fx), fy=float(fx), cx=W / 2.0, cy=H / 2.0,
                W=int(W), H=int(H), x0=int(x0), y0=int(y0), w=int(w),
                h=int(h), c2w=np.asarray(c2w, np.float64).copy(),
                t=float(t))


def _sh_random(rng, n, degree, dc_half=1.75, hi_std=0.1):
    s = (degree + 1) ** 2
    sh = np.empty((s, 3, n), np.float32)
    sh[0] = rng.uniform(-dc_half, dc_half, (3, n))
    if s > 1:
        sh[1:] = rng.normal(0.0, hi_std, (s - 1, 3, n))
    return sh


def config1(seed=1):
    rng = np.random.default_rng(seed)
    lv, ijk = full_grid(3)
    lv, ijk = random_subdivide(lv, ijk, 512, 6, rng)
    assert lv.shape[0] == 4096
    cidx, upos = dedup_corners(lv, ijk, 6)
    dens = rng.normal(0.0, 1.0, upos.shape[0]).astype(np.float32)
    sh = _sh_random(rng, lv.shape[0], 0)
    bg = make_octree(root_min=(-0.5, -0.5, -0.5), root_size=1.0,
                     max_level=6, level=lv, ijk=ijk, corner_idx=cidx,
                     corner_density=dens, sh=sh)
    a, e = np.deg2rad(30.0), np.deg2rad(20.0)
    eye = 2.5 * np.array([np.cos(a) * np.cos(e), np.sin(a) * np.cos(e),
                          np.sin(e)])
    view = make_view(128, 96, 60.0, look_at_c2w(eye, (0.0, 0.0, 0.0)))
    scene = dict(octrees=[bg], tracks=[None])
    opts = dict(K=1, eps_stop=1e-4, tau_near=0.0, bg=(0.0, 0.0, 0.0),
                explin_c=1.1)
    return dict(name="static-4096-128x96", scene=scene, views=[view],
                opts=opts)


def make_config(k, seed=None, **kw):
    """Workload k in 1..5 (seed defaults to k)."""
    seed = k if seed is None else seed
    if k == 1:
        return config1(seed)
    from . import driving
    return driving.make_driving_config(k, seed, **kw)
