"""Hand-built tiny scenes for pins and parity edge cases."""
import numpy as np

from synth.octree import make_octree, dedup_corners, full_grid, random_subdivide
from synth.configs import make_view, look_at_c2w

Y00 = 0.5 / np.sqrt(np.pi)


def dc_for_colour(rgb):
    """SH DC coefficient giving colour ``rgb`` (independent of the oracle)."""
    return (np.asarray(rgb, np.float64) - 0.5) / Y00


def octree_private(root_min, size, max_level, leaves, g8, sh, box=None):
    """Octree whose leaves own private corners: leaves [(l,i,j,k)],
    g8 [N,8], sh [S,3,N]."""
    leaves = np.asarray(leaves, np.int64).reshape(-1, 4)
    n = leaves.shape[0]
    lv = leaves[:, 0].astype(np.uint8)
    ijk = leaves[:, 1:].T.astype(np.int32)
    cidx = np.arange(8 * n, dtype=np.int32).reshape(n, 8).T.copy()
    dens = np.asarray(g8, np.float32).reshape(n, 8).ravel()
    kw = {}
    if box is not None:
        kw = dict(box_min=box[0], box_max=box[1])
    return make_octree(root_min, size, max_level, lv, ijk, cidx, dens,
                       np.asarray(sh, np.float32).reshape(-1, 3, n), **kw)


def empty_octree(root_min=(0, 0, 0), size=1.0, max_level=1, deg=0):
    s = (deg + 1) ** 2
    return make_octree(root_min, size, max_level, np.zeros(0, np.uint8),
                       np.zeros((3, 0), np.int32), np.zeros((8, 0), np.int32),
                       np.zeros(0, np.float32), np.zeros((s, 3, 0), np.float32))


def random_octree(rng, root_min, size, base_level, n_sub, max_level, deg,
                  g_mean=0.0, g_std=1.0, box=None, shared=True):
    lv, ijk = full_grid(base_level)
    lv, ijk = random_subdivide(lv, ijk, n_sub, max_level, rng)
    n = lv.shape[0]
    if shared:
        cidx, upos = dedup_corners(lv, ijk, max_level)
        dens = rng.normal(g_mean, g_std, upos.shape[0]).astype(np.float32)
    else:
        cidx = np.arange(8 * n, dtype=np.int32).reshape(n, 8).T.copy()
        dens = rng.normal(g_mean, g_std, 8 * n).astype(np.float32)
    s = (deg + 1) ** 2
    sh = np.empty((s, 3, n), np.float32)
    sh[0] = rng.uniform(-1.75, 1.75, (3, n))
    if s > 1:
        sh[1:] = rng.normal(0, 0.3, (s - 1, 3, n))
    kw = {}
    if box is not None:
        kw = dict(box_min=box[0], box_max=box[1])
    return make_octree(root_min, size, max_level, lv, ijk, cidx, dens, sh, **kw)


def static_track(yaw, p, t0=-1e3, t1=1e3):
    return dict(t=np.array([t0, t1]), yaw=np.array([yaw, yaw]),
                trans=np.array([p, p], np.float64))


def moving_track(yaw0, yaw1, p0, p1, t0=0.0, t1=10.0):
    return dict(t=np.array([t0, t1]), yaw=np.array([yaw0, yaw1]),
                trans=np.array([p0, p1], np.float64))


def actor_scene(seed=0, n_actors=2, deg=1, overlap=False, K=1, bg_levels=(2, 24, 4),
                fov=60.0, target=(0.0, 0.0, 0.0)):
    """Small background cube [-2,2]^3 with two or three actor cubes of side
    1 inside the view; useful for parity and gradient pins.  The default
    view shows actor leaves of about one pixel; a narrow ``fov`` aimed at an
    actor (``target``) shows them several pixels wide."""
    rng = np.random.default_rng(seed)
    b0, nsub, lmax = bg_levels
    bg = random_octree(rng, (-2.0, -2.0, -2.0), 4.0, b0, nsub, lmax, deg,
                       g_mean=-1.0, g_std=1.0)
    octs = [bg]
    tracks = [None]
    centres = [(-0.6, 0.3, 0.113), (0.7, -0.4, -0.187), (0.1, 0.2, 0.521)]
    if overlap:
        centres = [(-0.2, 0.1, 0.013), (0.2, 0.0, 0.117), (0.1, 0.2, 0.521)]
    for i in range(n_actors):
        a = random_octree(rng, (-0.5, -0.5, -0.5), 1.0, 2, 10, 4, deg,
                          g_mean=0.5, g_std=1.5,
                          box=((-0.45, -0.4, -0.35), (0.45, 0.4, 0.35)))
        octs.append(a)
        c = np.array(centres[i])
        tracks.append(moving_track(0.2 + 0.3 * i, 0.5 + 0.3 * i, c, c + (0.3, 0.1, 0.0)))
    eye = np.array([3.0, 1.5, 1.2])
    view = make_view(64, 48, fov, look_at_c2w(eye, target), t=2.5)
    opts = dict(K=K, eps_stop=0.0, tau_near=0.0, bg=(0.1, 0.2, 0.3),
                explin_c=1.1)
    return dict(scene=dict(octrees=octs, tracks=tracks), views=[view],
                opts=opts)


def dense_scene(seed=0, n_actors=2, level=5, deg=1, actor_level=None,
                overlap=False):
    """Background cube [-2,2]^3 fully tiled by (2^level)^3 leaves of low
    density (rays cross all of them), with actor cubes inside: a small view
    whose tile lists exceed the compositing chunk length, so long lists are
    split into chunks that are merged back."""
    rng = np.random.default_rng(seed)
    bg = random_octree(rng, (-2.0, -2.0, -2.0), 4.0, level, 0, level, deg,
                       g_mean=-2.5, g_std=0.7)
    octs = [bg]
    tracks = [None]
    centres = [(-0.6, 0.3, 0.113), (0.7, -0.4, -0.187), (0.1, 0.2, 0.521)]
    if overlap:
        centres = [(-0.2, 0.1, 0.013), (0.2, 0.0, 0.117), (0.1, 0.2, 0.521)]
    for i in range(n_actors):
        if actor_level is None:
            a = random_octree(rng, (-0.5, -0.5, -0.5), 1.0, 2, 10, 4, deg,
                              g_mean=0.5, g_std=1.5,
                              box=((-0.45, -0.4, -0.35), (0.45, 0.4, 0.35)))
        else:
            # fully tiled asset, density varying from empty to opaque:
            # long (tile, actor) lists
            a = random_octree(rng, (-0.5, -0.5, -0.5), 1.0, actor_level, 0,
                              actor_level, deg, g_mean=-0.5, g_std=1.5,
                              box=((-0.45, -0.4, -0.35), (0.45, 0.4, 0.35)))
        octs.append(a)
        c = np.array(centres[i])
        tracks.append(moving_track(0.2 + 0.3 * i, 0.5 + 0.3 * i, c, c + (0.3, 0.1, 0.0)))
    eye = np.array([4.2, 2.1, 1.7])
    view = make_view(64, 48, 50.0, look_at_c2w(eye, (0.0, 0.0, 0.0)), t=2.5)
    opts = dict(K=1, eps_stop=0.0, tau_near=0.0, bg=(0.1, 0.2, 0.3),
                explin_c=1.1)
    return dict(scene=dict(octrees=octs, tracks=tracks), views=[view],
                opts=opts)


def crowd_scene(seed=0, n_actors=12, deg=1, W=32, H=32):
    """Many small actor boxes stacked along the view direction (spaced
    closer than their depth, so neighbours overlap): the central tiles hold
    every box, for the segment builders' many-box paths."""
    rng = np.random.default_rng(seed)
    bg = random_octree(rng, (-2.0, -2.0, -2.0), 4.0, 2, 10, 4, deg,
                       g_mean=-1.5, g_std=1.0)
    octs = [bg]
    tracks = [None]
    eye = np.array([3.0, 1.5, 1.2])
    fwd = -eye / np.linalg.norm(eye)
    for i in range(n_actors):
        a = random_octree(rng, (-0.15, -0.15, -0.15), 0.3, 1, 4, 3, deg,
                          g_mean=1.0, g_std=1.0,
                          box=((-0.13, -0.12, -0.1), (0.13, 0.12, 0.1)))
        octs.append(a)
        c = 0.5 * fwd + (i * 0.6 / max(n_actors, 1)) * fwd + rng.normal(0, 0.03, 3)
        tracks.append(static_track(0.4 * i, c))
    view = make_view(W, H, 12.0, look_at_c2w(eye, (0.0, 0.0, 0.0)), t=1.0)
    opts = dict(K=1, eps_stop=0.0, tau_near=0.0, bg=(0.1, 0.2, 0.3),
                explin_c=1.1)
    return dict(scene=dict(octrees=octs, tracks=tracks), views=[view],
                opts=opts)
