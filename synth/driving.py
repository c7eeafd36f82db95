"""Driving-shaped synthetic workloads (stand-ins for the paper's PandaSet
scenes: 1920x1080 cameras, a large static background from LiDAR-like
points, rigid box-shaped vehicles on lanes).

Background: a 200 x 200 m ground plane plus random box buildings off a road
cross; LiDAR-like sweeps (64 beams x 1024 azimuths, 100 m range) from ego
positions along the roads give the point cloud.  The octree (root cube
819.2 m) starts from 1.6 m cells over the inner region and is subdivided
near the points toward 0.2 m cells (threshold found by bisection to reach
the leaf budget); a coarse far shell (25.6 m / 51.2 m cells, finer only
where grid alignment needs it) fills the rest above ground.  Corner
densities follow the soft prior of the paper's initialisation section with
s = 0.2 m, v_far = -10 and v_close given (the paper's -2, or +10 for
opaque, trained-like surfaces).  Cars are 4.5 x 1.9 x 1.6 m solid boxes in
a 5.4 m root cube (1.2 x the longest side), subdivided near the box
surface; their tracks are yaw + translation, linear in time, on lanes at
least 8 m apart.
"""
import numpy as np
from scipy.spatial import cKDTree

from .octree import (children, dedup_corners, make_octree, corner_positions,
                     morton_order_leaves, morton_order_corners)
from .configs import make_view, look_at_c2w, _sh_random

ROOT_SIZE = 819.2
ROOT_MIN = np.array([-409.6, -409.6, -409.6])
INNER_LO = np.array([-102.4, -102.4, -1.6])
INNER_HI = np.array([102.4, 102.4, 33.6])
V_FAR = -10.0
CAR = np.array([4.5, 1.9, 1.6])
# car centre height: the body rests 1.37 cm above the ground, which keeps the
# horizontal faces of the actor box (centre +- 2.7 m) off the background's
# 0.1 m grid planes; a box face lying exactly on a leaf face makes the image a
# kinked function of the actor's height
CAR_Z = 0.8 + 0.0137


def soft_prior(d, s, v_close, v_far=V_FAR):
    return v_far + (v_close - v_far) * np.exp(-2.0 * d * d / (s * s))


# ------------------------------------------------------------------ world
def make_buildings(rng, n=40, half=100.0, road_half=10.0):
    out = []
    while len(out) < n:
        w, d = rng.uniform(8, 30, 2)
        h = rng.uniform(5, 30)
        cx, cy = rng.uniform(-half + w / 2, half - w / 2), rng.uniform(-half + d / 2, half - d / 2)
        lo = np.array([cx - w / 2, cy - d / 2, 0.0])
        hi = np.array([cx + w / 2, cy + d / 2, h])
        if lo[0] < road_half and hi[0] > -road_half:
            continue
        if lo[1] < road_half and hi[1] > -road_half:
            continue
        out.append((lo, hi))
    return out


def lidar_points(rng, buildings, step=2.0, beams=64, azimuths=1024,
                 rng_max=100.0, height=1.8, half=100.0):
    """Ray-cast sweeps from ego positions along both roads.  Each building
    is tested only against the azimuth columns its footprint spans."""
    el = np.deg2rad(np.linspace(-25.0, 15.0, beams))
    az = np.linspace(0, 2 * np.pi, azimuths, endpoint=False)
    E, A = np.meshgrid(el, az, indexing="ij")          # [beams, azimuths]
    dirs = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A),
                     np.sin(E)], -1)
    inv = 1.0 / np.where(dirs == 0, 1e-30, dirs)
    pos = [(x, 0.0) for x in np.arange(-half, half + 1e-9, step)]
    pos += [(0.0, y) for y in np.arange(-half, half + 1e-9, step) if abs(y) > 1e-9]
    dz = dirs[..., 2]
    down = dz < 0
    pts = []
    for (x, y) in pos:
        o = np.array([x, y, height])
        t = np.full(dz.shape, rng_max)
        tg = np.where(down, -o[2] / np.where(down, dz, -1.0), np.inf)
        t = np.minimum(t, tg)
        for lo, hi in buildings:
            cx = np.array([lo[0], hi[0], hi[0], lo[0]]) - x
            cy = np.array([lo[1], lo[1], hi[1], hi[1]]) - y
            if np.hypot(np.clip(x, lo[0], hi[0]) - x,
                        np.clip(y, lo[1], hi[1]) - y) > rng_max:
                continue
            ang = np.mod(np.arctan2(cy, cx), 2 * np.pi)
            srt = np.sort(ang)
            gaps = np.diff(np.concatenate([srt, srt[:1] + 2 * np.pi]))
            k = int(np.argmax(gaps))
            a0 = srt[(k + 1) % 4]
            span = 2 * np.pi - gaps[k]
            i0 = int(np.floor(a0 / (2 * np.pi) * azimuths)) - 1
            i1 = int(np.ceil((a0 + span) / (2 * np.pi) * azimuths)) + 1
            cols = np.arange(i0, i1 + 1) % azimuths
            d_ = dirs[:, cols]
            iv = inv[:, cols]
            t0 = (lo - o) * iv
            t1 = (hi - o) * iv
            tn = np.minimum(t0, t1).max(-1)
            tf = np.maximum(t0, t1).min(-1)
            hit = (tf >= tn) & (tn > 0)
            tc = t[:, cols]
            t[:, cols] = np.where(hit & (tn < tc), tn, tc)
        ok = t < rng_max
        p = o + t[ok][:, None] * dirs[ok]
        inside = (np.abs(p[:, 0]) <= half) & (np.abs(p[:, 1]) <= half)
        pts.append(p[inside])
    pts = np.concatenate(pts, 0)
    # de-duplicate on a 5 cm grid
    key = np.round(pts / 0.05).astype(np.int64) + (1 << 20)
    key = (key[:, 0] << 42) | (key[:, 1] << 21) | key[:, 2]
    _, idx = np.unique(key, return_index=True)
    return pts[np.sort(idx)]


# ------------------------------------------------------------------ octree
def _cells_box(lo, hi, level):
    """Integer cells of ``level`` covering [lo, hi) (aligned)."""
    h = ROOT_SIZE / (1 << level)
    a = np.round((lo - ROOT_MIN) / h).astype(np.int64)
    b = np.round((hi - ROOT_MIN) / h).astype(np.int64)
    g = np.stack(np.meshgrid(np.arange(a[0], b[0]), np.arange(a[1], b[1]),
                             np.arange(a[2], b[2]), indexing="ij"), -1)
    return g.reshape(-1, 3)


def _centres(cells, level):
    h = ROOT_SIZE / (1 << level)
    return ROOT_MIN + (cells + 0.5) * h


def _point_counts(pts, level):
    """Number of points in every occupied cell of ``level``: (keys, counts)
    with key = (i * 2^20 + j) * 2^20 + k."""
    h = ROOT_SIZE / (1 << level)
    c = np.floor((pts - ROOT_MIN) / h).astype(np.int64)
    key = (c[:, 0] << 40) | (c[:, 1] << 20) | c[:, 2]
    return np.unique(key, return_counts=True)


def _lookup(keys, counts, cells):
    key = (cells[:, 0] << 40) | (cells[:, 1] << 20) | cells[:, 2]
    i = np.searchsorted(keys, key)
    i = np.minimum(i, len(keys) - 1)
    return np.where(keys[i] == key, counts[i], 0)


def inner_leaves(pts, target, base=9, top=12):
    """Proximity subdivision of the inner region: a cell is split while it
    holds at least n_th * (h / h_top)^2 LiDAR points (points per unit of
    surface area), so cells near the dense part of the sweeps reach the
    finest level first; n_th is found by bisection so the leaf count is
    close to ``target``.  Returns (list of (level, cells), n_th)."""
    levels = {base: _cells_box(INNER_LO, INNER_HI, base)}
    cnt = {}
    parent = {}
    for l in range(base, top):
        keys, counts = _point_counts(pts, l)
        c = levels[l]
        cnt[l] = _lookup(keys, counts, c) / float(4 ** (top - l))
        cand = np.nonzero(cnt[l] > 0)[0]
        _, ch = children(l, c[cand].T)
        levels[l + 1] = ch.T.astype(np.int64)
        parent[l + 1] = np.tile(cand, 8)

    def build(nth, counts_only=False):
        sub = {}
        out = []
        n = 0
        for l in range(base, top):
            alive = sub[l - 1][parent[l]] if l > base else np.ones(len(cnt[l]), bool)
            s = alive & (cnt[l] >= nth)
            sub[l] = s
            leaf = alive & ~s
            if counts_only:
                n += int(leaf.sum())
            else:
                out.append((l, levels[l][leaf]))
        last = sub[top - 1][parent[top]]
        if counts_only:
            return n + int(last.sum())
        out.append((top, levels[top][last]))
        return out

    lo, hi = 1e-3, 1e6
    for _ in range(50):
        mid = np.sqrt(lo * hi)
        if build(mid, True) > target:
            lo = mid
        else:
            hi = mid
    return build(hi), hi


def far_shell(z_lo=-1.6, z_hi=64.0, coarse=4, near=5):
    """Leaves outside the inner box: 51.2 m cells, 25.6 m cells within one
    coarse cell of the inner box, finer cells only where alignment with
    the inner box needs them; cells entirely below z_lo or above z_hi are
    dropped (height filter)."""
    out = {}
    pad = ROOT_SIZE / (1 << coarse)

    def rec(l, c):
        h = ROOT_SIZE / (1 << l)
        lo = ROOT_MIN + c * h
        hi = lo + h
        if hi[2] <= z_lo or lo[2] >= z_hi:
            return
        inside = np.all(lo >= INNER_LO - 1e-9) and np.all(hi <= INNER_HI + 1e-9)
        if inside:
            return
        overlap = np.all(lo < INNER_HI - 1e-9) and np.all(hi > INNER_LO + 1e-9)
        near_box = np.all(lo < INNER_HI + pad) and np.all(hi > INNER_LO - pad)
        if not overlap and (l >= near or (l >= coarse and not near_box)):
            out.setdefault(l, []).append(c)
            return
        for m in range(8):
            rec(l + 1, 2 * c + np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1]))

    rec(0, np.zeros(3, np.int64))
    return [(l, np.array(v, np.int64)) for l, v in sorted(out.items())]


def background_octree(rng, target_leaves, v_close, n_buildings=40,
                      sweep_step=4.0, top=12):
    blds = make_buildings(rng, n_buildings)
    pts = lidar_points(rng, blds, step=sweep_step)
    far = far_shell()
    n_far = sum(len(c) for _, c in far)
    inner, tau = inner_leaves(pts, max(1, target_leaves - n_far), top=top)
    # nearest-point distances on a 10 cm thinning of the cloud
    key = np.round(pts / 0.1).astype(np.int64)
    key = (key[:, 0] << 42) ^ (key[:, 1] << 21) ^ key[:, 2]
    _, idx = np.unique(key, return_index=True)
    tree = cKDTree(pts[idx])
    parts = inner + far
    lv = np.concatenate([np.full(len(c), l, np.uint8) for l, c in parts])
    ijk = np.concatenate([c for _, c in parts], 0).T.astype(np.int32)
    # leaves and corners stored in Morton order (spatially compact runs)
    lv, ijk = morton_order_leaves(lv, ijk, top)
    cidx, upos = morton_order_corners(*dedup_corners(lv, ijk, top))
    cpos = ROOT_MIN + upos * (ROOT_SIZE / (1 << top))
    # beyond 1 m the prior equals v_far to double precision (s <= 0.2 m)
    d, _ = tree.query(cpos, k=1, distance_upper_bound=1.0, workers=-1)
    s_min = ROOT_SIZE / (1 << top)
    dens = soft_prior(d, s_min, v_close).astype(np.float32)
    sh = _sh_random(rng, lv.shape[0], 3)
    o = make_octree(ROOT_MIN, ROOT_SIZE, top, lv, ijk, cidx, dens, sh)
    info = dict(n_points=len(pts), points_per_cell=tau, n_far=n_far,
                buildings=blds, s=s_min)
    return o, info, pts


# ------------------------------------------------------------------ actors
def _box_distance(p, half):
    q = np.abs(p) - half
    return np.linalg.norm(np.maximum(q, 0.0), axis=-1)


_CAR_CACHE = {}


def car_octree(rng, target, v_close, base=4, top=6):
    """A car octree: structure and corner densities depend only on the leaf
    budget and v_close (built once per pair and copied), the SH coefficients
    are drawn from rng per car."""
    key = (int(target), float(v_close), base, top)
    if key not in _CAR_CACHE:
        _CAR_CACHE.clear()
        _CAR_CACHE[key] = _car_structure(target, v_close, base, top)
    rmin, side, lv, ijk, cidx, dens = _CAR_CACHE[key]
    sh = _sh_random(rng, lv.shape[0], 3)
    return make_octree(rmin, side, top, lv.copy(), ijk.copy(), cidx.copy(),
                       dens.copy(), sh)


def _car_structure(target, v_close, base, top):
    side = 1.2 * CAR.max()
    rmin = -side / 2 * np.ones(3)
    half = CAR / 2

    def centres(cells, l):
        return rmin + (cells + 0.5) * (side / (1 << l))

    g = np.stack(np.meshgrid(*[np.arange(1 << base)] * 3, indexing="ij"), -1).reshape(-1, 3)
    # distance of each cell's centre to the box surface (inside: depth)
    def surf(c, l):
        p = centres(c, l)
        out = _box_distance(p, half)
        inside = np.all(np.abs(p) < half, axis=-1)
        depth = np.min(half - np.abs(p), axis=-1)
        return np.where(inside, depth, out)

    def build(tau):
        leaves = []
        cur = g
        for l in range(base, top):
            r = (side / (1 << l)) * np.sqrt(3) / 2
            s = surf(cur, l) < tau + r
            leaves.append((l, cur[~s]))
            _, ch = children(l, cur[s].T)
            cur = ch.T.astype(np.int64)
        leaves.append((top, cur))
        return leaves

    lo, hi = 0.0, side
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        if sum(len(c) for _, c in build(mid)) < target:
            lo = mid
        else:
            hi = mid
    parts = build(lo)
    lv = np.concatenate([np.full(len(c), l, np.uint8) for l, c in parts])
    ijk = np.concatenate([c for _, c in parts], 0).T.astype(np.int32)
    lv, ijk = morton_order_leaves(lv, ijk, top)
    cidx, upos = morton_order_corners(*dedup_corners(lv, ijk, top))
    cpos = rmin + upos * (side / (1 << top))
    d = _box_distance(cpos, half)
    s_min = side / (1 << top)
    dens = soft_prior(d, s_min, v_close).astype(np.float32)
    return (rmin, side, np.ascontiguousarray(lv), np.ascontiguousarray(ijk),
            np.ascontiguousarray(cidx), np.ascontiguousarray(dens))


def car_tracks(rng, n, t_end=10.0, lane_ys=(-4.0, 4.0), x_start=-30.0,
               gap=12.0):
    """Cars on lanes parallel to x, equal speed per lane, >= gap apart."""
    tracks = []
    per_lane = int(np.ceil(n / len(lane_ys)))
    speeds = rng.uniform(5.0, 15.0, len(lane_ys))
    for i in range(n):
        lane = i % len(lane_ys)
        slot = i // len(lane_ys)
        x0 = x_start + slot * gap + rng.uniform(0, 2.0) + lane * 3.0
        y = lane_ys[lane]
        yaw = np.deg2rad(rng.uniform(-5.0, 5.0))
        v = speeds[lane]
        tracks.append(dict(t=np.array([0.0, t_end]), yaw=np.array([yaw, yaw]),
                           trans=np.array([[x0, y, CAR_Z],
                                           [x0 + v * t_end, y, CAR_Z]])))
    return tracks


# ------------------------------------------------------------------ configs
SPECS = {
    2: dict(bg=1_000_000, cars=8, car_vox=20_000, views="front", top=12,
            lanes=(-4.0, 4.0)),
    3: dict(bg=3_000_000, cars=30, car_vox=50_000, views="rig", top=13,
            lanes=(-8.0, 0.0, 8.0)),
    4: dict(bg=1_000_000, cars=8, car_vox=20_000, views="front", top=12,
            lanes=(-4.0, 4.0)),
    5: dict(bg=8_000_000, cars=100, car_vox=50_000, views="rig4", top=14,
            lanes=(-8.0, 0.0, 8.0)),
}


def make_driving_config(k, seed, v_close=10.0, scale=1.0, n_cars=None,
                        car_vox=None, W=1920, H=1080):
    """Workload k in {2, 3, 4, 5}.  ``scale`` shrinks leaf budgets (tests)."""
    spec = SPECS[k]
    rng = np.random.default_rng(seed)
    bg, info, pts = background_octree(rng, int(spec["bg"] * scale), v_close,
                                      top=spec["top"])
    info = dict(info, points=pts)
    nc = spec["cars"] if n_cars is None else n_cars
    cv = int((spec["car_vox"] if car_vox is None else car_vox) * min(1.0, scale * 4))
    octs = [bg]
    tracks = [None]
    for tr in car_tracks(rng, nc, lane_ys=spec["lanes"]):
        octs.append(car_octree(rng, cv, v_close))
        tracks.append(tr)
    views = []
    eye = np.array([-40.0, 0.0, 1.6])
    if spec["views"] == "front":
        views.append(make_view(W, H, 60.0, look_at_c2w(eye, eye + (1, 0, 0)), t=0.0))
    else:
        times = (0.0,) if spec["views"] == "rig" else (0.0, 0.1, 0.2, 0.3)
        for t in times:
            for i in range(6):
                a = np.deg2rad(60.0 * i)
                views.append(make_view(W, H, 70.0, look_at_c2w(
                    eye, eye + (np.cos(a), np.sin(a), 0.0)), t=t))
    opts = dict(K=1, eps_stop=1e-4, tau_near=0.0, bg=(0.0, 0.0, 0.0),
                explin_c=1.1)
    n_total = sum(o["level"].shape[0] for o in octs)
    names = {2: "driving-1M+8x20k-1080p-fwdbwd", 3: "driving-3M+30x50k-6x1080p",
             4: "driving-1M+8x20k-serving", 5: "driving-8M+100x50k-24x1080p"}
    return dict(name=names[k], scene=dict(octrees=octs, tracks=tracks),
                views=views, opts=opts, info=dict(info, n_total=n_total,
                                                  v_close=v_close))


def init_workload(seed=2, top=12, sweep_step=4.0, n_buildings=40, deg=3):
    """Inputs of the background initialisation (Sec. 3.3): the LiDAR-like
    point cloud of the workload-2 world and the starting grid before the
    proximity rounds, i.e. uniform 1.6 m cells over the inner region plus
    the coarse far shell, every corner at v_far, random SH.  Returns
    (octree dict, points [n, 3] FP64)."""
    rng = np.random.default_rng(seed)
    blds = make_buildings(rng, n_buildings)
    pts = lidar_points(rng, blds, step=sweep_step)
    parts = [(9, _cells_box(INNER_LO, INNER_HI, 9))] + far_shell()
    lv = np.concatenate([np.full(len(c), l, np.uint8) for l, c in parts])
    ijk = np.concatenate([c for _, c in parts], 0).T.astype(np.int32)
    cidx, upos = dedup_corners(lv, ijk, top)
    dens = np.full(upos.shape[0], V_FAR, np.float32)
    sh = _sh_random(rng, lv.shape[0], deg)
    return make_octree(ROOT_MIN, ROOT_SIZE, top, lv, ijk, cidx, dens, sh), pts
