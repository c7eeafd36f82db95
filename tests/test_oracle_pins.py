"""Pins of the FP64 oracle against closed forms, invariants, library
routines and brute force (none of these re-types the oracle's own code)."""
import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle import render as RD
from oracle import field as F
from oracle import sh as SH
from oracle import binning as B
from synth import make_config, make_view, look_at_c2w
from scenes import (octree_private, empty_octree, dc_for_colour, Y00,
                    random_octree, static_track, actor_scene)

OPTS = dict(K=1, eps_stop=0.0, tau_near=0.0, bg=(0.2, 0.3, 0.4),
            explin_c=1.1)


def _explin_ref(x, c=1.1):
    # closed form of the reading, evaluated independently
    return x if x > c else c * math.exp(x / c - 1.0)


def _axis_view(eye, target, W=8, H=8, fov=10.0):
    return make_view(W, H, fov, look_at_c2w(eye, target, up=(0, 0, 1)))


# ---------------------------------------------------------------- P1
def test_p1_empty_scene_returns_background():
    sc = dict(octrees=[empty_octree()], tracks=[None])
    v = _axis_view((3, 0.2, 0.1), (0, 0, 0))
    img = RD.render_image(sc, v, OPTS)
    assert np.all(img["rgb"] == np.array(OPTS["bg"])[:, None, None])
    assert np.all(img["depth"] == 0.0)
    assert np.all(img["normal"] == 0.0)
    assert np.all(img["T"] == 1.0)


def test_p1_ray_missing_everything():
    o = octree_private((0, 0, 0), 1.0, 0, [(0, 0, 0, 0)], np.zeros((1, 8)),
                       dc_for_colour([0.5, 0.5, 0.5]).reshape(1, 3, 1))
    sc = dict(octrees=[o], tracks=[None])
    v = _axis_view((3, 5, 0.5), (3, 10, 0.5))     # looks away
    img = RD.render_image(sc, v, OPTS)
    assert np.all(img["T"] == 1.0) and np.all(img["depth"] == 0.0)


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("g,K", [(-1.0, 1), (0.3, 3), (2.5, 1), (4.0, 7)])
def test_p2_single_constant_voxel(g, K):
    col = np.array([0.9, 0.4, 0.1])
    o = octree_private((0, 0, 0), 1.0, 0, [(0, 0, 0, 0)], np.full((1, 8), g),
                       dc_for_colour(col).reshape(1, 3, 1).astype(np.float32))
    col32 = np.maximum(Y00 * o["sh"][0, :, 0].astype(np.float64) + 0.5, 0)
    sc = dict(octrees=[o], tracks=[None])
    opts = dict(OPTS, K=K)
    eye = np.array([2.3, 0.37, 0.61])
    ctx = RD.ViewContext(sc, _axis_view(eye, (0.5, 0.5, 0.5)), opts)
    # a ray along -x through (y,z) = (0.37, 0.61): chord [1.3, 2.3]
    o_, d_ = eye, np.array([-1.0, 0.0, 0.0])
    r, pc, _ = RD.render_ray(ctx, o_, d_)
    g = float(np.float32(g))                      # parameters are FP32
    T = math.exp(-_explin_ref(g) * 1.0)
    assert abs(r["T"] - T) < 1e-14
    assert np.allclose(r["rgb"], (1 - T) * col32 + T * np.array(opts["bg"]),
                       atol=1e-14, rtol=0)
    assert abs(r["depth"] - (1 - T) * 0.5 * (1.3 + 2.3)) < 1e-13
    assert np.all(r["normal"] == 0.0)          # constant field: no normal
    # an oblique ray: chord from the exact slab
    d2 = np.array([-1.0, 0.2, -0.1])
    d2 /= np.linalg.norm(d2)
    r2, pc2, _ = RD.render_ray(ctx, eye, d2)
    tx = [(1.0 - eye[0]) / d2[0], (0.0 - eye[0]) / d2[0]]
    ty = [(0.0 - eye[1]) / d2[1], (1.0 - eye[1]) / d2[1]]
    tz = [(0.0 - eye[2]) / d2[2], (1.0 - eye[2]) / d2[2]]
    t0 = max(min(tx), min(ty), min(tz))
    t1 = min(max(tx), max(ty), max(tz))
    assert abs(r2["T"] - math.exp(-_explin_ref(g) * (t1 - t0))) < 1e-14


# ---------------------------------------------------------------- P3
def test_p3_linear_regime_midpoint_exact():
    # corners vary along x only: g = 2 + 3 x (above the knee everywhere)
    g8 = np.array([[2.0 + 3.0 * (m & 1) for m in range(8)]])
    o = octree_private((0, 0, 0), 1.0, 0, [(0, 0, 0, 0)], g8,
                       dc_for_colour([0.5, 0.5, 0.5]).reshape(1, 3, 1))
    sc = dict(octrees=[o], tracks=[None])
    eye = np.array([-1.0, 0.3, 0.6])
    ctx = RD.ViewContext(sc, _axis_view(eye, (0.5, 0.3, 0.6)), OPTS)
    r, _, _ = RD.render_ray(ctx, eye, np.array([1.0, 0.0, 0.0]))
    # integral of 2 + 3x over [0,1] = 3.5
    assert abs(r["T"] - math.exp(-3.5)) < 1e-14
    # normal = -grad/|grad| = (-1, 0, 0)
    assert np.allclose(r["normal"], (1 - math.exp(-3.5)) * np.array([-1, 0, 0]),
                       atol=1e-14)


# ---------------------------------------------------------------- P4
def test_p4_two_stacked_voxels_over_operator():
    g8 = np.array([np.full(8, 0.4), np.full(8, 2.0)])
    cols = np.array([[0.8, 0.2, 0.1], [0.1, 0.7, 0.9]])
    sh = np.stack([dc_for_colour(c) for c in cols], -1).reshape(1, 3, 2)
    o = octree_private((0, 0, 0), 2.0, 1, [(1, 0, 0, 0), (1, 1, 0, 0)], g8,
                       sh.astype(np.float32))
    c32 = np.maximum(Y00 * o["sh"][0].astype(np.float64) + 0.5, 0).T
    sc = dict(octrees=[o], tracks=[None])
    eye = np.array([-0.5, 0.5, 0.5])
    ctx = RD.ViewContext(sc, _axis_view(eye, (1, 0.5, 0.5)), OPTS)
    r, _, _ = RD.render_ray(ctx, eye, np.array([1.0, 0, 0]))
    e1 = math.exp(-_explin_ref(float(np.float32(0.4))))
    e2 = math.exp(-_explin_ref(2.0))
    C = (1 - e1) * c32[0] + e1 * (1 - e2) * c32[1]
    assert np.allclose(r["C"], C, atol=1e-14, rtol=0)
    assert abs(r["T"] - e1 * e2) < 1e-15
    D = (1 - e1) * 1.0 + e1 * (1 - e2) * 2.0
    assert abs(r["depth"] - D) < 1e-14
    # associativity: (C1,T1) over (C2,T2) == sequential
    C1, T1 = (1 - e1) * c32[0], e1
    C2, T2 = (1 - e2) * c32[1], e2
    assert np.allclose(C1 + T1 * C2, r["C"], atol=1e-15)
    assert abs(T1 * T2 - r["T"]) < 1e-15


# ---------------------------------------------------------------- P5
def _pointwise_sigma_colour(scene, ctx, x_w):
    """Independent evaluation of the density field and colour at a world
    point: owner = lowest-index actor whose box contains the point, else the
    background; then the leaf of that octree containing it (brute force)."""
    owner = 0
    for k in range(1, len(scene["octrees"])):
        ent = ctx.oct[k]
        if not ent["active"]:
            continue
        xl = ent["R"].T @ (x_w - ent["p"])
        bmin, bmax = ent["box"]
        if np.all(xl >= bmin) and np.all(xl < bmax):
            owner = k
            break
    ent = ctx.oct[owner]
    o = scene["octrees"][owner]
    xl = ent["R"].T @ (x_w - ent["p"])
    inside = np.all((xl >= ent["vmin"]) & (xl < ent["vmax"]), axis=1)
    idx = np.nonzero(inside)[0]
    if idx.size == 0:
        return 0.0, np.zeros(3)
    v = idx[0]
    u = (xl - ent["vmin"][v]) / ent["h"][v]
    g = o["corner_density"].astype(np.float64)[o["corner_idx"][:, v]]
    val = 0.0
    for m in range(8):
        wgt = 1.0
        for a in range(3):
            wgt *= u[a] if (m >> a) & 1 else 1 - u[a]
        val += wgt * g[m]
    return _explin_ref(val), ent["col"][v]


def test_p5_dense_sampling_matches_field_definition():
    cfg = actor_scene(seed=3, n_actors=2, deg=1, K=64, bg_levels=(1, 3, 2))
    sc, v = cfg["scene"], cfg["views"][0]
    opts = dict(cfg["opts"], K=64)
    ctx = RD.ViewContext(sc, v, opts)
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(6):
        px, py = rng.integers(8, 56), rng.integers(8, 40)
        o, d = G.camera_ray(v, px, py)
        r, pc, _ = RD.render_ray(ctx, o, d)
        if pc["a"].size == 0:
            continue
        t_lo, t_hi = pc["a"][0], pc["b"][-1]
        n = 40000
        dt = (t_hi - t_lo) / n
        T, C = 1.0, np.zeros(3)
        for i in range(n):
            t = t_lo + (i + 0.5) * dt
            s, c = _pointwise_sigma_colour(sc, ctx, o + t * d)
            e = math.exp(-s * dt)
            C += T * (1 - e) * c
            T *= e
        assert abs(T - r["T"]) < 2e-4, (px, py)
        assert np.abs(C - r["C"]).max() < 2e-4
        checked += 1
    assert checked >= 3


def test_p5_midpoint_error_bound_small_K():
    # quadratic-ish field (knee crossing) stays within the composite
    # midpoint-rule bound l^3 max|sigma''| / (24 K^2) per piece
    g8 = np.array([[-3.0, 4.0, -2.0, 3.0, -1.0, 2.5, 0.0, 5.0]])
    o = octree_private((0, 0, 0), 1.0, 0, [(0, 0, 0, 0)], g8,
                       dc_for_colour([0.5, 0.5, 0.5]).reshape(1, 3, 1))
    sc = dict(octrees=[o], tracks=[None])
    eye = np.array([-1.0, 0.3, 0.6])
    d = np.array([1.0, 0.1, -0.05])
    d /= np.linalg.norm(d)
    taus = []
    for K in (1, 2, 4, 8, 256):
        ctx = RD.ViewContext(sc, _axis_view(eye, eye + d), dict(OPTS, K=K))
        r, pc, smp = RD.render_ray(ctx, eye, d)
        taus.append(smp["tau"][0])
    exact = taus[-1]
    l = pc["b"][0] - pc["a"][0]
    # sigma'' <= max over the trilinear range of explin'' * (dg/dt)^2 +
    # explin' * d2g/dt2; bound loosely with corner spread
    spread = 9.0
    bound = lambda K: l ** 3 * (spread ** 2 / 1.1 + 4 * spread) / (24 * K * K) * 10
    for K, t in zip((1, 2, 4, 8), taus[:4]):
        assert abs(t - exact) <= bound(K)
    # and it converges at second order
    e1, e8 = abs(taus[0] - exact), abs(taus[3] - exact)
    assert e8 < e1 / 20


# ---------------------------------------------------------------- P6
def test_p6_identity_pose_actor_equals_merged_octree():
    rng = np.random.default_rng(7)
    # background: root [0,8]^3, level-2 cells, minus the level-1 cell that
    # the actor occupies ([4,8] x [0,4] x [0,4])
    leaves = []
    for i in range(4):
        for j in range(4):
            for k in range(4):
                if i >= 2 and j < 2 and k < 2:
                    continue
                leaves.append((2, i, j, k))
    nb = len(leaves)
    gb = rng.normal(-0.5, 1.0, (nb, 8))
    shb = rng.uniform(-1.5, 1.5, (4, 3, nb)).astype(np.float32)
    bg = octree_private((0, 0, 0), 8.0, 3, leaves, gb, shb)
    # actor: root [4,8]x[0,4]x[0,4] in world == local (identity pose)
    al = [(2, i, j, k) for i in range(4) for j in range(4) for k in range(4)]
    na = len(al)
    ga = rng.normal(0.5, 1.0, (na, 8))
    sha = rng.uniform(-1.5, 1.5, (4, 3, na)).astype(np.float32)
    act = octree_private((4.0, 0.0, 0.0), 4.0, 2, al, ga, sha)
    sc2 = dict(octrees=[bg, act], tracks=[None, static_track(0.0, (0, 0, 0))])
    merged = octree_private((0, 0, 0), 8.0, 3,
                            leaves + [(3, 4 + i, j, k) for (_, i, j, k) in al],
                            np.concatenate([gb, ga]),
                            np.concatenate([shb, sha], axis=2))
    sc1 = dict(octrees=[merged], tracks=[None])
    v = make_view(24, 18, 70.0, look_at_c2w((14.0, -6.0, 9.0), (4, 4, 3)))
    a = RD.render_image(sc1, v, OPTS)
    b = RD.render_image(sc2, v, OPTS)
    for key in ("rgb", "depth", "normal", "T"):
        assert np.abs(a[key] - b[key]).max() <= 1e-12, key
    assert (a["T"] < 0.99).sum() > 50


# ---------------------------------------------------------------- P7
def _rigid(M, t, R, p):
    return M @ R, M @ p + t


def test_p7_rigid_comotion():
    rng = np.random.default_rng(11)
    cfg = actor_scene(seed=5, n_actors=2, deg=2)
    sc = cfg["scene"]
    sc = dict(octrees=[empty_octree((-2, -2, -2), 4.0)] + sc["octrees"][1:],
              tracks=sc["tracks"])
    v = cfg["views"][0]
    ctx = RD.ViewContext(sc, v, cfg["opts"])
    poses = [(ctx.oct[k]["R"], ctx.oct[k]["p"]) for k in (1, 2)]
    base = RD.render_image(sc, v, cfg["opts"], pose_override=poses)
    # random rotation + translation applied to camera and actors
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    M = q * np.sign(np.linalg.det(q))
    t = rng.normal(size=3)
    v2 = dict(v)
    c2w = v["c2w"].copy()
    c2w[:, :3] = M @ c2w[:, :3]
    c2w[:, 3] = M @ c2w[:, 3] + t
    v2["c2w"] = c2w
    moved = RD.render_image(sc, v2, cfg["opts"],
                            pose_override=[_rigid(M, t, R, p) for R, p in poses])
    for key in ("rgb", "depth", "T"):
        assert np.abs(base[key] - moved[key]).max() <= 1e-12, key
    # normals are world-frame vectors: rotate with the scene
    assert np.abs(np.einsum("ab,bhw->ahw", M, base["normal"]) - moved["normal"]).max() <= 1e-12
    assert (base["T"] < 0.9).sum() > 20


def test_p7_global_translation_with_background():
    cfg = actor_scene(seed=6, n_actors=2, deg=1)
    sc, v = cfg["scene"], cfg["views"][0]
    ctx = RD.ViewContext(sc, v, cfg["opts"])
    poses = [(ctx.oct[k]["R"], ctx.oct[k]["p"]) for k in (1, 2)]
    base = RD.render_image(sc, v, cfg["opts"], pose_override=poses)
    t = np.array([0.5, -0.25, 0.125])           # dyadic: exact shifts
    bg = dict(sc["octrees"][0])
    bg["root_min"] = bg["root_min"] + t
    sc2 = dict(octrees=[bg] + sc["octrees"][1:], tracks=sc["tracks"])
    v2 = dict(v)
    v2["c2w"] = v["c2w"].copy()
    v2["c2w"][:, 3] += t
    moved = RD.render_image(sc2, v2, cfg["opts"],
                            pose_override=[(R, p + t) for R, p in poses])
    for key in ("rgb", "depth", "normal", "T"):
        assert np.abs(base[key] - moved[key]).max() <= 1e-10, key


# ---------------------------------------------------------------- P8
def test_p8_ownership_swap_only_changes_overlap_rays():
    cfg = actor_scene(seed=9, n_actors=2, deg=1, overlap=True)
    sc, v = cfg["scene"], cfg["views"][0]
    sw = dict(octrees=[sc["octrees"][0], sc["octrees"][2], sc["octrees"][1]],
              tracks=[None, sc["tracks"][2], sc["tracks"][1]])
    a = RD.render_image(sc, v, cfg["opts"])
    b = RD.render_image(sw, v, cfg["opts"])
    ctx = RD.ViewContext(sc, v, cfg["opts"])
    diff = np.abs(a["rgb"] - b["rgb"]).max(0) + np.abs(a["T"] - b["T"])
    n_overlap = 0
    for py in range(v["h"]):
        for px in range(v["w"]):
            o, d = G.camera_ray(v, px, py)
            fr = RD.ray_frames(ctx, o, d)
            iv = []
            for k in (1, 2):
                t0, t1, _, _ = G.slab(*fr[k], *ctx.oct[k]["box"])
                iv.append((max(t0, 0.0), t1))
            crosses = min(iv[0][1], iv[1][1]) > max(iv[0][0], iv[1][0])
            if not crosses:
                assert diff[py, px] <= 1e-12
            else:
                n_overlap += 1
    assert n_overlap > 10
    assert diff.max() > 1e-6


# ---------------------------------------------------------------- P9
def test_p9_sh_orthonormal_gram():
    xs, ws = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct = np.repeat(xs, nphi)
    st = np.sqrt(1 - ct ** 2)
    ph = np.tile(phi, len(xs))
    w = np.repeat(ws, nphi) * (2 * np.pi / nphi)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1)
    Y = SH.basis(dirs, 3)
    gram = (Y * w[:, None]).T @ Y
    assert np.abs(gram - np.eye(16)).max() < 1e-12


def test_p9_sh_matches_scipy_complex_harmonics():
    import scipy.special as ss
    rng = np.random.default_rng(1)
    dirs = rng.normal(size=(50, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    theta = np.arccos(dirs[:, 2])
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    Y = SH.basis(dirs, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = ss.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            else:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            assert np.abs(Y[:, l * l + l + m] - ref).max() < 1e-12, (l, m)
    # degree 0 is a constant; degree 1 is proportional to (y, z, x)
    assert np.allclose(Y[:, 0], 0.5 / math.sqrt(math.pi), atol=1e-15)
    s3 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 1:4], s3 * dirs[:, [1, 2, 0]], atol=1e-14)


# ---------------------------------------------------------------- P10/P11
def test_p10_trilinear():
    rng = np.random.default_rng(2)
    g8 = rng.normal(size=8)
    for m in range(8):
        u = np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1], np.float64)
        assert abs(F.trilinear_weights(u) @ g8 - g8[m]) < 1e-15
    u = rng.uniform(size=(100, 3))
    assert np.allclose(F.trilinear_weights(u).sum(1), 1.0, atol=1e-15)
    gw = F.trilinear_weight_grads(u)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (F.trilinear_weights(u + e) - F.trilinear_weights(u - e)) / (2 * h)
        assert np.abs(fd - gw[..., a]).max() < 1e-9


def test_p11_explin():
    c = 1.1
    assert abs(F.explin(c, c) - c) < 1e-15
    assert abs(F.explin(c - 1e-9, c) - (c - 1e-9)) < 1e-15
    h = 1e-7
    left = (F.explin(c, c) - F.explin(c - h, c)) / h
    assert abs(left - 1.0) < 1e-6
    for x in (1.2, 3.0, 10.0):
        assert F.explin(x, c) == x
    assert abs(F.explin(-10.0, c) - 4.6e-5) < 1e-6
    xs = np.linspace(-5, 5, 101)
    fd = (F.explin(xs + 1e-7, c) - F.explin(xs - 1e-7, c)) / 2e-7
    ok = np.abs(xs - c) > 1e-6
    assert np.abs(fd - F.explin_grad(xs, c))[ok].max() < 1e-6


# ---------------------------------------------------------------- P12/P13
def _scene_cases():
    cfg = make_config(1)
    yield cfg["scene"], cfg["views"][0]
    # camera inside the root of a random octree
    rng = np.random.default_rng(4)
    o = random_octree(rng, (-1, -1, -1), 2.0, 2, 40, 5, 0)
    v = make_view(48, 40, 90.0, look_at_c2w((0.13, -0.21, 0.07), (1, 0.4, 0.2)))
    yield dict(octrees=[o], tracks=[None]), v
    a = actor_scene(seed=1, n_actors=2)
    yield a["scene"], a["views"][0]


def test_p12_rank_order_matches_entry_distance():
    for sc, v in _scene_cases():
        poses = G.octree_poses(sc, v)
        ctx = RD.ViewContext(sc, v, OPTS)
        ranks = [B.leaf_ranks(o, v, poses[k][1], poses[k][2]) if poses[k][0] else None
                 for k, o in enumerate(sc["octrees"])]
        for py in range(0, v["h"], 3):
            for px in range(0, v["w"], 3):
                o_, d_ = G.camera_ray(v, px, py)
                fr = RD.ray_frames(ctx, o_, d_)
                for k, ent in enumerate(ctx.oct):
                    if not ent["active"]:
                        continue
                    t0, t1, _, _ = G.slab_many(*fr[k], ent["vmin"], ent["vmax"])
                    hit = np.nonzero(t1 > np.maximum(t0, 0.0))[0]
                    if hit.size < 2:
                        continue
                    order = hit[np.argsort(ranks[k][hit], kind="stable")]
                    assert np.all(np.diff(np.maximum(t0[order], 0.0)) > 0) or \
                        np.all(np.diff(t1[order]) > 0)
                    assert np.all(np.diff(t1[order]) > 0)


def test_p13_binning_is_superset_of_exact_hits():
    for sc, v in _scene_cases():
        poses = G.octree_poses(sc, v)
        lists = B.expected_tile_lists(sc, v, poses)
        sets = {t: set(l) for t, l in lists.items()}
        ctx = RD.ViewContext(sc, v, OPTS)
        ntx = (v["w"] + 15) // 16
        for py in range(v["h"]):
            for px in range(0, v["w"], 2):
                o_, d_ = G.camera_ray(v, px + v["x0"], py + v["y0"])
                fr = RD.ray_frames(ctx, o_, d_)
                tile = (py >> 4) * ntx + (px >> 4)
                for k, ent in enumerate(ctx.oct):
                    if not ent["active"]:
                        continue
                    t0, t1, _, _ = G.slab_many(*fr[k], ent["vmin"], ent["vmax"])
                    for vv in np.nonzero(t1 > np.maximum(t0, 0.0))[0]:
                        assert (k, int(vv)) in sets.get(tile, ()), (k, vv, tile)


def test_p13_actor_box_binning_superset():
    a = actor_scene(seed=2, n_actors=3)
    sc, v = a["scene"], a["views"][0]
    poses = G.octree_poses(sc, v)
    al = B.actor_tile_lists(sc, v, poses)
    ctx = RD.ViewContext(sc, v, OPTS)
    ntx = (v["w"] + 15) // 16
    for py in range(v["h"]):
        for px in range(v["w"]):
            o_, d_ = G.camera_ray(v, px, py)
            own, boxes = RD.owned_intervals(ctx, RD.ray_frames(ctx, o_, d_))
            tile = (py >> 4) * ntx + (px >> 4)
            for (k, A, Bv, _, _) in boxes:
                assert k in al.get(tile, [])


# ---------------------------------------------------------------- P16
def test_p16_conservation_and_bounds():
    cfg = actor_scene(seed=4, n_actors=2, deg=2)
    sc, v = cfg["scene"], cfg["views"][0]
    ctx = RD.ViewContext(sc, v, cfg["opts"])
    maxc = max(ent["col"].max() for ent in ctx.oct)
    for py in range(0, v["h"], 4):
        for px in range(0, v["w"], 4):
            o, d = G.camera_ray(v, px, py)
            r, _, _ = RD.render_ray(ctx, o, d)
            assert abs(r["w"].sum() + r["T"] - 1.0) < 1e-13
            assert 0.0 <= r["T"] <= 1.0
            assert np.all(np.diff(np.concatenate([[1.0], r["Tb"], [r["T"]]])) <= 0)
            assert np.all(r["C"] >= 0) and np.all(r["C"] <= maxc + 1e-12)


def test_eps_stop_bounded_change():
    cfg = make_config(1)
    sc, v = cfg["scene"], cfg["views"][0]
    a = RD.render_image(sc, v, dict(cfg["opts"], eps_stop=0.0))
    b = RD.render_image(sc, v, dict(cfg["opts"], eps_stop=0.2))
    assert np.abs(a["rgb"] - b["rgb"]).max() <= 0.2 * 1.0 + 1e-12


def test_p13_binning_superset_near_plane_boxes():
    # camera a fraction of a millimetre from leaf faces, wide field of view:
    # many leaves straddle the plane Z = 1e-3 and get clipped rectangles
    rng = np.random.default_rng(21)
    o = random_octree(rng, (-1, -1, -1), 2.0, 3, 60, 5, 0)
    for eye, tgt in (((0.0003, 0.2502, -0.0004), (1.0, 0.3, 0.1)),
                     ((0.5, 0.5001, 0.4998), (-1.0, 0.2, 0.6))):
        v = make_view(40, 32, 100.0, look_at_c2w(eye, tgt))
        sc = dict(octrees=[o], tracks=[None])
        poses = G.octree_poses(sc, v)
        st, *_ = B.leaf_rects(o, v, poses[0][1], poses[0][2])
        lists = B.expected_tile_lists(sc, v, poses)
        sets = {t: set(l) for t, l in lists.items()}
        ctx = RD.ViewContext(sc, v, OPTS)
        ntx = (v["w"] + 15) // 16
        ent = ctx.oct[0]
        n_full = int((st == 2).sum())
        for py in range(v["h"]):
            for px in range(v["w"]):
                o_, d_ = G.camera_ray(v, px, py)
                t0, t1, _, _ = G.slab_many(o_, d_, ent["vmin"], ent["vmax"])
                tile = (py >> 4) * ntx + (px >> 4)
                for vv in np.nonzero(t1 > np.maximum(t0, 0.0))[0]:
                    assert (0, int(vv)) in sets.get(tile, ()), (vv, tile)
        # the near-plane rule keeps most straddling leaves off the full window
        assert n_full < 30
