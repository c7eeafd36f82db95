"""Pins of the oracle's structure edits (Sec. 3.3 initialisation; Supp.
adaptive schedule): children tile their parent exactly, subdivision keeps
the trilinear field, pruning keeps it on the remaining leaves, the
point-to-box distance against dense sampling, the proximity rule on hand
placed points, and the corner prior against Eq. 1."""
import numpy as np
import pytest

from oracle import prior as PR
from oracle import structure as ST
from scenes import random_octree


def _octree(seed=0):
    rng = np.random.default_rng(seed)
    return random_octree(rng, (-1.0, -1.0, -1.0), 2.0, 2, 6, 5, 0,
                         g_mean=0.0, g_std=1.0)


def test_children_tile_parent_exactly():
    o = _octree(1)
    split = np.zeros(len(o["level"]), bool)
    split[[0, 3, 7]] = True
    o2 = ST.subdivide(o, split)
    lo, hi, h = ST.leaf_boxes(o)
    lo2, hi2, h2 = ST.leaf_boxes(o2)
    n_keep = int((~split).sum())
    assert len(o2["level"]) == n_keep + 8 * int(split.sum())
    # the kept leaves come first, unchanged, then 8 children per parent
    assert np.array_equal(o2["ijk"][:, :n_keep], o["ijk"][:, ~split])
    for j, p in enumerate(np.nonzero(split)[0]):
        c = slice(n_keep + 8 * j, n_keep + 8 * j + 8)
        assert np.allclose(h2[c], h[p] / 2)
        # children are disjoint, inside the parent, and fill its volume
        assert np.all(lo2[c] >= lo[p] - 1e-15) and np.all(hi2[c] <= hi[p] + 1e-15)
        assert abs((h2[c] ** 3).sum() - h[p] ** 3) < 1e-12
        cen = 0.5 * (lo2[c] + hi2[c])
        assert len({tuple(np.round(x, 12)) for x in cen}) == 8


def test_subdivision_preserves_the_trilinear_field():
    # a uniform grid with shared corners: a new child corner never meets an
    # existing corner of a finer neighbour (there is none), so the field is
    # preserved everywhere inside the split leaves
    rng = np.random.default_rng(3)
    o = random_octree(rng, (-1.0, -1.0, -1.0), 2.0, 2, 0, 4, 0)
    o = dict(o, corner_density=o["corner_density"].astype(np.float64))
    split = rng.uniform(size=len(o["level"])) < 0.3
    o2 = ST.subdivide(o, split)
    lo, hi, h = ST.leaf_boxes(o)
    for v in np.nonzero(split)[0][:10]:
        for _ in range(5):
            x = lo[v] + rng.uniform(0.02, 0.98, 3) * h[v]
            assert abs(ST.field_at(o2, x) - ST.field_at(o, x)) < 1e-12
    # existing corners keep their values
    old = {tuple(p): val for p, val in zip(ST.corner_world_positions(o).round(12),
                                           o["corner_density"])}
    new = dict(zip(map(tuple, ST.corner_world_positions(o2).round(12)),
                   o2["corner_density"]))
    for k, val in old.items():
        if k in new:
            assert new[k] == val


def test_subdivision_next_to_finer_leaves_keeps_existing_corners():
    # mixed levels: where a child's corner already exists (a finer
    # neighbour's), it keeps its value; the parent's own corners too
    o = _octree(2)
    o = dict(o, corner_density=o["corner_density"].astype(np.float64))
    rng = np.random.default_rng(13)
    split = (rng.uniform(size=len(o["level"])) < 0.3) & (o["level"] < o["max_level"])
    o2 = ST.subdivide(o, split)
    old = dict(zip(map(tuple, ST.corner_world_positions(o).round(12)),
                   o["corner_density"]))
    new = dict(zip(map(tuple, ST.corner_world_positions(o2).round(12)),
                   o2["corner_density"]))
    assert all(new[k] == v for k, v in old.items() if k in new)
    assert len(new) > len(old)


def test_prune_keeps_the_field_and_drops_unused_corners():
    o = _octree(4)
    o = dict(o, corner_density=o["corner_density"].astype(np.float64))
    rng = np.random.default_rng(5)
    keep = rng.uniform(size=len(o["level"])) < 0.6
    o2 = ST.prune(o, keep)
    assert len(o2["level"]) == int(keep.sum())
    used = np.unique(o2["corner_idx"])
    assert np.array_equal(used, np.arange(len(o2["corner_density"])))
    lo, hi, h = ST.leaf_boxes(o)
    for v in np.nonzero(keep)[0][:10]:
        x = lo[v] + rng.uniform(0.05, 0.95, 3) * h[v]
        assert abs(ST.field_at(o2, x) - ST.field_at(o, x)) < 1e-12
    # corners in canonical (sorted position) order
    keys = [tuple(p) for p in o2["corner_pos"]]
    assert keys == sorted(keys)


def test_point_box_distance_against_sampling():
    rng = np.random.default_rng(6)
    lo, hi = np.array([0.0, 1.0, -1.0]), np.array([0.5, 2.0, 0.25])
    pts = rng.uniform(-2, 3, size=(40, 3))
    d = ST.point_box_distance(pts, lo, hi)
    # dense grid over the box (faces included)
    g = np.stack(np.meshgrid(*[np.linspace(lo[a], hi[a], 41) for a in range(3)],
                             indexing="ij"), -1).reshape(-1, 3)
    for p, dd in zip(pts, d):
        ds = np.sqrt(((g - p) ** 2).sum(1)).min()
        assert dd <= ds + 1e-12 and ds - dd <= 0.04      # grid step 0.05 max
    assert ST.point_box_distance(np.array([[0.2, 1.5, 0.0]]), lo, hi)[0] == 0.0


def test_proximity_rule_hand_placed_points():
    # one level-1 octree over [0, 2]^3: 8 leaves of side 1
    lv = np.ones(8, np.uint8)
    ijk = np.array([[m & 1, (m >> 1) & 1, (m >> 2) & 1] for m in range(8)]).T
    o = dict(root_min=np.zeros(3), root_size=2.0, max_level=3, level=lv, ijk=ijk)
    # a point inside leaf 0, one 0.4 from leaf 7's box, none near the rest
    pts = np.array([[0.5, 0.5, 0.5], [2.4, 1.5, 1.5]])
    f = ST.proximity_flags(o, pts, ratio=0.5)
    # leaf 0 contains a point; leaf 7 ([1,2]^3) and leaves 1/3/5 touching
    # x = 2 are within 0.4 of the second point only if their box is
    lo, hi, h = ST.leaf_boxes(o)
    ref = np.array([min(ST.point_box_distance(pts, lo[v], hi[v])) <= 0.5 for v in range(8)])
    assert np.array_equal(f, ref)
    assert f[0] and f[7] and not f[6]


def test_corner_prior_is_eq1_of_the_nearest_point():
    o = _octree(7)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-1, 1, size=(30, 3))
    s = 0.25
    v = ST.corner_prior(o, pts, s)
    cw = ST.corner_world_positions(o)
    d = np.array([np.sqrt(((pts - c) ** 2).sum(1)).min() for c in cw])
    assert np.allclose(v, -10.0 + 8.0 * np.exp(-2.0 * d * d / (s * s)), atol=1e-13)


def test_sources_name_the_parent_and_the_old_corner_at_the_same_place():
    # leaf_src: kept leaves name themselves, children a leaf whose box holds
    # theirs; corner_src: an old corner at the same world position with the
    # same value, -1 exactly where no old corner sits; children carry their
    # parent's SH
    o = _octree(9)
    rng = np.random.default_rng(10)
    split = (rng.uniform(size=len(o["level"])) < 0.25) & (o["level"] < o["max_level"])
    o2 = ST.subdivide(o, split)
    lo, hi, _ = ST.leaf_boxes(o)
    lo2, hi2, _ = ST.leaf_boxes(o2)
    src = o2["leaf_src"]
    n_keep = int((~split).sum())
    assert np.array_equal(src[:n_keep], np.nonzero(~split)[0])
    assert np.all(split[src[n_keep:]])
    assert np.all(lo2 >= lo[src] - 1e-15) and np.all(hi2 <= hi[src] + 1e-15)
    assert np.array_equal(o2["sh"], o["sh"][:, :, src])
    old_w = ST.corner_world_positions(o)
    new_w = ST.corner_world_positions(o2)
    old_set = {tuple(p) for p in old_w.round(12)}
    cs = o2["corner_src"]
    for c in range(len(cs)):
        if cs[c] >= 0:
            assert np.array_equal(new_w[c], old_w[cs[c]])
            assert o2["corner_density"][c] == o["corner_density"][cs[c]]
        else:
            assert tuple(new_w[c].round(12)) not in old_set
    assert (cs < 0).any() and (cs >= 0).any()
    # prune: sources are the kept leaves, corners all old
    keep = rng.uniform(size=len(o["level"])) < 0.5
    o3 = ST.prune(o, keep)
    assert np.array_equal(o3["leaf_src"], np.nonzero(keep)[0])
    assert np.all(o3["corner_src"] >= 0)
    assert np.array_equal(ST.corner_world_positions(o3),
                          old_w[o3["corner_src"]])


def test_refine_rounds_reach_the_minimum_size_near_points():
    # uniform level-2 grid over [-1, 1]^3 (leaf 0.5), points on a plane:
    # after refinement every leaf within ratio * h of a point is below the
    # minimum size (or at the maximum level), the leaves still tile the
    # cube, and the field of the uniform start grid is unchanged
    rng = np.random.default_rng(11)
    o = random_octree(rng, (-1.0, -1.0, -1.0), 2.0, 2, 0, 6, 0)
    o = dict(o, corner_density=o["corner_density"].astype(np.float64))
    pts = np.column_stack([rng.uniform(-1, 1, 60), rng.uniform(-1, 1, 60),
                           np.full(60, 0.1)])
    r = ST.refine(o, pts, ratio=0.5, min_size=0.1)
    lo, hi, h = ST.leaf_boxes(r)
    assert r["rounds"] == 3                      # 0.5 -> 0.25 -> 0.125 -> 0.0625
    assert abs((h ** 3).sum() - 8.0) < 1e-12
    near = ST.proximity_flags(r, pts, 0.5)
    assert np.all((h[near] < 0.1) | (r["level"][near] == r["max_level"]))
    assert h.min() < 0.1 and h.max() == 0.5
    lo0, hi0, _ = ST.leaf_boxes(o)
    src = r["leaf_src"]
    assert np.all(lo >= lo0[src] - 1e-15) and np.all(hi <= hi0[src] + 1e-15)
    # each round stores its densities as float32 (half an ulp each) and the
    # next interpolates them with convex weights, so the field moves by at
    # most rounds * 2^-24 * max|g|
    tol = r["rounds"] * 2.0 ** -24 * np.abs(o["corner_density"]).max()
    for _ in range(40):
        x = rng.uniform(-0.98, 0.98, 3)
        assert abs(ST.field_at(r, x) - ST.field_at(o, x)) <= tol
    # corner sources refer to the input table
    old_w = ST.corner_world_positions(o)
    new_w = ST.corner_world_positions(r)
    cs = r["corner_src"]
    assert np.array_equal(new_w[cs >= 0], old_w[cs[cs >= 0]])
