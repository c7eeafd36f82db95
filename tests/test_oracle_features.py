"""Pins of the oracle's feature accumulation render (Sec. 4.3, 3D semantic
segmentation: per-leaf features composited in place of colour) and of its
adjoint (the fusion of per-pixel features into the leaves)."""
import copy

import numpy as np
import pytest

from oracle import features as FT
from oracle import render as RD
from scenes import actor_scene

OPTS = dict(K=1, eps_stop=0.0, tau_near=0.0, bg=(0.2, 0.3, 0.4), explin_c=1.1)


def _feats(scene, F, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(F, len(o["level"]))) for o in scene["octrees"]]


def _setup(seed=4):
    cfg = actor_scene(seed=seed, n_actors=2, deg=1)
    v = dict(cfg["views"][0], w=16, h=12, x0=24, y0=18)
    return cfg["scene"], v, RD.window_pixels(v)


def test_constant_feature_is_opacity_times_value():
    sc, v, pix = _setup()
    c = np.array([0.7, -1.3, 2.0, 0.25])
    feats = [np.tile(c[:, None], (1, len(o["level"]))) for o in sc["octrees"]]
    out, T = FT.render_features(sc, v, OPTS, feats, pix)
    assert T.min() < 0.9          # the window sees geometry
    ref = (1.0 - T)[:, None] * c[None, :]
    assert np.abs(out - ref).max() < 1e-12


def test_three_channels_of_colour_reproduce_the_colour_render():
    sc, v, pix = _setup()
    ctx = RD.ViewContext(sc, v, OPTS)
    feats = [ent["col"].T.copy() for ent in ctx.oct]      # clamped SH colour
    out, T = FT.render_features(sc, v, OPTS, feats, pix)
    rgb = RD.render_pixels(sc, v, OPTS, pix)
    bg = np.asarray(OPTS["bg"])
    assert np.abs(out - (rgb[:, 0:3] - T[:, None] * bg)).max() < 1e-12
    assert np.abs(T - rgb[:, 7]).max() == 0.0


def test_linear_in_features_and_group_mapping():
    sc, v, pix = _setup(5)
    f1, f2 = _feats(sc, 5, 1), _feats(sc, 5, 2)
    o1, _ = FT.render_features(sc, v, OPTS, f1, pix)
    o2, _ = FT.render_features(sc, v, OPTS, f2, pix)
    mix = [2.0 * a - 0.5 * b for a, b in zip(f1, f2)]
    om, _ = FT.render_features(sc, v, OPTS, mix, pix)
    assert np.abs(om - (2.0 * o1 - 0.5 * o2)).max() < 1e-12
    # channel 3 rendered alone (as channel 0 of a one-channel feature)
    one = [f[3:4] for f in f1]
    o3, _ = FT.render_features(sc, v, OPTS, one, pix)
    assert np.abs(o3[:, 0] - o1[:, 3]).max() < 1e-13
    # the second group's missing third channel contributes nothing
    g = FT.group_channels(f1[0], 1)
    assert np.all(g[:, 2] == 0.0) and np.all(g[:, :2] == f1[0][3:5].T)


def test_fusion_adjoint_equals_exact_differences():
    sc, v, pix = _setup(6)
    feats = _feats(sc, 3, 3)
    rng = np.random.default_rng(7)
    G = np.zeros((len(pix), 8))
    G[:, 0:3] = rng.normal(size=(len(pix), 3))
    ref = FT.feature_adjoint(sc, v, OPTS, feats, pix, G, 0)

    def loss(fs):
        out, _ = FT.render_features(sc, v, OPTS, fs, pix)
        return float((out * G[:, 0:3]).sum())

    # the render is linear in the features: differences are exact
    for k in range(len(feats)):
        for idx in np.argsort(-np.abs(ref["feat"][k]).ravel())[:4]:
            ch, leaf = np.unravel_index(idx, feats[k].shape)
            fp = copy.deepcopy(feats)
            fp[k][ch, leaf] += 1.0
            d = loss(fp) - loss(feats)
            assert abs(d - ref["feat"][k][ch, leaf]) < 1e-10


def test_feature_corner_gradient_matches_central_differences():
    sc, v, pix = _setup(8)
    feats = _feats(sc, 3, 9)
    rng = np.random.default_rng(10)
    G = rng.normal(size=(len(pix), 8))
    G[:, 4:7] = 0.0
    ref = FT.feature_adjoint(sc, v, OPTS, feats, pix, G, 0)

    def loss(s_):
        out, T = FT.render_features(s_, v, OPTS, feats, pix)
        ctxo = RD.render_pixels(s_, v, OPTS, pix)
        return float((out * G[:, 0:3]).sum() + (ctxo[:, 3] * G[:, 3]).sum()
                     + (T * G[:, 7]).sum())

    h = 1e-6
    for k in range(len(sc["octrees"])):
        cg = ref["corner"][k]
        for c in np.argsort(-np.abs(cg))[:2]:
            sp = copy.deepcopy(sc)
            sm = copy.deepcopy(sc)
            sp["octrees"][k]["corner_density"] = sp["octrees"][k]["corner_density"].astype(np.float64)
            sm["octrees"][k]["corner_density"] = sm["octrees"][k]["corner_density"].astype(np.float64)
            sp["octrees"][k]["corner_density"][c] += h
            sm["octrees"][k]["corner_density"][c] -= h
            fd = (loss(sp) - loss(sm)) / (2 * h)
            assert abs(fd - cg[c]) <= 1e-6 * abs(fd) + 1e-8, (k, c, fd, cg[c])
