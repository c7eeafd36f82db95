"""Pins of the oracle's sky environment map (Sec. 3.1, Eq. 2): texel
centres, bilinear reproduction of a map linear in longitude (across the
wrap), a constant map against the constant background, and the texture
gradient against a finite difference (L is linear in the texture)."""
import numpy as np

from oracle import adjoint as AD
from oracle import render as RD
from oracle import sky as SKY
from scenes import actor_scene


def _rand_sky(rng, H=8, W=16):
    return rng.uniform(0.0, 1.0, size=(3, H, W))


def test_texel_centres_sample_the_texel():
    rng = np.random.default_rng(0)
    sky = _rand_sky(rng)
    _, H, W = sky.shape
    for j in range(H):
        for i in range(W):
            d = SKY.texel_direction(i, j, W, H)
            assert np.allclose(SKY.sample(sky, 3.0 * d), sky[:, j, i], atol=1e-12)


def test_linear_in_longitude_is_reproduced_including_the_seam():
    H, W = 6, 12
    sky = np.zeros((3, H, W))
    # channel 0: cos/sin of the column's longitude are not linear in the
    # column index, so use the index itself away from the seam ...
    sky[0] = np.arange(W)[None, :]
    # ... and a map that is linear across the seam: column index shifted
    # by half a turn, taken modulo W
    sky[1] = ((np.arange(W) + W // 2) % W)[None, :]
    for phi in np.linspace(-np.pi + 1e-3, np.pi - 1e-3, 97):
        theta = 1.1
        d = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                      np.cos(theta)])
        u = (phi + np.pi) / (2 * np.pi) * W - 0.5
        c = SKY.sample(sky, d)
        if 0.0 <= u <= W - 1:
            assert abs(c[0] - u) < 1e-9
        us = (u + W // 2) % W
        if 0.0 <= us <= W - 1:
            assert abs(c[1] - us) < 1e-9


def test_poles_clamp_rows():
    rng = np.random.default_rng(1)
    sky = _rand_sky(rng)
    _, H, W = sky.shape
    # straight up: colatitude 0, v = -1/2, both rows clamp to row 0; the
    # longitude of (0, 0, 1) is atan2(0, 0) = 0, i.e. u = W/2 - 1/2
    c = SKY.sample(sky, np.array([0.0, 0.0, 1.0]))
    ref = 0.5 * (sky[:, 0, W // 2 - 1] + sky[:, 0, W // 2])
    assert np.allclose(c, ref, atol=1e-12)
    c = SKY.sample(sky, np.array([0.0, 0.0, -1.0]))
    ref = 0.5 * (sky[:, H - 1, W // 2 - 1] + sky[:, H - 1, W // 2])
    assert np.allclose(c, ref, atol=1e-12)


def _scene():
    cfg = actor_scene(seed=4, n_actors=1, deg=1)
    opts = dict(cfg["opts"], eps_stop=0.0)
    return cfg["scene"], cfg["views"][0], opts


def test_constant_map_equals_constant_background():
    scene, view, opts = _scene()
    col = (0.25, 0.5, 0.75)
    sky = np.empty((3, 4, 8))
    sky[:] = np.asarray(col)[:, None, None]
    pix = RD.window_pixels(view)[::37]
    a = RD.render_pixels(scene, view, dict(opts, bg=col), pix)
    b = RD.render_pixels(scene, view, dict(opts, bg=(9.0, 9.0, 9.0), sky=sky), pix)
    assert np.allclose(a, b, atol=1e-12)


def test_sky_gradient_matches_finite_difference():
    scene, view, opts = _scene()
    rng = np.random.default_rng(2)
    sky = _rand_sky(rng, H=4, W=8)
    pix = RD.window_pixels(view)[::53]
    grads = rng.normal(size=(len(pix), 8))
    _, gr = AD.render_and_grad(scene, view, dict(opts, sky=sky), grads, pix)

    def loss(s):
        out = RD.render_pixels(scene, view, dict(opts, sky=s), pix)
        return float((out * grads).sum())

    base = loss(sky)
    top = np.argsort(-np.abs(gr["sky"]).ravel())[:4]
    assert np.abs(gr["sky"].ravel()[top]).min() > 0
    for (c, j, i) in [np.unravel_index(t, sky.shape) for t in top]:
        s2 = sky.copy()
        s2[c, j, i] += 0.5
        fd = (loss(s2) - base) / 0.5
        assert abs(fd - gr["sky"][c, j, i]) < 1e-9 * max(1.0, abs(fd)), (c, j, i)
    # some texels are hit
    assert np.abs(gr["sky"]).sum() > 0
