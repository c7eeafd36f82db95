"""P14: the oracle's analytic adjoint against FP64 central differences."""
import copy

import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import render as RD
from oracle import geometry as G
from scenes import actor_scene

H = 1e-6


def _loss(scene, view, opts, pixels, gout, pose_override):
    out = RD.render_pixels(scene, view, opts, pixels, pose_override)
    return float((out * gout).sum())


def _f64(scene):
    sc = copy.deepcopy(scene)
    for o in sc["octrees"]:
        o["corner_density"] = o["corner_density"].astype(np.float64)
        o["sh"] = o["sh"].astype(np.float64)
    return sc


def _pick_pixels(scene, view, opts, n, rng):
    """Pixels whose rays cross actor boxes (so pose terms are exercised)
    plus a few plain background pixels."""
    ctx = RD.ViewContext(scene, view, opts)
    hit, other = [], []
    for py in range(view["h"]):
        for px in range(view["w"]):
            o, d = G.camera_ray(view, px, py)
            own, boxes = RD.owned_intervals(ctx, RD.ray_frames(ctx, o, d))
            (hit if boxes else other).append((px, py))
    rng.shuffle(hit)
    rng.shuffle(other)
    return np.array(hit[:n] + other[:max(2, n // 4)])


@pytest.mark.parametrize("seed,K,overlap", [(0, 1, False), (1, 2, False),
                                            (2, 1, True)])
def test_p14_adjoint_matches_central_differences(seed, K, overlap):
    rng = np.random.default_rng(100 + seed)
    cfg = actor_scene(seed=seed, n_actors=2, deg=2, K=K, overlap=overlap)
    sc, v = _f64(cfg["scene"]), cfg["views"][0]
    opts = dict(cfg["opts"], K=K, eps_stop=0.0)
    pix = _pick_pixels(sc, v, opts, 10, rng)
    gout = rng.normal(size=(len(pix), 8))
    ctx = RD.ViewContext(sc, v, opts)
    poses = [(ctx.oct[k]["R"].copy(), ctx.oct[k]["p"].copy())
             for k in range(1, len(sc["octrees"]))]
    _, grads = AD.render_and_grad(sc, v, opts, gout, pix, poses)

    def check(analytic, perturb):
        fd = (perturb(+H) - perturb(-H)) / (2 * H)
        if abs(analytic - fd) <= 1e-6 * abs(fd) + 2e-8:
            return fd
        # the loss is piecewise smooth (leaf and box faces sweep over the
        # fixed pixel rays); near a face the O(h^2) term of the h = 1e-6
        # difference can exceed the bound, so retry with a 10x smaller step
        # (round-off then ~1e-16 |L| / 1e-7)
        h2 = H / 10
        fd2 = (perturb(+h2) - perturb(-h2)) / (2 * h2)
        assert abs(analytic - fd2) <= 1e-6 * abs(fd2) + 2e-7, (analytic, fd, fd2)
        return fd2

    n_checked = 0
    # corner densities: those with a non-zero analytic gradient, plus zeros
    for k in range(len(sc["octrees"])):
        g = grads["corner"][k]
        nz = np.nonzero(np.abs(g) > 1e-6)[0]
        picks = list(rng.choice(nz, size=min(4, nz.size), replace=False)) if nz.size else []
        zz = np.nonzero(g == 0)[0]
        picks += list(rng.choice(zz, size=min(1, zz.size), replace=False))
        for c in picks:
            def pert(hh, k=k, c=c):
                s2 = copy.deepcopy(sc)
                s2["octrees"][k]["corner_density"][c] += hh
                return _loss(s2, v, opts, pix, gout, poses)
            check(g[c], pert)
            n_checked += 1
    # SH coefficients
    for k in range(len(sc["octrees"])):
        g = grads["sh"][k]
        nz = np.argwhere(np.abs(g) > 1e-6)
        for idx in nz[rng.choice(len(nz), size=min(4, len(nz)), replace=False)]:
            s_, c_, v_ = idx

            def pert(hh, k=k, s_=s_, c_=c_, v_=v_):
                s2 = copy.deepcopy(sc)
                s2["octrees"][k]["sh"][s_, c_, v_] += hh
                return _loss(s2, v, opts, pix, gout, poses)
            check(g[s_, c_, v_], pert)
            n_checked += 1
    # poses: every entry of R and p of every actor
    for i in range(len(poses)):
        for a in range(3):
            for b in range(3):
                def pert(hh, i=i, a=a, b=b):
                    pp = [(R.copy(), p.copy()) for R, p in poses]
                    pp[i][0][a, b] += hh
                    return _loss(sc, v, opts, pix, gout, pp)
                check(grads["dR"][i + 1][a, b], pert)
            def pertp(hh, i=i, a=a):
                pp = [(R.copy(), p.copy()) for R, p in poses]
                pp[i][1][a] += hh
                return _loss(sc, v, opts, pix, gout, pp)
            check(grads["dp"][i + 1][a], pertp)
    assert n_checked > 8
    assert max(np.abs(grads["dR"][i + 1]).max() for i in range(len(poses))) > 1e-3
