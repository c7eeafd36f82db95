"""Pins of the analytic SH direction gradient (Sec. 3.1 colour; used by the
camera-position term of pose gradients): closed forms of the degree-1 and
degree-2 functions, the polynomial identity it rests on, scale invariance
and central differences of the basis itself."""
import math

import numpy as np

from oracle import sh as SH


def _dirs(n=64, seed=0):
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(n, 3))
    return w / np.linalg.norm(w, axis=1, keepdims=True)


def _proj(w, g):
    return g - (g @ w) * w


def test_polynomial_form_equals_basis():
    w = np.concatenate([_dirs(), [[0, 0, 1.0], [0, 0, -1.0], [1, 0, 0]]])
    assert np.abs(SH.basis_polynomial_form(w, 3) - SH.basis(w, 3)).max() < 1e-14


def test_closed_form_low_degrees():
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    c2 = 0.5 * math.sqrt(15.0 / math.pi)
    c20 = 0.25 * math.sqrt(5.0 / math.pi)
    for w in _dirs(16, 1):
        x, y, z = w
        g = SH.basis_grad(w[None], 2)[0]
        assert np.allclose(g[0], 0.0, atol=1e-15)
        # Y_{1,-1} = c1 y, Y_{1,0} = c1 z, Y_{1,1} = c1 x
        for idx, e in ((1, [0, 1, 0]), (2, [0, 0, 1]), (3, [1, 0, 0])):
            assert np.allclose(g[idx], _proj(w, c1 * np.array(e, float)),
                               atol=1e-14)
        # Y_{2,-2} = c2 x y and Y_{2,2} = c2 / 2 (x^2 - y^2)
        assert np.allclose(g[4], _proj(w, c2 * np.array([y, x, 0.0])),
                           atol=1e-14)
        assert np.allclose(g[8], _proj(w, c2 * np.array([x, -y, 0.0])),
                           atol=1e-14)
        # Y_{2,0} = c20 (3 z^2 - 1) on the sphere
        assert np.allclose(g[6], _proj(w, c20 * np.array([0, 0, 6 * z])),
                           atol=1e-14)


def test_gradient_is_tangent():
    w = _dirs()
    g = SH.basis_grad(w, 3)
    assert np.abs(np.einsum("nsa,na->ns", g, w)).max() < 1e-14


def _fd(w, h):
    fd = np.zeros(w.shape[:-1] + (16, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        p, q = w + e, w - e
        p = p / np.linalg.norm(p, axis=-1, keepdims=True)
        q = q / np.linalg.norm(q, axis=-1, keepdims=True)
        fd[..., a] = (SH.basis(p, 3) - SH.basis(q, 3)) / (2 * h)
    return fd


def test_gradient_matches_central_differences():
    w = _dirs(200, 2)
    assert np.abs(SH.basis_grad(w, 3) - _fd(w, 1e-5)).max() < 1e-8
    # at the poles the longitude is undefined but the functions are smooth
    poles = np.array([[0, 0, 1.0], [0, 0, -1.0]])
    assert np.abs(SH.basis_grad(poles, 3) - _fd(poles, 1e-4)).max() < 1e-6
