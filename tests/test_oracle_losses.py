"""Pins of the oracle's training losses and optimiser step (Supp.
'Optimization Details', Training Losses): SSIM against a brute-force
window evaluation and its closed forms, every gradient against central
differences, the simple terms against hand-computed values, and Adam
against torch's implementation."""
import math

import numpy as np
import pytest

from oracle import losses as LS

LAM = dict(color=1.0, ssim=0.2, depth=0.3, normal=0.05, sky=0.1)


def _ssim_bruteforce(x, y, size=11, sigma=1.5):
    """Windowed moments with explicit loops (zero outside the image)."""
    H, W = x.shape
    r = size // 2
    g1 = [math.exp(-((i - r) ** 2) / (2 * sigma * sigma)) for i in range(size)]
    s1 = sum(g1)
    wts = [[g1[i] * g1[j] / (s1 * s1) for j in range(size)] for i in range(size)]
    tot = 0.0
    for py in range(H):
        for px in range(W):
            mx = my = exx = eyy = exy = 0.0
            for i in range(size):
                for j in range(size):
                    qy, qx = py + i - r, px + j - r
                    if 0 <= qy < H and 0 <= qx < W:
                        a, b, wt = x[qy, qx], y[qy, qx], wts[i][j]
                        mx += wt * a
                        my += wt * b
                        exx += wt * a * a
                        eyy += wt * b * b
                        exy += wt * a * b
            sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
            c1, c2 = 0.01 ** 2, 0.03 ** 2
            tot += ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return tot / (H * W)


def test_ssim_matches_bruteforce_windows():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(1, 9, 13))
    y = np.clip(x + 0.2 * rng.normal(size=x.shape), 0, 1)
    assert abs(LS.ssim(x, y) - _ssim_bruteforce(x[0], y[0])) < 1e-13


def test_ssim_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 20, 24))
    assert abs(LS.ssim(x, x) - 1.0) < 1e-12
    # at x = y SSIM is maximal: the gradient vanishes
    assert np.abs(LS.ssim_grad(x, x)).max() < 1e-12
    # constant images a, b: variances vanish away from the border, where
    # S = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    S, _ = LS.ssim_map(np.full((30, 30), a), np.full((30, 30), b),
                       LS.gaussian_window())
    ref = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    assert abs(S[15, 15] - ref) < 1e-12


def test_window_is_normalised_gaussian():
    w = LS.gaussian_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    g = np.exp(-(np.arange(11) - 5.0) ** 2 / (2 * 1.5 ** 2))
    assert np.allclose(w[5] / w[5, 5], g, atol=1e-15)


def _planes(rng, H=10, W=14):
    out = dict(rgb=rng.uniform(size=(3, H, W)), depth=rng.uniform(1, 5, size=(H, W)),
               normal=rng.normal(size=(3, H, W)), T=rng.uniform(size=(H, W)))
    out["normal"][:, 0, 0] = 0.0          # an empty ray
    tgt = dict(rgb=rng.uniform(size=(3, H, W)),
               depth=np.where(rng.uniform(size=(H, W)) < 0.3,
                              rng.uniform(1, 5, size=(H, W)), 0.0),
               normal=rng.normal(size=(3, H, W)),
               sky=(rng.uniform(size=(H, W)) < 0.25).astype(np.float64))
    tgt["normal"][:, 1, :3] = 0.0         # no pseudo normal there
    return out, tgt


def test_total_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    out, tgt = _planes(rng)
    _, _, grads = LS.training_loss(out, tgt, LAM)
    h = 1e-6
    for key in ("rgb", "depth", "normal", "T"):
        flat = out[key].reshape(-1)
        for idx in rng.choice(flat.size, 12, replace=False):
            p = {k: v.copy() for k, v in out.items()}
            m = {k: v.copy() for k, v in out.items()}
            p[key].reshape(-1)[idx] += h
            m[key].reshape(-1)[idx] -= h
            fd = (LS.training_loss(p, tgt, LAM)[1] - LS.training_loss(m, tgt, LAM)[1]) / (2 * h)
            an = grads[key].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (key, idx, fd, an)


def test_simple_terms_hand_computed():
    z = np.zeros((1, 2))
    out = dict(rgb=np.zeros((3, 1, 2)), depth=np.array([[2.0, 5.0]]),
               normal=np.stack([np.array([[1.0, 0.0]]), np.array([[0.0, 2.0]]), z]),
               T=np.array([[0.5, 0.9]]))
    tgt = dict(rgb=np.zeros((3, 1, 2)), depth=np.array([[3.5, 0.0]]),
               normal=np.stack([np.array([[0.0, 0.0]]), np.array([[1.0, -3.0]]), z]),
               sky=np.array([[1.0, 0.0]]))
    terms, _, _ = LS.training_loss(out, tgt, LAM)
    assert terms["depth"] == 1.5                      # only pixel 0 has LiDAR
    # pixel 0: (1,0,0) vs (0,1,0): cos 0; pixel 1: (0,2,0) vs (0,-3,0): cos -1
    assert abs(terms["normal"] - 1.5) < 1e-15
    assert terms["sky"] == 0.25                       # (0.5 - 1)^2 on pixel 0
    assert terms["l1"] == 0.0


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = LS.adam_step(p, g, m, v, t, 0.01)
        assert np.abs(p - tp.detach().numpy()).max() < 1e-14
    # first step: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    p1, _, _ = LS.adam_step(p0, grads[0], np.zeros(50), np.zeros(50), 1, 0.01)
    g0 = grads[0]
    assert np.allclose(p0 - p1, 0.01 * g0 / (np.abs(g0) + 1e-8), atol=1e-16, rtol=1e-14)
