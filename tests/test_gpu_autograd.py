"""The torch.autograd binding: gradients reached through loss.backward() must
equal the oracle's FP64 adjoint (gradient bar of test_gpu_backward) for
corner densities, SH coefficients and explicit actor poses."""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import render as RD
from scenes import actor_scene

pytestmark = pytest.mark.gpu


def _close(name, g, ref, rel=1e-3, floor=1e-2):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    if scale == 0.0:
        assert np.abs(g).max() == 0.0, name
        return
    bound = rel * np.maximum(np.abs(ref), floor * scale)
    err = np.abs(g - ref)
    print(f"  {name}: max|ref| {scale:.3e} worst err/bound {(err / bound).max():.3f}")
    assert np.all(err <= bound), name


def test_autograd_matches_oracle_adjoint():
    import torch
    from paper_2606_23031_amd import dv
    from paper_2606_23031_amd.autograd import render, track_poses
    cfg = actor_scene(seed=5, n_actors=2, deg=2)
    scene, view, opts = cfg["scene"], cfg["views"][0], cfg["opts"]
    ctx = dv.dv_ctx_create(0)
    sc = dv.Scene(ctx, scene)
    for o in sc.octs:
        o["corner_density"].requires_grad_(True)
        o["sh"].requires_grad_(True)
    poses = track_poses(scene, [view]).requires_grad_(True)
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_NORMAL | dv.DV_OUT_T
    out = render(ctx, sc, [view], opts, mask, poses=poses)[0]
    rng = np.random.default_rng(5)
    h, w = view["h"], view["w"]
    G = dict(rgb=rng.normal(size=(3, h, w)), depth=0.3 * rng.normal(size=(h, w)),
             normal=rng.normal(size=(3, h, w)), T=rng.normal(size=(h, w)))
    Gt = {k: torch.tensor(v, dtype=torch.float32, device="cuda") for k, v in G.items()}
    loss = sum((out[k] * Gt[k]).sum() for k in G)
    loss.backward()
    torch.cuda.synchronize()
    pix = RD.window_pixels(view)
    gy, gx = pix[:, 1] - view["y0"], pix[:, 0] - view["x0"]
    g32 = {k: v.astype(np.float32).astype(np.float64) for k, v in G.items()}
    grads = np.zeros((len(pix), 8))
    grads[:, 0:3] = g32["rgb"][:, gy, gx].T
    grads[:, 3] = g32["depth"][gy, gx]
    grads[:, 4:7] = g32["normal"][:, gy, gx].T
    grads[:, 7] = g32["T"][gy, gx]
    _, ref = AD.render_and_grad(scene, view, opts, grads, pix)
    for k, o in enumerate(sc.octs):
        _close(f"corner[{k}]", o["corner_density"].grad.cpu().numpy(), ref["corner"][k])
        _close(f"sh[{k}]", o["sh"].grad.cpu().numpy(), ref["sh"][k])
    gp = poses.grad.numpy()[0]
    for i in range(sc.n_actors):
        _close(f"dR[{i}]", gp[i, :9].reshape(3, 3), ref["dR"][i + 1])
        _close(f"dp[{i}]", gp[i, 9:], ref["dp"][i + 1])


def test_autograd_descent_step_lowers_l1():
    """One plain gradient step on corner densities and SH through the binding
    lowers an L1 photometric loss against a fixed target (the training use
    the binding serves); the state of the step is released by backward."""
    import torch
    from paper_2606_23031_amd import dv
    from paper_2606_23031_amd.autograd import render
    cfg = actor_scene(seed=6, n_actors=2, deg=1)
    scene, view, opts = cfg["scene"], cfg["views"][0], cfg["opts"]
    ctx = dv.dv_ctx_create(0)
    sc = dv.Scene(ctx, scene)
    params = []
    for o in sc.octs:
        params += [o["corner_density"].requires_grad_(True), o["sh"].requires_grad_(True)]
    target = torch.rand(3, view["h"], view["w"], device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(6))
    losses = []
    for _ in range(3):
        rgb = render(ctx, sc, [view], opts, dv.DV_OUT_RGB)[0]["rgb"]
        loss = (rgb - target).abs().mean()
        losses.append(float(loss))
        for p in params:
            p.grad = None
        loss.backward()
        with torch.no_grad():
            for p in params:
                p -= 5.0 * p.grad
    print("  L1:", losses)
    assert losses[1] < losses[0] and losses[2] < losses[1]
