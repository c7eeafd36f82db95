"""Feature accumulation render (Sec. 4.3, 3D semantic segmentation) on the
GPU through the C ABI: per-leaf F-channel features composited in place of
the SH colour, three channels per render, and the backward's feature
gradient (the fusion of per-pixel features into the leaves), against the
FP64 oracle; and three channels equal to the colours reproduce the colour
render bit for bit."""
import numpy as np
import pytest

from oracle import features as FT
from oracle import render as RD
from scenes import actor_scene, dense_scene
from test_gpu_backward import _close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from gpu_helpers import gpu_ctx
    return gpu_ctx()


def _feat_tensors(scene, F, seed):
    import torch
    rng = np.random.default_rng(seed)
    host = [rng.normal(size=(F, len(o["level"]))).astype(np.float32)
            for o in scene["octrees"]]
    return host, [torch.tensor(h, device="cuda") for h in host]


def test_three_colour_channels_reproduce_colour_render(ctx):
    import torch
    from paper_2606_23031_amd import dv
    cfg = actor_scene(seed=21, n_actors=2, deg=0)
    scene, view = cfg["scene"], cfg["views"][0]
    opts = dict(cfg["opts"], bg=(0.0, 0.0, 0.0), eps_stop=1e-4)
    sc = dv.Scene(ctx, scene)
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_T
    ref = dv.alloc_outputs([view], mask)
    dv.dv_render(ctx, sc, [view], dv.make_opts(opts, mask), ref)
    # the leaf colours exactly as the preprocess forms them (degree 0:
    # max(0, Y00 k + 1/2) in FP32)
    y00 = torch.tensor(0.28209479177387814, dtype=torch.float32, device="cuda")
    feats = [torch.clamp(o["sh"][0] * y00 + 0.5, min=0.0).contiguous()
             for o in sc.octs]
    got = dv.alloc_outputs([view], mask)
    dv.dv_render(ctx, sc, [view], dv.make_opts(dict(opts, feat=feats, feat_group=0),
                                               mask), got)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "T"):
        assert torch.equal(ref[0][k], got[0][k]), k


@pytest.mark.parametrize("dense", [False, True])
def test_feature_render_and_fusion_match_oracle(ctx, dense):
    import torch
    from paper_2606_23031_amd import dv
    cfg = dense_scene(seed=2, deg=1) if dense else actor_scene(seed=22, n_actors=2, deg=1)
    scene, view = cfg["scene"], cfg["views"][0]
    if dense:
        # two tiles of the dense scene (chunked lists); keeps the oracle short
        view = dict(view, x0=16, y0=16, w=32, h=16)
    opts = dict(cfg["opts"], eps_stop=0.0)
    F = 5
    host, feats = _feat_tensors(scene, F, 23)
    sc = dv.Scene(ctx, scene)
    h, w = view["h"], view["w"]
    out = [torch.zeros(F, h, w, device="cuda")]
    states = dv.render_features(ctx, sc, [view], opts, feats, out,
                                mask=dv.DV_OUT_DEPTH | dv.DV_OUT_T, keep=True)
    torch.cuda.synchronize()
    pix = RD.window_pixels(view)
    ref, T = FT.render_features(scene, view, opts, [x.astype(np.float64) for x in host],
                                pix)
    got = out[0].cpu().numpy().reshape(F, -1).T
    err = float(np.abs(got - ref).max())
    print(f"  features: max abs err {err:.3e} (max |ref| {np.abs(ref).max():.2f})")
    assert err <= 1e-4
    assert float(np.abs(states[0][1][0]["T"].cpu().numpy().ravel() - T).max()) <= 1e-4
    # backward of each group with a random upstream feature gradient
    rng = np.random.default_rng(24)
    GF = rng.normal(size=(F, h, w)).astype(np.float32)
    acc = [dict(corner=torch.zeros(len(o["corner_density"]), device="cuda"),
                feat=torch.zeros(F, len(o["level"]), device="cuda"))
           for o in scene["octrees"]]
    na = len(scene["octrees"]) - 1
    pg = torch.zeros(1, na, 12, device="cuda")
    gy, gx = pix[:, 1] - view["y0"], pix[:, 0] - view["x0"]
    rcorner = [np.zeros(len(o["corner_density"])) for o in scene["octrees"]]
    rcorner_abs = [np.zeros(len(o["corner_density"])) for o in scene["octrees"]]
    rfeat = [np.zeros((F, len(o["level"]))) for o in scene["octrees"]]
    rfeat_abs = [np.zeros((F, len(o["level"]))) for o in scene["octrees"]]
    rdR = [np.zeros((3, 3)) for _ in scene["octrees"]]
    rdp = [np.zeros(3) for _ in scene["octrees"]]
    for g, (st, tmp) in enumerate(states):
        nc = min(3, F - 3 * g)
        gi = torch.zeros(3, h, w, device="cuda")
        gi[:nc] = torch.tensor(GF[3 * g:3 * g + nc], device="cuda")
        dv.dv_render_backward(ctx, sc, st, [dict(rgb=gi)], acc, pg)
        dv.dv_fwd_state_release(st)
        G = np.zeros((len(pix), 8))
        G[:, 0:nc] = GF[3 * g:3 * g + nc][:, gy, gx].T
        r = FT.feature_adjoint(scene, view, opts, [x.astype(np.float64) for x in host],
                               pix, G, g)
        for k in range(len(scene["octrees"])):
            rfeat[k][3 * g:3 * g + nc] = r["feat"][k][:nc]
            rfeat_abs[k][3 * g:3 * g + nc] = r["feat_abs"][k][:nc]
            rcorner[k] += r["corner"][k]
            rcorner_abs[k] += r["corner_abs"][k]
            rdR[k] += r["dR"][k]
            rdp[k] += r["dp"][k]
    torch.cuda.synchronize()
    if dense:
        from test_gpu_fullsize import _close as close_sum
        worst = {}
        for k in range(len(acc)):
            worst[f"feat[{k}]"] = close_sum(f"feat[{k}]", acc[k]["feat"].cpu().numpy(),
                                            rfeat[k], mag=rfeat_abs[k], rel_elem=1e-2)
            worst[f"corner[{k}]"] = close_sum(f"corner[{k}]", acc[k]["corner"].cpu().numpy(),
                                              rcorner[k], mag=rcorner_abs[k], rel_elem=1e-2)
        bad = {k: x for k, x in worst.items() if x > 1.0}
        assert not bad, bad
        return
    for k in range(len(acc)):
        _close(f"feat[{k}]", acc[k]["feat"].cpu().numpy(), rfeat[k])
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), rcorner[k])
    p = pg.cpu().numpy()[0]
    for i in range(na):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), rdR[i + 1])
        _close(f"dp[{i}]", p[i, 9:], rdp[i + 1])


def test_feature_render_rejects_bad_group(ctx):
    import torch
    from paper_2606_23031_amd import dv
    cfg = actor_scene(seed=25, n_actors=2, deg=0)
    sc = dv.Scene(ctx, cfg["scene"])
    _, feats = _feat_tensors(cfg["scene"], 4, 26)
    outs = dv.alloc_outputs(cfg["views"], dv.DV_OUT_RGB)
    with pytest.raises(dv.DVError) as ei:
        dv.dv_render(ctx, sc, cfg["views"],
                     dv.make_opts(dict(cfg["opts"], feat=feats, feat_group=2),
                                  dv.DV_OUT_RGB), outs)
    assert ei.value.status == -1
