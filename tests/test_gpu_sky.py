"""GPU sky environment map (Sec. 3.1, Eq. 2) against the FP64 oracle,
through the C ABI: the composite C_voxels + T_final C_sky, the map's
gradient T_final G_C over the bilinear taps, and the voxel and pose
gradients, which see C_sky through the transmittance's share of L.

Bars: outputs within 1e-4 absolute; every gradient elementwise within
1e-3 of max(|ref|, 1e-2 max|ref|) (chunked tiles: 1e-3 in the 2-norm for
the sky map).  The pose gradients (a 3x3 and a 3-vector per actor) are
signed sums over every pixel; the oracle also reports each element's
summand magnitude (sum of |contribution|, thousands of times the element
where it cancels), and the bar adds the FP32 rounding of those summands,
2^-20 of that magnitude (one element of the seed-1 scene sums to 0.0356
from summands of total magnitude 4505; its FP32 error, 2.7e-4, is 6e-8 =
one ulp of that magnitude).  The map gradient's bar also adds, per texel,
the FP32 error of the tap positions (see _tap_position_bound): the map
coordinates come from the FP32 ray direction, and longitude is
ill-conditioned near the poles."""
import numpy as np
import pytest

from oracle import adjoint as AD
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


# FP32 position of a ray's taps on the map.  The kernels compute the ray
# direction in FP32 (each component within EPS_D of the exact unit vector)
# and the map coordinates from it, so a tap's weight moves by up to
#   du + dv,  du = W / (2 pi) EPS_D / |d_xy| + EPS_U W,
#             dv = H / pi EPS_D + EPS_U H
# (longitude is ill-conditioned near the poles, where |d_xy| -> 0; EPS_U
# covers the rounding of the coordinate arithmetic itself), and near a
# texel boundary the tap with the small weight may fall on the neighbour
# of the oracle's texel.  The map-gradient bar adds, per texel, that weight
# error times |T_final G_C| of every pixel whose taps lie within one texel.
EPS_D = 8 * 2.0 ** -24
EPS_U = 4 * 2.0 ** -24


def _tap_position_bound(view, T, Grgb, shape):
    from oracle import geometry as GEO
    from oracle import sky as SK
    _, H, W = shape
    out = np.zeros(shape)
    pix = RD.window_pixels(view)
    for (px, py) in pix:
        y, x = py - view["y0"], px - view["x0"]
        _, d = GEO.camera_ray(view, px, py)
        rho = max(np.hypot(d[0], d[1]), 1e-30)
        du = W / (2 * np.pi) * EPS_D / rho + EPS_U * W
        dv = H / np.pi * EPS_D + EPS_U * H
        dw = min(1.0, du + dv)
        t = SK.taps(d, W, H)
        rows = {min(max(j + o, 0), H - 1) for j, _, _ in t for o in (-1, 0, 1)}
        cols = {(i + o) % W for _, i, _ in t for o in (-1, 0, 1)}
        g = np.abs(T[y, x] * Grgb[:, y, x]) * dw
        for j in rows:
            for i in cols:
                out[:, j, i] += g
    return out


def _sky32(seed, H=16, W=32):
    rng = np.random.default_rng(100 + seed)
    return rng.uniform(0.0, 1.0, size=(3, H, W)).astype(np.float32)


def _run(ctx, cfg, sky, seed, normals=True):
    import torch
    from paper_2606_23031_amd import dv
    scene, view, opts = cfg["scene"], cfg["views"][0], cfg["opts"]
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_T
    if normals:
        mask |= dv.DV_OUT_NORMAL
    sky_t = torch.tensor(sky, device="cuda")
    sc = dv.Scene(ctx, scene)
    outs = dv.alloc_outputs([view], mask)
    st = dv.dv_render(ctx, sc, [view], dv.make_opts(dict(opts, sky=sky_t), mask),
                      outs, keep=True)
    rng = np.random.default_rng(seed)
    h, w = view["h"], view["w"]
    G = dict(rgb=rng.normal(size=(3, h, w)), depth=rng.normal(size=(h, w)) * 0.3,
             normal=rng.normal(size=(3, h, w)) if normals else np.zeros((3, h, w)),
             T=rng.normal(size=(h, w)))
    gt = {k: torch.tensor(v, dtype=torch.float32, device="cuda") for k, v in G.items()}
    if not normals:
        gt["normal"] = None
    acc = [dict(corner=torch.zeros(len(o["corner_density"]), device="cuda"),
                sh=torch.zeros(o["sh"].shape, device="cuda"))
           for o in scene["octrees"]]
    na = len(scene["octrees"]) - 1
    pg = torch.zeros(1, max(na, 1), 12, device="cuda")
    sg = torch.zeros(sky.shape, device="cuda")
    dv.dv_render_backward(ctx, sc, st, [gt], acc, pg, sky_grad=sg)
    torch.cuda.synchronize()
    dv.dv_fwd_state_release(st)
    got = {k: (t.cpu().numpy().astype(np.float64) if t is not None else None)
           for k, t in outs[0].items()}
    # oracle on the same (float32) map
    o_opts = dict(opts, sky=sky.astype(np.float64))
    pix = RD.window_pixels(view)
    gy, gx = pix[:, 1] - view["y0"], pix[:, 0] - view["x0"]
    grads = np.zeros((len(pix), 8))
    g32 = {k: v.astype(np.float32).astype(np.float64) for k, v in G.items()}
    grads[:, 0:3] = g32["rgb"][:, gy, gx].T
    grads[:, 3] = g32["depth"][gy, gx]
    grads[:, 4:7] = g32["normal"][:, gy, gx].T
    grads[:, 7] = g32["T"][gy, gx]
    out, ref = AD.render_and_grad(scene, view, o_opts, grads, pix)
    ref_img = dict(rgb=out[:, 0:3].T.reshape(3, h, w), depth=out[:, 3].reshape(h, w),
                   normal=out[:, 4:7].T.reshape(3, h, w), T=out[:, 7].reshape(h, w))
    ref["sky_pos"] = _tap_position_bound(view, ref_img["T"], g32["rgb"], sky.shape)
    return got, ref_img, acc, pg, sg, ref


@pytest.mark.parametrize("seed", [0, 1])
def test_sky_forward_and_backward_match_oracle(ctx, seed):
    cfg = actor_scene(seed=seed, n_actors=2, deg=2)
    cfg["opts"] = dict(cfg["opts"], eps_stop=0.0)
    sky = _sky32(seed)
    got, ref_img, acc, pg, sg, ref = _run(ctx, cfg, sky, seed)
    for k in ("rgb", "depth", "normal", "T"):
        err = float(np.abs(got[k] - ref_img[k]).max())
        print(f"  {k}: max abs err {err:.3e}")
        assert err <= 1e-4, (k, err)
    # the sky is visible: some texels receive gradient
    assert np.abs(ref["sky"]).max() > 0
    _close("sky", sg.cpu().numpy(), ref["sky"], extra=ref["sky_pos"])
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])
        _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k])
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1],
               summed=ref["dR_abs"][i + 1])
        _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1],
               summed=ref["dp_abs"][i + 1])


def test_constant_map_equals_constant_background(ctx):
    import torch
    from paper_2606_23031_amd import dv
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=5, n_actors=2, deg=1)
    v = cfg["views"][0]
    col = (0.25, 0.5, 0.75)
    a, _, sc = render_gpu(ctx, cfg["scene"], [v], dict(cfg["opts"], bg=col))
    sky = torch.empty(3, 8, 16, device="cuda")
    for c in range(3):
        sky[c] = col[c]
    b, _, _ = render_gpu(ctx, cfg["scene"], [v],
                         dict(cfg["opts"], bg=(9.0, 9.0, 9.0), sky=sky), dv_scene=sc)
    for k in ("rgb", "depth", "normal", "T"):
        assert np.abs(a[0][k] - b[0][k]).max() <= 1e-6, k


def test_sky_chunked_tiles(ctx):
    # chunked tiles: T_final is the product of the chunks' transmittances,
    # and the T_final C_sky term enters S_after of every chunk, so corner,
    # SH and pose gradients of chunked tiles see the map too
    from test_gpu_backward import _dense_bar
    cfg = dense_scene(seed=1, deg=1)
    cfg["opts"] = dict(cfg["opts"], eps_stop=0.0)
    sky = _sky32(7, H=32, W=64)
    got, ref_img, acc, pg, sg, ref = _run(ctx, cfg, sky, 7)
    for k in ("rgb", "depth", "normal", "T"):
        tol = 1e-4 * (1.0 + np.abs(ref_img["depth"])) if k == "depth" else 1e-4
        err = np.abs(got[k] - ref_img[k])
        print(f"  {k}: max abs err {float(err.max()):.3e}")
        assert np.all(err <= tol), k
    g, r = sg.cpu().numpy().astype(np.float64), ref["sky"]
    assert np.abs(r).max() > 0
    rel = np.linalg.norm(g - r) / np.linalg.norm(r)
    print(f"  sky grad: relative 2-norm error {rel:.3e}")
    assert rel <= 1e-3
    _dense_bar(acc, pg, ref)


def test_sky_zenith_wide_map(ctx):
    """A view that contains the zenith, with a map 256 texels wide: near the
    pole a tile's rays cover every column of the top rows, so the tile's
    texel footprint exceeds the 256-entry LDS table and the map gradient
    takes the direct-atomic path (and the wrapped columns of the pole rows
    repeat texels).  Outputs and every gradient against the oracle."""
    from synth.configs import make_view, look_at_c2w
    cfg = actor_scene(seed=2, n_actors=2, deg=2)
    cfg["opts"] = dict(cfg["opts"], eps_stop=0.0)
    v = cfg["views"][0]
    # below both actors inside the background cube, looking straight up
    # (the up vector only fixes the image's roll)
    eye = np.array([0.05, 0.02, -1.5])
    c2w = look_at_c2w(eye, eye + np.array([0.0, 0.0, 1.0]), up=(1.0, 0.0, 0.0))
    cfg["views"] = [make_view(64, 48, 90.0, c2w, t=v["t"])]
    sky = _sky32(11, H=64, W=256)
    got, ref_img, acc, pg, sg, ref = _run(ctx, cfg, sky, 11)
    for k in ("rgb", "depth", "normal", "T"):
        err = float(np.abs(got[k] - ref_img[k]).max())
        print(f"  {k}: max abs err {err:.3e}")
        assert err <= 1e-4, (k, err)
    assert np.abs(ref["sky"]).max() > 0
    # the taps of the pole row go all the way round in longitude (the tiles
    # next to the zenith span half the map's columns or more)
    cols = np.nonzero(np.abs(ref["sky"][:, 0, :]).sum(0))[0]
    gaps = np.diff(np.concatenate([cols, cols[:1] + sky.shape[2]]))
    assert len(cols) > 8 and gaps.max() < sky.shape[2] // 4
    _close("sky", sg.cpu().numpy(), ref["sky"], extra=ref["sky_pos"])
    for k in range(len(acc)):
        if np.abs(ref["corner"][k]).max() > 0:
            _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])
            _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k])
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        if np.abs(ref["dR"][i + 1]).max() > 0:
            _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1],
                   summed=ref["dR_abs"][i + 1])
            _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1],
                   summed=ref["dp_abs"][i + 1])


def test_autograd_sky_gradient(ctx):
    """The autograd binding returns dL/dsky for a map that requires grad,
    equal to the oracle's (and so to a direct dv_render_backward call)."""
    import torch
    from paper_2606_23031_amd import dv
    from paper_2606_23031_amd.autograd import render
    cfg = actor_scene(seed=0, n_actors=2, deg=2)
    scene, view = cfg["scene"], cfg["views"][0]
    opts = dict(cfg["opts"], eps_stop=0.0)
    sky = _sky32(0)
    sky_t = torch.tensor(sky, device="cuda").requires_grad_(True)
    sc = dv.Scene(ctx, scene)
    mask = dv.DV_OUT_RGB | dv.DV_OUT_T
    out = render(ctx, sc, [view], dict(opts, sky=sky_t), mask)[0]
    rng = np.random.default_rng(21)
    h, w = view["h"], view["w"]
    G = rng.normal(size=(3, h, w)).astype(np.float32)
    (out["rgb"] * torch.tensor(G, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    assert sky_t.grad is not None
    pix = RD.window_pixels(view)
    gy, gx = pix[:, 1] - view["y0"], pix[:, 0] - view["x0"]
    grads = np.zeros((len(pix), 8))
    grads[:, 0:3] = G.astype(np.float64)[:, gy, gx].T
    _, ref = AD.render_and_grad(scene, view, dict(opts, sky=sky.astype(np.float64)),
                                grads, pix)
    _close("sky (autograd)", sky_t.grad.cpu().numpy(), ref["sky"])
