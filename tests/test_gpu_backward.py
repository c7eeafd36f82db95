"""GPU backward parity against the oracle's FP64 adjoint (itself pinned to
central differences), through the C ABI.

Bar (gradient reading): per gradient tensor, elementwise
|g - g_ref| <= 1e-3 * max(|g_ref|, 1e-2 * max|g_ref|).  eps_stop = 0 so
both sides differentiate the same pieces.
"""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import render as RD
from scenes import actor_scene, dense_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from gpu_helpers import gpu_ctx
    return gpu_ctx()


# An FP32 summand carries a relative rounding error of a few ulps; a
# gradient element that is a signed sum of many summands inherits their
# errors in absolute terms, so where the oracle reports the element's
# summand magnitude (sum of |contribution|) the bar adds 2^-20 of it
# (16 ulps per summand) to the relative bar.
SUMMAND_ULPS = 2.0 ** -20


def _close(name, g, ref, rel=1e-3, floor=1e-2, summed=None, extra=None):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    if scale == 0.0:
        assert np.abs(g).max() == 0.0, name
        return
    bound = rel * np.maximum(np.abs(ref), floor * scale)
    if summed is not None:
        bound = bound + SUMMAND_ULPS * np.asarray(summed, np.float64)
    if extra is not None:
        bound = bound + np.asarray(extra, np.float64)
    err = np.abs(g - ref)
    worst = float((err / bound).max())
    print(f"  {name}: max|ref| {scale:.3e} worst err/bound {worst:.3f}")
    assert np.all(err <= bound), (name, worst)


def _run(ctx, cfg, mask_normals=True, seed=0, pose=True, normal_grad=True):
    import torch
    from paper_2606_23031_amd import dv
    scene, view, opts = cfg["scene"], cfg["views"][0], cfg["opts"]
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_T
    if mask_normals:
        mask |= dv.DV_OUT_NORMAL
    sc = dv.Scene(ctx, scene)
    outs = dv.alloc_outputs([view], mask)
    st = dv.dv_render(ctx, sc, [view], dv.make_opts(opts, mask), outs, keep=True)
    rng = np.random.default_rng(seed)
    h, w = view["h"], view["w"]
    G = dict(rgb=rng.normal(size=(3, h, w)), depth=rng.normal(size=(h, w)) * 0.3,
             normal=(rng.normal(size=(3, h, w)) if mask_normals and normal_grad
                     else np.zeros((3, h, w))),
             T=rng.normal(size=(h, w)))
    gt = {k: torch.tensor(v, dtype=torch.float32, device="cuda") for k, v in G.items()}
    if not (mask_normals and normal_grad):
        gt["normal"] = None
    acc = [dict(corner=torch.zeros(len(o["corner_density"]), device="cuda"),
                sh=torch.zeros(o["sh"].shape, device="cuda"))
           for o in scene["octrees"]]
    na = len(scene["octrees"]) - 1
    pg = torch.zeros(1, max(na, 1), 12, device="cuda") if pose else None
    dv.dv_render_backward(ctx, sc, st, [gt], acc, pg)
    torch.cuda.synchronize()
    dv.dv_fwd_state_release(st)
    # oracle
    pix = RD.window_pixels(view)
    gy, gx = pix[:, 1] - view["y0"], pix[:, 0] - view["x0"]
    grads = np.zeros((len(pix), 8))
    g32 = {k: v.astype(np.float32).astype(np.float64) for k, v in G.items()}
    grads[:, 0:3] = g32["rgb"][:, gy, gx].T
    grads[:, 3] = g32["depth"][gy, gx]
    grads[:, 4:7] = g32["normal"][:, gy, gx].T
    grads[:, 7] = g32["T"][gy, gx]
    _, ref = AD.render_and_grad(scene, view, opts, grads, pix)
    return acc, pg, ref, sc


@pytest.mark.parametrize("seed,K,overlap,normals", [
    (0, 1, False, True), (1, 2, False, True), (2, 1, True, True),
    (3, 1, False, False)])
def test_backward_matches_oracle_adjoint(ctx, seed, K, overlap, normals):
    cfg = actor_scene(seed=seed, n_actors=3 if overlap else 2, deg=2,
                      overlap=overlap, K=K)
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=normals, seed=seed)
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])
        _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k])
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1])
        _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1])


@pytest.mark.parametrize("fov", [30.0, 14.0])
def test_backward_actor_close_up(ctx, fov):
    """Actor leaves several pixels wide: the actor backward walks over the
    wave's entries with the butterfly reduction (all steps at 14 degrees,
    about half at 30, the rest per lane with per-lane slot adds)."""
    cfg = actor_scene(seed=13, n_actors=2, deg=2, fov=fov,
                      target=(-0.55, 0.33, 0.11))
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=True, seed=13)
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])
        _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k])
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1])
        _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1])


@pytest.mark.parametrize("n_actors", [12, 44])
def test_backward_crowded_tiles(ctx, n_actors):
    """Tiles holding 12 or 44 overlapping actor boxes (the segment
    builder's wide register sweep, and the sweep through memory).  Deep in
    the stack an actor owns a thin slice of each ray behind up to 2 n - 1
    segments: its gradients are small, while their absolute FP32 error is
    that of the whole ray's sums (background included).  So besides the
    summand-magnitude term, the floor of every array is taken from the
    largest gradient of the scene (1e-5 of it), not of that octree."""
    from scenes import crowd_scene
    cfg = crowd_scene(seed=4, n_actors=n_actors)
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=True, seed=4)
    top_c = max(float(np.abs(r).max()) for r in ref["corner"])
    top_s = max(float(np.abs(r).max()) for r in ref["sh"])
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k],
               summed=ref["corner_abs"][k], extra=1e-5 * top_c)
        _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k],
               summed=ref["sh_abs"][k], extra=1e-5 * top_s)
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1],
               summed=ref["dR_abs"][i + 1])
        _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1], summed=ref["dp_abs"][i + 1])


def test_backward_normals_rendered_without_normal_gradient(ctx):
    """Normals are rendered but no view passes a normal gradient: the
    backward runs without normal terms (they are exactly zero), and the
    gradients equal the oracle's adjoint with a zero normal gradient."""
    cfg = actor_scene(seed=5, n_actors=2, deg=2)
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=True, seed=5, normal_grad=False)
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])
        _close(f"sh[{k}]", acc[k]["sh"].cpu().numpy(), ref["sh"][k])
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        _close(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1])
        _close(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1])


def test_backward_without_pose_buffer(ctx):
    cfg = actor_scene(seed=4, n_actors=2, deg=1)
    acc, _, ref, _ = _run(ctx, cfg, seed=4, pose=False)
    for k in range(len(acc)):
        _close(f"corner[{k}]", acc[k]["corner"].cpu().numpy(), ref["corner"][k])


def test_backward_chunked_tiles(ctx):
    # tile lists split into chunks: chunk-local walks with T_pre / S_after
    # from the merged partials, segments spliced by the chunk that holds
    # them, the pieces around a segment possibly in different chunks
    cfg = dense_scene(seed=1, deg=1)
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=True, seed=1)
    _dense_bar(acc, pg, ref)


@pytest.mark.parametrize("overlap", [False, True])
def test_backward_chunked_actor_lists(ctx, overlap):
    # split (tile, actor) lists: chunk-local asset walks with W_c / R_c of
    # the segment, single-segment rays per chunk, two-segment rays whole
    cfg = dense_scene(seed=3, actor_level=4, overlap=overlap)
    acc, pg, ref, _ = _run(ctx, cfg, mask_normals=True, seed=3)
    _dense_bar(acc, pg, ref)


def _dense_bar(acc, pg, ref):
    """Scenes whose rays cross thousands of small leaves: each tensor within
    1e-3 relative in the 2-norm, and every significant element within 1e-2
    of the sum of |contributions| behind it.  Among thousands of chords some
    only graze a leaf; a chord of length l at distance t carries a relative
    FP32 error ~2^-24 t / l (the camera-relative leaf position itself is
    rounded to that), which reaches 1e-3 for l ~ 5e-4 t and can be the only
    contribution to a small leaf's gradient.  The elementwise bar is there
    to catch structural mistakes (a wrong chunk boundary or splice moves an
    element by its own size), the norm bar holds the tensor to 1e-3."""
    from test_gpu_fullsize import _close as close_sum
    worst = {}
    for k in range(len(acc)):
        worst[f"corner[{k}]"] = close_sum(f"corner[{k}]", acc[k]["corner"].cpu().numpy(),
                                          ref["corner"][k], mag=ref["corner_abs"][k],
                                          rel_elem=1e-2)
        worst[f"sh[{k}]"] = close_sum(f"sh[{k}]", acc[k]["sh"].cpu().numpy(),
                                      ref["sh"][k], mag=ref["sh_abs"][k], rel_elem=1e-2)
    p = pg.cpu().numpy()[0]
    for i in range(len(acc) - 1):
        worst[f"dR[{i}]"] = close_sum(f"dR[{i}]", p[i, :9].reshape(3, 3), ref["dR"][i + 1],
                                      rel_elem=1e-2)
        worst[f"dp[{i}]"] = close_sum(f"dp[{i}]", p[i, 9:], ref["dp"][i + 1], rel_elem=1e-2)
    bad = {k: w for k, w in worst.items() if w > 1.0}
    assert not bad, bad


def test_multiview_leaf_major_equals_views_alone(ctx):
    """Six views of the actor scene in one launch, with every leaf binned in
    most of them (more records than 1.5 x the leaves): the SH and corner
    gradients are then summed per leaf across its records (leaf-major
    pass).  They must equal the sum of the six views' gradients rendered
    one view at a time (one record per leaf and launch: the per-record pass
    the oracle adjoint checks above); pose gradients row by row."""
    import torch
    from paper_2606_23031_amd import dv
    from synth.configs import make_view, look_at_c2w
    cfg = actor_scene(seed=3, deg=2)
    scene, opts = cfg["scene"], cfg["opts"]
    eyes = [(5.0, 2.5, 2.0), (-5.0, 1.5, 1.5), (1.5, -5.0, 2.5),
            (-2.5, -4.0, -1.5), (4.0, 4.0, -2.5), (0.8, 4.5, 3.5)]
    views = [make_view(64, 48, 75.0, look_at_c2w(np.array(e), (0.0, 0.0, 0.0)), t=2.5)
             for e in eyes]
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_NORMAL | dv.DV_OUT_T
    copts = dv.make_opts(opts, mask)
    sc = dv.Scene(ctx, scene)
    na = len(scene["octrees"]) - 1
    gen = torch.Generator(device="cpu").manual_seed(7)
    grads = []
    for v in views:
        h, w = v["h"], v["w"]
        grads.append({k: t.cuda() for k, t in dict(
            rgb=torch.randn(3, h, w, generator=gen),
            depth=0.3 * torch.randn(h, w, generator=gen),
            normal=torch.randn(3, h, w, generator=gen),
            T=torch.randn(h, w, generator=gen)).items()})

    def zeros():
        return [dict(corner=torch.zeros(len(o["corner_density"]), device="cuda"),
                     sh=torch.zeros(o["sh"].shape, device="cuda"))
                for o in scene["octrees"]]

    outs = dv.alloc_outputs(views, mask)
    st = dv.dv_render(ctx, sc, views, copts, outs, keep=True)
    info = dv.dv_fwd_state_info(st)
    padded = sum((len(o["level"]) + 63) // 64 * 64 for o in scene["octrees"])
    print(f"  {info['n_visible']} records, {padded} leaf threads")
    assert info["n_visible"] >= 1.5 * padded  # the leaf-major pass runs
    acc = zeros()
    pg = torch.zeros(len(views), na, 12, device="cuda")
    dv.dv_render_backward(ctx, sc, st, grads, acc, pg)
    torch.cuda.synchronize()
    dv.dv_fwd_state_release(st)
    ref = zeros()
    pref = torch.zeros(len(views), na, 12, device="cuda")
    for i, v in enumerate(views):
        o1 = dv.alloc_outputs([v], mask)
        s1 = dv.dv_render(ctx, sc, [v], copts, o1, keep=True)
        a1 = zeros()
        p1 = torch.zeros(1, na, 12, device="cuda")
        dv.dv_render_backward(ctx, sc, s1, [grads[i]], a1, p1)
        torch.cuda.synchronize()
        dv.dv_fwd_state_release(s1)
        for k in range(len(ref)):
            ref[k]["corner"] += a1[k]["corner"]
            ref[k]["sh"] += a1[k]["sh"]
        pref[i] = p1[0]
    for k in range(len(ref)):
        for key in ("corner", "sh"):
            x, y = acc[k][key], ref[k][key]
            scale = float(y.abs().max())
            err = float((x - y).abs().max())
            print(f"  octree {k} {key}: max|ref| {scale:.3e} max err {err:.2e}")
            assert scale > 0.0 and err <= 1e-5 * scale, (k, key)
    scale = float(pref.abs().max())
    assert scale > 0.0 and float((pg - pref).abs().max()) <= 1e-5 * scale
