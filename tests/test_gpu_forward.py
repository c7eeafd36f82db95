"""GPU forward parity against the FP64 oracle (through the C ABI).

Bar: tile lists and their order bit-exact; RGB, depth, normal and T within
1e-4 absolute (FP32 kernel vs FP64 oracle) on scenes whose depths are of
order metres.  Parity runs use eps_stop = 0 (no early stop) so both sides
composite the same pieces; a separate case bounds the effect of the stop.
"""
import numpy as np
import pytest

from oracle import render as RD
from oracle import binning as B
from oracle import geometry as G
from synth import make_config, make_view, look_at_c2w
from scenes import actor_scene, dense_scene, empty_octree, random_octree

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from gpu_helpers import gpu_ctx
    return gpu_ctx()


def _oracle(scene, view, opts):
    return RD.render_image(scene, view, opts, procs=RD.default_procs())


def _compare(gpu, ref, tol=TOL, keys=("rgb", "depth", "normal", "T")):
    for k in keys:
        if gpu.get(k) is None:
            continue
        err = float(np.abs(gpu[k] - ref[k]).max())
        print(f"  {k}: max abs err {err:.3e}")
        assert err <= tol, (k, err)


def _lists_equal(ctx, st, scene, view, view_idx=0):
    from paper_2606_23031_amd import dv
    info = dv.dv_fwd_state_info(st)
    ntiles = ((view["w"] + 15) // 16) * ((view["h"] + 15) // 16)
    ts, eo, el, ast, ao = dv.dv_fwd_state_export_lists(
        st, view_idx, ntiles, int(info["n_pairs"]) + 1, int(info["n_actor_pairs"]) + 1)
    poses = G.octree_poses(scene, view)
    ref = B.expected_tile_lists(scene, view, poses)
    for t in range(ntiles):
        got = list(zip(eo[ts[t]:ts[t + 1]].tolist(), el[ts[t]:ts[t + 1]].tolist()))
        assert got == ref.get(t, []), f"tile {t}: {len(got)} vs {len(ref.get(t, []))}"
    aref = B.actor_tile_lists(scene, view, poses)
    for t in range(ntiles):
        assert ao[ast[t]:ast[t + 1]].tolist() == aref.get(t, []), t
    return int(ts[-1])


def test_c1_forward_parity_and_lists(ctx):
    from gpu_helpers import render_gpu
    cfg = make_config(1)
    opts = dict(cfg["opts"], eps_stop=0.0)
    v = cfg["views"][0]
    res, st, sc = render_gpu(ctx, cfg["scene"], [v], opts, keep=True)
    ref = _oracle(cfg["scene"], v, opts)
    _compare(res[0], ref)
    n = _lists_equal(ctx, st, cfg["scene"], v)
    assert n > 1000


def test_c1_eps_stop_bounded(ctx):
    from gpu_helpers import render_gpu
    cfg = make_config(1)
    v = cfg["views"][0]
    eps = 0.05
    res, _, _ = render_gpu(ctx, cfg["scene"], [v], dict(cfg["opts"], eps_stop=eps))
    ref = _oracle(cfg["scene"], v, dict(cfg["opts"], eps_stop=0.0))
    assert np.abs(res[0]["rgb"] - ref["rgb"]).max() <= eps * 1.0 + TOL


@pytest.mark.parametrize("seed,overlap,K", [(0, False, 1), (1, False, 2),
                                            (2, True, 1), (3, True, 3)])
def test_actor_scene_parity(ctx, seed, overlap, K):
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=seed, n_actors=3 if overlap else 2, deg=2,
                      overlap=overlap, K=K)
    v = cfg["views"][0]
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"], keep=True)
    ref = _oracle(cfg["scene"], v, cfg["opts"])
    _compare(res[0], ref)
    _lists_equal(ctx, st, cfg["scene"], v)


@pytest.mark.parametrize("fov", [30.0, 14.0])
def test_actor_close_up_parity(ctx, fov):
    # the default actor views show leaves of about a pixel, so the actor
    # walks take every lane's own entries; close up (leaves several pixels
    # wide) the walk over the wave's entries runs too: at 30 degrees about
    # half of the (quadrant, batch) steps take each walk, at 14 all take
    # the wave's
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=12, n_actors=2, deg=2, fov=fov,
                      target=(-0.55, 0.33, 0.11))
    v = cfg["views"][0]
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"], keep=True)
    ref = _oracle(cfg["scene"], v, cfg["opts"])
    _compare(res[0], ref)
    _lists_equal(ctx, st, cfg["scene"], v)


@pytest.mark.parametrize("n_actors", [12, 44])
def test_crowded_tiles_parity(ctx, n_actors):
    # every tile holds all n_actors boxes, stacked and overlapping along the
    # rays: 12 takes the segment builder's wide register sweep, 44 (more
    # than it holds) the sweep through memory
    from gpu_helpers import render_gpu
    from scenes import crowd_scene
    cfg = crowd_scene(seed=3, n_actors=n_actors)
    v = cfg["views"][0]
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"], keep=True)
    ref = _oracle(cfg["scene"], v, cfg["opts"])
    _compare(res[0], ref)
    _lists_equal(ctx, st, cfg["scene"], v)


def test_wide_digit_pair_sort_lists_exact(ctx):
    # nine 1920x1080 views in one launch: 73 440 tiles, so the (leaf, tile)
    # pairs carry 17-bit tile keys, which the pair sort takes in two passes
    # of 9-bit digits; the per-tile lists must equal the oracle's binning
    # and depth order exactly
    from gpu_helpers import render_gpu
    from paper_2606_23031_amd import dv
    cfg = actor_scene(seed=21, n_actors=2, deg=1)
    views = []
    for i in range(9):
        a = 2.0 * np.pi * i / 9
        eye = np.array([3.2 * np.cos(a), 3.2 * np.sin(a), 1.0 + 0.1 * i])
        views.append(make_view(1920, 1080, 60.0, look_at_c2w(eye, (0.0, 0.0, 0.0)),
                               t=2.5))
    res, st, _ = render_gpu(ctx, cfg["scene"], views, cfg["opts"], keep=True)
    assert dv.dv_fwd_state_info(st)["tile_bits"] == 17
    for vi in (0, 4, 8):
        _lists_equal(ctx, st, cfg["scene"], views[vi], view_idx=vi)
    dv.dv_fwd_state_release(st)


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_chunked_tiles_parity(ctx, eps):
    # every tile's list (2.7k-4.2k entries) is split into chunks whose
    # partial states are merged; asset segments fall inside chunks and on
    # chunk boundaries.  With eps > 0 a chunk tests the stop on its own T,
    # which moves a colour by at most eps.
    from gpu_helpers import render_gpu
    from paper_2606_23031_amd import dv
    cfg = dense_scene(seed=0)
    v = cfg["views"][0]
    opts = dict(cfg["opts"], eps_stop=eps)
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], opts, keep=True)
    info = dv.dv_fwd_state_info(st)
    assert info["n_items"] > info["n_tiles"] and info["n_chunk_slots"] > 0
    ref = _oracle(cfg["scene"], v, dict(opts, eps_stop=0.0))
    if eps == 0.0:
        _compare(res[0], ref)
        _lists_equal(ctx, st, cfg["scene"], v)
    else:
        assert np.abs(res[0]["rgb"] - ref["rgb"]).max() <= eps + TOL
    dv.dv_fwd_state_release(st)


@pytest.mark.parametrize("overlap", [False, True])
def test_chunked_actor_lists_parity(ctx, overlap):
    # fully tiled assets: (tile, actor) lists of 2.4k-3.7k entries split into
    # chunks for rays with one segment of the actor; with overlapping boxes
    # some rays have two segments of one actor and walk the whole list
    from gpu_helpers import render_gpu
    from paper_2606_23031_amd import dv
    cfg = dense_scene(seed=2, actor_level=4, overlap=overlap)
    v = cfg["views"][0]
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"], keep=True)
    info = dv.dv_fwd_state_info(st)
    assert info["n_actor_items"] > info["n_actor_pairs"]
    ref = _oracle(cfg["scene"], v, cfg["opts"])
    _compare(res[0], ref)
    dv.dv_fwd_state_release(st)


def test_empty_scene_returns_background(ctx):
    from gpu_helpers import render_gpu
    sc = dict(octrees=[empty_octree()], tracks=[None])
    v = make_view(40, 24, 50.0, look_at_c2w((3, 0.2, 0.1), (0, 0, 0)))
    opts = dict(K=1, eps_stop=1e-4, tau_near=0.0, bg=(0.2, 0.3, 0.4), explin_c=1.1)
    res, _, _ = render_gpu(ctx, sc, [v], opts)
    assert np.all(res[0]["rgb"] == np.float32([0.2, 0.3, 0.4]).astype(np.float64)[:, None, None])
    assert np.all(res[0]["T"] == 1.0) and np.all(res[0]["depth"] == 0.0)


def test_window_crop_ragged_tiles_and_near_plane(ctx):
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=5, n_actors=2, deg=1)
    v = dict(cfg["views"][0])
    v.update(x0=7, y0=5, w=37, h=29)            # ragged 16x16 tiles
    opts = dict(cfg["opts"], tau_near=2.6)
    res, st, _ = render_gpu(ctx, cfg["scene"], [v], opts, keep=True)
    ref = _oracle(cfg["scene"], v, opts)
    _compare(res[0], ref)
    _lists_equal(ctx, st, cfg["scene"], v)


def test_camera_inside_octree(ctx):
    from gpu_helpers import render_gpu
    rng = np.random.default_rng(4)
    o = random_octree(rng, (-1, -1, -1), 2.0, 2, 40, 5, 1, g_mean=-0.5)
    sc = dict(octrees=[o], tracks=[None])
    v = make_view(48, 40, 90.0, look_at_c2w((0.13, -0.21, 0.07), (1, 0.4, 0.2)))
    opts = dict(K=2, eps_stop=0.0, tau_near=0.0, bg=(0.0, 0.0, 0.0), explin_c=1.1)
    res, st, _ = render_gpu(ctx, sc, [v], opts, keep=True)
    ref = _oracle(sc, v, opts)
    _compare(res[0], ref)
    _lists_equal(ctx, st, sc, v)


def test_multi_view_batch_equals_single(ctx):
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=6, n_actors=2, deg=2)
    v0 = cfg["views"][0]
    v1 = make_view(40, 30, 70.0, look_at_c2w((-2.5, 2.0, 1.0), (0, 0, 0)), t=4.0)
    both, _, _ = render_gpu(ctx, cfg["scene"], [v0, v1], cfg["opts"])
    a, _, _ = render_gpu(ctx, cfg["scene"], [v0], cfg["opts"])
    b, _, _ = render_gpu(ctx, cfg["scene"], [v1], cfg["opts"])
    for k in ("rgb", "depth", "normal", "T"):
        assert np.array_equal(both[0][k], a[0][k])
        assert np.array_equal(both[1][k], b[0][k])
    ref = _oracle(cfg["scene"], v1, cfg["opts"])
    _compare(b[0], ref)


def test_forward_deterministic(ctx):
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=7, n_actors=2, deg=3)
    v = cfg["views"][0]
    a, _, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"])
    b, _, _ = render_gpu(ctx, cfg["scene"], [v], cfg["opts"])
    for k in ("rgb", "depth", "normal", "T"):
        assert np.array_equal(a[0][k], b[0][k])


def test_two_streams_share_the_pool(ctx):
    """Renders alternating between two streams with no synchronisation in
    between: buffers freed by a call on one stream are reused by the other
    only after that call's stamp event, so every result equals the
    default-stream render bit for bit."""
    import torch
    from paper_2606_23031_amd import dv
    from gpu_helpers import render_gpu
    cfg = actor_scene(seed=7, n_actors=2, deg=3)
    v = cfg["views"][0]
    ref, _, sc = render_gpu(ctx, cfg["scene"], [v], cfg["opts"])
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_NORMAL | dv.DV_OUT_T
    copts = dv.make_opts(cfg["opts"], mask)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results = []
    for i in range(8):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            outs = dv.alloc_outputs([v], mask)
            dv.dv_render(ctx, sc, [v], copts, outs, stream=s)
        results.append(outs[0])
    torch.cuda.synchronize()
    for i, o in enumerate(results):
        for k in ("rgb", "depth", "normal", "T"):
            got = o[k].cpu().numpy().astype(np.float64)
            assert np.array_equal(got, ref[0][k]), (i, k)
