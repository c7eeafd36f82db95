"""dv_render_noalloc: the allocation-free variant of dv_render, through the
C ABI.  Its outputs equal dv_render's bit for bit (same kernels), on two
calls in a row whose second input is smaller; it takes nothing from the
context's pool or from torch; a render that needs more than the static
workspace fails with DV_ERR_LIMIT."""
import numpy as np
import pytest

from scenes import actor_scene
from synth import make_config, make_view, look_at_c2w

pytestmark = pytest.mark.gpu


def _pair(dv, ctx, sc, views, opts, mask):
    import torch
    copts = dv.make_opts(opts, mask)
    ref = dv.alloc_outputs(views, mask)
    dv.dv_render(ctx, sc, views, copts, ref)
    torch.cuda.synchronize()
    got = dv.alloc_outputs(views, mask)
    for o in got:                       # stale values must be overwritten
        for t in o.values():
            if t is not None:
                t.fill_(-7.0)
    torch.cuda.synchronize()
    in_use0, cached0 = dv.dv_ctx_memory(ctx)
    alloc0 = torch.cuda.memory_allocated()
    dv.dv_render_noalloc(ctx, sc, views, copts, got)
    torch.cuda.synchronize()
    assert dv.dv_ctx_memory(ctx) == (in_use0, cached0)
    assert torch.cuda.memory_allocated() == alloc0
    return ref, got


def _equal(ref, got):
    for a, b in zip(ref, got):
        for k, t in a.items():
            if t is not None:
                assert np.array_equal(t.cpu().numpy(), b[k].cpu().numpy()), k


def test_noalloc_equals_render_two_calls_second_smaller():
    import torch
    from paper_2606_23031_amd import dv
    assert torch.cuda.is_available()
    ctx = dv.dv_ctx_create(0)
    assert dv.dv_noalloc_capacity() == 128 << 20
    cfg = actor_scene(seed=12, n_actors=2, deg=2)
    sc = dv.Scene(ctx, cfg["scene"])
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_NORMAL | dv.DV_OUT_T
    # first call: two views (one of them 128x96)
    v0 = cfg["views"][0]
    eye = np.array([-2.8, 2.0, 1.5])
    v1 = make_view(128, 96, 60.0, look_at_c2w(eye, (0.0, 0.0, 0.0)), t=3.0)
    ref, got = _pair(dv, ctx, sc, [v0, v1], cfg["opts"], mask)
    _equal(ref, got)
    # second call: a smaller input (a 40x24 window of one view)
    w = dict(v0, x0=9, y0=13, w=40, h=24)
    ref2, got2 = _pair(dv, ctx, sc, [w], dict(cfg["opts"], eps_stop=1e-4), mask)
    _equal(ref2, got2)
    # the first call's outputs are untouched by the second
    _equal(ref, got)
    sc.close()
    # the plain forward workload (static octree, 128x96)
    c1 = make_config(1)
    sc1 = dv.Scene(ctx, c1["scene"])
    ref3, got3 = _pair(dv, ctx, sc1, c1["views"], c1["opts"], mask)
    _equal(ref3, got3)
    sc1.close()
    dv.dv_ctx_destroy(ctx)


def test_noalloc_rejects_oversized_render():
    import torch
    from paper_2606_23031_amd import dv
    ctx = dv.dv_ctx_create(0)
    cfg = actor_scene(seed=13, n_actors=2, deg=1)
    sc = dv.Scene(ctx, cfg["scene"])
    eye = np.array([3.0, 1.5, 1.2])
    # eight 1920x1080 views: the per-pixel state alone is ~1 GiB
    views = [make_view(1920, 1080, 60.0, look_at_c2w(eye, (0.0, 0.0, 0.0)), t=2.5)
             for _ in range(8)]
    mask = dv.DV_OUT_RGB | dv.DV_OUT_T
    outs = dv.alloc_outputs(views, mask)
    with pytest.raises(dv.DVError) as ei:
        dv.dv_render_noalloc(ctx, sc, views, dv.make_opts(cfg["opts"], mask), outs)
    assert ei.value.status == -6
    assert "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    # the context still renders afterwards, with and without allocations
    v = cfg["views"][0]
    ref, got = _pair(dv, ctx, sc, [v], cfg["opts"], mask)
    _equal(ref, got)
    sc.close()
    dv.dv_ctx_destroy(ctx)
