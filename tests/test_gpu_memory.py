"""Device memory through the allocator callback of dv_ctx_create: with
torch as the provider, the library's pool takes its blocks from torch's
caching allocator, so torch's allocated bytes rise while a scene and a
render hold memory and fall back when the pool hands its idle blocks back;
without it (hipMalloc) torch sees nothing."""
import numpy as np
import pytest

from scenes import actor_scene

pytestmark = pytest.mark.gpu


def _buffers(dv, cfg):
    """Caller-side tensors of one render + backward (torch's own memory)."""
    import torch
    view = cfg["views"][0]
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_T
    outs = dv.alloc_outputs([view], mask)
    g = [dict(rgb=torch.ones_like(outs[0]["rgb"]))]
    acc = [dict(corner=torch.zeros(len(o["corner_density"]), device="cuda"),
                sh=torch.zeros(o["sh"].shape, device="cuda"))
           for o in cfg["scene"]["octrees"]]
    torch.cuda.synchronize()
    return mask, outs, g, acc


def _render_once(dv, ctx, sc, cfg, bufs):
    """Render + backward; returns torch's allocated bytes while the forward
    state is still held."""
    import torch
    mask, outs, g, acc = bufs
    st = dv.dv_render(ctx, sc, cfg["views"], dv.make_opts(cfg["opts"], mask), outs,
                      keep=True)
    dv.dv_render_backward(ctx, sc, st, g, acc)
    torch.cuda.synchronize()
    during = torch.cuda.memory_allocated()
    dv.dv_fwd_state_release(st)
    torch.cuda.synchronize()
    return during


def test_torch_provider_memory_rises_and_falls():
    import torch
    from paper_2606_23031_amd import dv
    cfg = actor_scene(seed=8, n_actors=2, deg=1)
    ctx = dv.dv_ctx_create(0, torch_memory=True)
    torch.cuda.synchronize()
    base0 = torch.cuda.memory_allocated()
    sc = dv.Scene(ctx, cfg["scene"])            # inputs: torch tensors
    bufs = _buffers(dv, cfg)
    torch.cuda.synchronize()
    in_use0, _ = dv.dv_ctx_memory(ctx)
    assert in_use0 > 0                          # the scene's packed tables
    base = torch.cuda.memory_allocated()
    during = _render_once(dv, ctx, sc, cfg, bufs)
    in_use, cached = dv.dv_ctx_memory(ctx)
    print(f"  base {base} during {during}; pool in use {in_use}, cached {cached}")
    # records, pairs, sort buffers and the forward state were torch memory
    assert during > base
    assert cached > 0
    dv.dv_ctx_trim(ctx)
    torch.cuda.synchronize()
    assert dv.dv_ctx_memory(ctx) == (in_use0, 0)
    assert torch.cuda.memory_allocated() == base
    # destroying the scene hands its tables back too
    sc.close()
    dv.dv_ctx_trim(ctx)
    torch.cuda.synchronize()
    assert dv.dv_ctx_memory(ctx) == (0, 0)
    assert torch.cuda.memory_allocated() == base - in_use0
    del sc, bufs
    dv.dv_ctx_destroy(ctx)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= base0


def test_hipmalloc_provider_is_invisible_to_torch():
    import torch
    from paper_2606_23031_amd import dv
    cfg = actor_scene(seed=9, n_actors=2, deg=1)
    ctx = dv.dv_ctx_create(0, torch_memory=False)
    sc = dv.Scene(ctx, cfg["scene"])
    bufs = _buffers(dv, cfg)
    base = torch.cuda.memory_allocated()
    during = _render_once(dv, ctx, sc, cfg, bufs)
    assert during == base
    in_use, cached = dv.dv_ctx_memory(ctx)
    assert in_use > 0 and cached > 0
    # the same images whichever provider holds the scratch
    ctx2 = dv.dv_ctx_create(0, torch_memory=True)
    sc2 = dv.Scene(ctx2, cfg["scene"])
    bufs2 = _buffers(dv, cfg)
    _render_once(dv, ctx2, sc2, cfg, bufs2)
    for k in ("rgb", "depth", "T"):
        assert np.array_equal(bufs[1][0][k].cpu().numpy(),
                              bufs2[1][0][k].cpu().numpy())
    sc.close()
    sc2.close()
    dv.dv_ctx_destroy(ctx)
    dv.dv_ctx_destroy(ctx2)
