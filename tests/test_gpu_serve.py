"""Serving loop through the C ABI: continuous batching gives the same
results as rendering each request alone (bitwise for the forward pass),
a tiny memory budget queues instead of failing, and a malformed request
fails only its own ticket."""
import threading
import time

import numpy as np
import pytest

from oracle import render as RD
from synth import make_view, look_at_c2w
from scenes import actor_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_23031_amd import dv
    ctx = dv.dv_ctx_create(0)
    cfg = actor_scene(seed=11, n_actors=2, deg=2)
    sc = dv.Scene(ctx, cfg["scene"])
    return dv, ctx, cfg, sc


def _requests(n, seed=0):
    rng = np.random.default_rng(seed)
    sizes = [(64, 48), (48, 32), (96, 64)]
    out = []
    for i in range(n):
        W, H = sizes[rng.integers(3)]
        a = rng.uniform(0, 2 * np.pi)
        eye = np.array([3.2 * np.cos(a), 3.2 * np.sin(a), rng.uniform(0.5, 1.5)])
        out.append(make_view(W, H, 60.0, look_at_c2w(eye, (0, 0, 0)),
                             t=float(rng.uniform(0, 10))))
    return out


def _poll(dv, srv, ticket, limit_s=60.0):
    """Wait for a ticket, at most limit_s seconds (a request that never
    completes fails the test instead of stalling it)."""
    r = dv.dv_serve_poll(srv, ticket, int(limit_s * 1e6))
    assert r[0] <= 0, f"ticket {ticket} still pending after {limit_s} s"
    return r


def _alloc(dv, v, mask):
    return dv.alloc_outputs([v], mask)[0]


def _serve(dv, ctx, sc, opts, views, batched, budget=8 << 30, stagger=0.0):
    import torch
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH
    srv = dv.dv_serve_create(ctx, sc, dv.make_opts(opts, mask), max_inflight=8,
                             mem_budget=budget, batched=batched, max_batch=4)
    outs = [_alloc(dv, v, mask) for v in views]
    torch.cuda.synchronize()
    tickets = []
    for v, o in zip(views, outs):
        tickets.append(dv.dv_serve_submit(srv, v, o))
        if stagger:
            time.sleep(stagger)
    res = [_poll(dv, srv, t) for t in tickets]
    dv.dv_serve_destroy(srv)
    return outs, res


def test_batched_results_equal_alone_bitwise(env):
    dv, ctx, cfg, sc = env
    views = _requests(24, seed=1)
    opts = cfg["opts"]
    mixed, res = _serve(dv, ctx, sc, opts, views, batched=True)
    assert all(r[0] == 0 for r in res)
    lat = sorted(r[3] - r[1] for r in res)
    print(f"  p50 {1e3 * lat[len(lat) // 2]:.2f} ms  p99 {1e3 * lat[-1]:.2f} ms")
    alone, res2 = _serve(dv, ctx, sc, opts, views, batched=False)
    assert all(r[0] == 0 for r in res2)
    for a, b in zip(mixed, alone):
        for k in ("rgb", "depth"):
            assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())
    # and one served frame against the oracle
    ref = RD.render_image(cfg["scene"], views[3], opts)
    assert np.abs(mixed[3]["rgb"].cpu().numpy() - ref["rgb"]).max() <= 1e-4


def test_tiny_memory_budget_queues(env):
    dv, ctx, cfg, sc = env
    views = _requests(10, seed=2)
    outs, res = _serve(dv, ctx, sc, cfg["opts"], views, batched=True, budget=1)
    assert all(r[0] == 0 for r in res)
    # with a budget of one byte, no two requests overlap in time
    spans = sorted((r[2], r[3]) for r in res)
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-6


def test_bad_request_fails_alone(env):
    import torch
    dv, ctx, cfg, sc = env
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH
    srv = dv.dv_serve_create(ctx, sc, dv.make_opts(cfg["opts"], mask),
                             batched=True, max_batch=4)
    views = _requests(5, seed=3)
    bad = dict(views[2])
    bad["c2w"] = bad["c2w"].copy()
    bad["c2w"][0, 3] = np.nan
    views[2] = bad
    outs = [_alloc(dv, v, mask) for v in views]
    tickets = [dv.dv_serve_submit(srv, v, o) for v, o in zip(views, outs)]
    res = [_poll(dv, srv, t) for t in tickets]
    assert res[2][0] == -1
    assert all(r[0] == 0 for i, r in enumerate(res) if i != 2)
    # a finished ticket is forgotten once its status was returned
    assert dv.dv_serve_poll(srv, tickets[0], 0)[0] == -7
    dv.dv_serve_destroy(srv)


def test_concurrent_submitters(env):
    dv, ctx, cfg, sc = env
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH
    srv = dv.dv_serve_create(ctx, sc, dv.make_opts(cfg["opts"], mask),
                             batched=True, max_batch=8)
    views = _requests(32, seed=4)
    outs = [_alloc(dv, v, mask) for v in views]
    tickets = [None] * len(views)

    def sub(idx):
        for i in idx:
            tickets[i] = dv.dv_serve_submit(srv, views[i], outs[i])
    th = [threading.Thread(target=sub, args=(range(k, 32, 4),)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    res = [_poll(dv, srv, t) for t in tickets]
    assert all(r[0] == 0 for r in res)
    dv.dv_serve_destroy(srv)


def test_serving_workload_scene_staggered_mix():
    """The serving workload: the 1M-leaf + 8-car driving scene resident,
    requests of mixed resolution (640x360, 960x540, 1920x1080), random
    timestamps and headings on the ego lane, submitted with Poisson
    arrivals so that requests join while others are on the GPU.  Every
    served frame equals the same view rendered alone by dv_render, bit for
    bit (the benchmark's launch options); sampled pixels of each resolution
    are within 1e-4 of the oracle (exact walk, eps_stop = 0)."""
    import torch
    from paper_2606_23031_amd import dv
    from synth import make_config
    import bench
    cfg = make_config(4)
    ctx = dv.dv_ctx_create(0)
    sc = dv.Scene(ctx, cfg["scene"])
    views = bench.serve_views(36, seed=14)
    sizes = {(v["w"], v["h"]) for v in views}
    assert len(sizes) == 3
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH
    rng = np.random.default_rng(15)
    gaps = rng.exponential(1.0 / 400.0, len(views))   # ~2.5 ms apart
    for eps in (cfg["opts"]["eps_stop"], 0.0):
        opts = dict(cfg["opts"], eps_stop=eps)
        srv = dv.dv_serve_create(ctx, sc, dv.make_opts(opts, mask), max_inflight=8,
                                 mem_budget=16 << 30, batched=True, max_batch=4)
        outs = [_alloc(dv, v, mask) for v in views]
        torch.cuda.synchronize()
        tickets = []
        for v, o, g in zip(views, outs, gaps):
            time.sleep(g)
            tickets.append(dv.dv_serve_submit(srv, v, o))
        res = [_poll(dv, srv, t) for t in tickets]
        dv.dv_serve_destroy(srv)
        assert all(r[0] == 0 for r in res)
        # requests overlapped: some were admitted before an earlier one was done
        admits = [r[2] for r in res]
        dones = [r[3] for r in res]
        overlap = sum(1 for i in range(1, len(res)) if admits[i] < dones[i - 1])
        print(f"  eps {eps}: {overlap} of {len(res) - 1} requests admitted while "
              f"the previous one was in flight")
        assert overlap > 0
        copts = dv.make_opts(opts, mask)
        for v, o in zip(views, outs):
            alone = dv.alloc_outputs([v], mask)
            dv.dv_render(ctx, sc, [v], copts, alone)
            torch.cuda.synchronize()
            for k in ("rgb", "depth"):
                assert torch.equal(alone[0][k], o[k]), (v["w"], k)
    # oracle on sampled pixels of one request per resolution (eps = 0 run)
    done = set()
    for v, o in zip(views, outs):
        key = (v["w"], v["h"])
        if key in done:
            continue
        done.add(key)
        pix = np.stack([rng.integers(0, v["w"], 6), rng.integers(0, v["h"], 6)], 1)
        ref = RD.render_pixels(cfg["scene"], v, dict(cfg["opts"], eps_stop=0.0), pix,
                               procs=RD.default_procs())
        gx, gy = pix[:, 0], pix[:, 1]
        rgb = o["rgb"].cpu().numpy().astype(np.float64)[:, gy, gx].T
        dep = o["depth"].cpu().numpy().astype(np.float64)[gy, gx]
        e_rgb = np.abs(rgb - ref[:, 0:3]).max()
        e_d = np.abs(dep - ref[:, 3])
        print(f"  {key}: rgb {e_rgb:.2e} depth {e_d.max():.2e}")
        assert e_rgb <= 1e-4
        assert np.all(e_d <= 1e-4 * (1.0 + np.abs(ref[:, 3])))


def test_persistent_drain_mode_is_refused(env):
    dv, ctx, cfg, sc = env
    mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH
    with pytest.raises(dv.DVError) as ei:
        dv.dv_serve_create(ctx, sc, dv.make_opts(cfg["opts"], mask), batched=2)
    assert "persistent-drain" in str(ei.value)
