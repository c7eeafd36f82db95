"""Helpers for GPU tests: run the HIP renderer through the C ABI binding."""
import numpy as np


def gpu_ctx():
    from paper_2606_23031_amd import dv
    return dv.dv_ctx_create(0)


def render_gpu(ctx, scene_dict, views, opts, mask=None, keep=False,
               pose_override=None, dv_scene=None):
    import torch
    from paper_2606_23031_amd import dv
    if mask is None:
        mask = dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_NORMAL | dv.DV_OUT_T
    sc = dv_scene or dv.Scene(ctx, scene_dict)
    outs = dv.alloc_outputs(views, mask)
    st = dv.dv_render(ctx, sc, views, dv.make_opts(opts, mask), outs,
                      pose_override=pose_override, keep=keep)
    torch.cuda.synchronize()
    res = []
    for o in outs:
        res.append({k: (t.cpu().numpy().astype(np.float64) if t is not None else None)
                    for k, t in o.items()})
    return res, st, sc


def max_abs(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())
