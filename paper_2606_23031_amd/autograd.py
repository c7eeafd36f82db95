"""torch.autograd binding of dv_render / dv_render_backward.

The renderer reads corner densities and SH coefficients through the raw
pointers of the Scene's own tensors, so those tensors are the leaves of the
graph: mark them ``requires_grad_(True)`` and update them in place (under
``torch.no_grad()``) after each step.  Actor poses (R row-major, then p per
view and actor) are an optional FP64 CPU tensor; the pose gradient comes back
in the same layout (dL/dR, dL/dp).  A sky environment map passed as
``opts['sky']`` (float32 CUDA tensor [3][H][W]) is a graph input too: when it
requires grad, its gradient dL/dsky is returned.

Nothing here computes: forward runs dv_render with a kept state, backward
runs dv_render_backward into fresh accumulators and releases the state."""
import numpy as np
import torch

from . import dv

_KEYS = ("rgb", "depth", "normal", "T")


class _State:
    """Owns a forward state; releases it once, also when the graph is freed
    without a backward pass."""

    def __init__(self, handle):
        self.handle = handle

    def release(self):
        if self.handle is not None:
            dv.dv_fwd_state_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(fctx, spec, poses, sky, *params):
        ctx, scene, views, opts, mask = spec
        opts = dict(opts, sky=sky)
        outs = dv.alloc_outputs(views, mask)
        po = None if poses is None else poses.detach().cpu().numpy()
        st = dv.dv_render(ctx, scene, views, dv.make_opts(opts, mask), outs,
                          pose_override=po, keep=True,
                          stream=torch.cuda.current_stream())
        fctx.state = _State(st)
        fctx.spec = spec
        fctx.sky_shape = None if sky is None else tuple(sky.shape)
        fctx.pose_meta = None if poses is None else (poses.dtype, poses.device,
                                                     poses.shape)
        flat = [o[k] for o in outs for k in _KEYS if o[k] is not None]
        return tuple(flat)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(fctx, *gouts):
        ctx, scene, views, opts, mask = fctx.spec
        if fctx.state.handle is None:
            raise RuntimeError("dv render: backward called twice on one forward")
        grads, i = [], 0
        for _ in views:
            g = {}
            for k in _KEYS:
                bit = {"rgb": dv.DV_OUT_RGB, "depth": dv.DV_OUT_DEPTH,
                       "normal": dv.DV_OUT_NORMAL, "T": dv.DV_OUT_T}[k]
                if mask & bit:
                    t = gouts[i]
                    g[k] = None if t is None else t.contiguous()
                    i += 1
            grads.append(g)
        need = fctx.needs_input_grad
        acc = []
        for k, o in enumerate(scene.octs):
            acc.append(dict(
                corner=torch.zeros_like(o["corner_density"]) if need[3 + 2 * k] else None,
                sh=torch.zeros_like(o["sh"]) if need[4 + 2 * k] else None))
        pg = None
        if fctx.pose_meta is not None and need[1] and scene.n_actors > 0:
            pg = torch.zeros(len(views), scene.n_actors, 12, device="cuda")
        sg = None
        if fctx.sky_shape is not None and need[2]:
            sg = torch.zeros(fctx.sky_shape, device="cuda")
        dv.dv_render_backward(ctx, scene, fctx.state.handle, grads, acc, pg,
                              stream=torch.cuda.current_stream(), sky_grad=sg)
        fctx.state.release()
        g_params = []
        for a in acc:
            g_params += [a["corner"], a["sh"]]
        g_pose = None
        if pg is not None:
            dt, dev, shape = fctx.pose_meta
            g_pose = pg.to(device=dev, dtype=dt).reshape(shape)
        return (None, g_pose, sg, *g_params)


def track_poses(scene, views):
    """Poses of every actor at each view's timestamp, from the scene's tracks
    (host evaluation of the library), as an FP64 [n_views][n_actors][12]
    tensor suitable for ``render(..., poses=...)``."""
    n_act = len(scene["octrees"]) - 1
    out = np.zeros((len(views), max(n_act, 0), 12))
    for i, v in enumerate(views):
        for k in range(n_act):
            act, R, p = dv.dv_track_pose(scene["tracks"][k + 1], v["t"])
            if not act:
                raise ValueError(f"actor {k + 1} is inactive at t={v['t']}; "
                                 "explicit poses make every actor active")
            out[i, k, :9] = R.ravel()
            out[i, k, 9:] = p
    return torch.from_numpy(out)


def render(ctx, scene, views, opts, mask=dv.DV_OUT_RGB | dv.DV_OUT_DEPTH | dv.DV_OUT_T,
           poses=None):
    """Differentiable render of ``views``: returns one dict per view with the
    requested outputs.  Gradients flow to the Scene's corner-density and SH
    tensors that require grad, to ``poses`` if given and requiring grad, and
    to the sky map ``opts['sky']`` if it requires grad."""
    params = []
    for o in scene.octs:
        params += [o["corner_density"], o["sh"]]
    opts = dict(opts)
    sky = opts.pop("sky", None)
    flat = _Render.apply((ctx, scene, list(views), opts, int(mask)), poses,
                         sky, *params)
    res, i = [], 0
    for _ in views:
        d = {}
        for k in _KEYS:
            bit = {"rgb": dv.DV_OUT_RGB, "depth": dv.DV_OUT_DEPTH,
                   "normal": dv.DV_OUT_NORMAL, "T": dv.DV_OUT_T}[k]
            if mask & bit:
                d[k] = flat[i]
                i += 1
        res.append(d)
    return res
