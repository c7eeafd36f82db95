"""Feature accumulation render (Sec. 4.3, '3D Semantic Segmentation'): the
colour step of the volume rendering is replaced by an F-channel per-leaf
feature, composited with the same weights as the colour, over a zero
background; its adjoint with respect to the features is the fusion of a
per-pixel feature map into the leaves (sum over pixels of w_i G).

TEST INFRASTRUCTURE ONLY (FP64, brute force): only the test suite, the
smoke check and the benchmark's CPU-baseline leg may use it.  It shares no
code with the HIP path.

The renderer composites three channels at a time; ``group`` g selects
channels 3g .. 3g + 2 (missing channels count as 0).  Features are taken
as given: no clamp and no view dependence (reading: the per-voxel feature
replaces the clamped SH colour of the colour render).
"""
import numpy as np

from . import adjoint as AD
from . import geometry as G
from . import render as RD


def group_channels(feat, group):
    """Channels 3g..3g+2 of one octree's features [F, N] as [N, 3]."""
    F, N = feat.shape
    out = np.zeros((N, 3))
    for c in range(3):
        if 3 * group + c < F:
            out[:, c] = feat[3 * group + c]
    return out


def feature_context(scene, view, opts, feats, group, pose_override=None):
    """A ViewContext whose per-leaf colour is the features' channel group
    and whose background is zero (no sky)."""
    o = dict(opts, bg=(0.0, 0.0, 0.0))
    o.pop("sky", None)
    ctx = RD.ViewContext(scene, view, o, pose_override)
    ctx.view_independent = True
    for k, ent in enumerate(ctx.oct):
        col = group_channels(np.asarray(feats[k], np.float64), group)
        ent["col"] = col
        # no clamp: every channel is 'active' for the adjoint's mask
        ent["raw"] = np.ones_like(col)
    return ctx


def render_features(scene, view, opts, feats, pixels):
    """Feature image at listed pixels: [n, F] = sum_i w_i f_i, and T [n]."""
    F = np.asarray(feats[0]).shape[0]
    pixels = np.asarray(pixels).reshape(-1, 2)
    out = np.zeros((len(pixels), F))
    T = np.zeros(len(pixels))
    for g in range((F + 2) // 3):
        ctx = feature_context(scene, view, opts, feats, g)
        for i, (px, py) in enumerate(pixels):
            o, d = G.camera_ray(view, px, py)
            r, _, _ = RD.render_ray(ctx, o, d)
            nc = min(3, F - 3 * g)
            out[i, 3 * g:3 * g + nc] = r["C"][:nc]
            T[i] = r["T"]
    return out, T


def feature_adjoint(scene, view, opts, feats, pixels, grads, group,
                    pose_override=None):
    """Adjoint of one group's feature render at listed pixels with upstream
    gradients grads [n, 8] = (G_F (3 channels), G_D, G_N, G_T): per octree
    dL/dfeatures of the group's channels [3, N] (the fusion sum_i w_i G_F),
    and the corner and pose gradients of the same render."""
    ctx = feature_context(scene, view, opts, feats, group, pose_override)
    acc = AD.new_accumulators(ctx)
    for (px, py), gg in zip(np.asarray(pixels).reshape(-1, 2), grads):
        o, d = G.camera_ray(view, px, py)
        AD.ray_adjoint(ctx, o, d, gg[0:3], gg[3], gg[4:7], gg[7], acc)
    fin = AD.finalize(ctx, acc)
    return dict(feat=[dc.T.copy() for dc in acc["dcol"]],
                feat_abs=[dc.T.copy() for dc in acc["dcol_abs"]],
                corner=fin["corner"], corner_abs=fin["corner_abs"],
                dR=fin["dR"], dp=fin["dp"])
