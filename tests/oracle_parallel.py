"""Test-side helpers that run the FP64 oracle over many rays in forked
worker processes (plumbing only; the arithmetic is the oracle's)."""
import multiprocessing as mp

import numpy as np

from oracle import adjoint as AD
from oracle import geometry as G
from oracle import render as RD

_CTX = None


def _grad_chunk(args):
    pix, grads = args
    ctx = _CTX
    acc = AD.new_accumulators(ctx)
    for (px, py), g in zip(pix, grads):
        o, d = G.camera_ray(ctx.view, px, py)
        AD.ray_adjoint(ctx, o, d, g[0:3], g[3], g[4:7], g[7], acc)
    out = {}
    for key in ("corner", "corner_abs", "dcol", "dcol_abs", "dnw"):
        lst = []
        for arr in acc[key]:
            if arr.size == 0:
                lst.append((np.zeros(0, np.int64), arr))
                continue
            nz = np.nonzero(arr.reshape(arr.shape[0], -1).any(1))[0]
            lst.append((nz, arr[nz]))
        out[key] = lst
    for key in ("dR", "dp", "dR_abs", "dp_abs"):
        out[key] = acc[key]
    out["sky"] = acc["sky"]
    return out


def render_and_grad_parallel(scene, view, opts, grads, pixels, procs):
    """Same result as oracle.adjoint.render_and_grad (gradients only),
    computed over ray chunks in forked processes."""
    global _CTX
    ctx = RD.ViewContext(scene, view, opts)
    _CTX = ctx
    chunks = np.array_split(np.arange(len(pixels)), max(1, procs * 2))
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_grad_chunk, [(pixels[c], grads[c]) for c in chunks])
    acc = AD.new_accumulators(ctx)
    for part in parts:
        for key in ("corner", "corner_abs", "dcol", "dcol_abs", "dnw"):
            for k, (nz, vals) in enumerate(part[key]):
                acc[key][k][nz] += vals
        for key in ("dR", "dp", "dR_abs", "dp_abs"):
            for k in range(len(acc[key])):
                acc[key][k] += part[key][k]
        if acc["sky"] is not None:
            acc["sky"] += part["sky"]
    _CTX = None
    return AD.finalize(ctx, acc)
