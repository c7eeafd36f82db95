"""Brute-force FP64 forward render (Sec. 3.4, Eq. 2, App. A / Alg. 1).

Per ray r(tau) = o + tau d:
1. each active actor i maps the ray to its local frame by (T_t^i)^-1 and
   intersects its box, giving [A_i, B_i) clipped at tau_near (Sec. 3.4);
2. ownership (reading for overlapping boxes, which the paper leaves open):
   tau belongs to the lowest-index actor whose box contains it, else to the
   background.  Without overlaps this is exactly Alg. 1's alternation of
   background and asset segments;
3. every leaf of every octree gives its chord [t0, t1] (in that octree's
   frame; rigid maps keep tau), clipped to the part its octree owns
   (App. A: only what lies inside the active interval is evaluated; a
   straddling leaf contributes its clipped pieces);
4. all pieces are sorted by entry distance and composited front to back
   with the running state (C, D, N, T), T starting at 1 (the paper's
   initial state reads 'D=1', taken as T=1);
5. per piece [a, b], l = b - a: K-point midpoint rule (reading of 'standard
   numerical integration'), tau_opt = (l/K) sum_q explin(g(x_q)),
   e = exp(-tau_opt), w = T (1 - e); C += w c, D += w (a+b)/2,
   N += w R n, T *= e; stop after a piece once T < eps_stop (Alg. 1's stop
   test, applied after every piece);
6. RGB = C + T * C_bg (Eq. 2 with a constant sky colour).
"""
import os
import numpy as np

from . import geometry as G
from . import field as F
from . import sh as SH
from . import sky as SKY

NO_SRC = (-1, -1)


class ViewContext:
    """Per-view, per-octree quantities that do not depend on the pixel:
    pose, camera position in the octree frame, leaf boxes, colour (SH at the
    leaf-centre direction) and world normals."""

    def __init__(self, scene, view, opts, pose_override=None):
        self.scene, self.view, self.opts = scene, view, opts
        self.K = int(opts.get("K", 1))
        self.eps = float(opts.get("eps_stop", 1e-4))
        self.tau_near = float(opts.get("tau_near", 0.0))
        self.c = float(opts.get("explin_c", 1.1))
        self.bg = np.asarray(opts.get("bg", (0.0, 0.0, 0.0)), np.float64)
        # sky environment map [3][H][W] (Sec. 3.1); None: the constant bg
        sky = opts.get("sky")
        self.sky = None if sky is None else np.asarray(sky, np.float64)
        self.cam = view["c2w"][:, 3].astype(np.float64)
        self.poses = G.octree_poses(scene, view, pose_override)
        self.oct = []
        for k, o in enumerate(scene["octrees"]):
            active, R, p = self.poses[k]
            vmin, h = G.voxel_boxes(o)
            P = R.T @ (self.cam - p)
            ctr = vmin + 0.5 * h[:, None]
            w = ctr - P[None, :]
            r = np.linalg.norm(w, axis=1)
            wdir = w / np.where(r > 0, r, 1.0)[:, None]
            col, raw = SH.colour(o["sh"], wdir)
            g8 = o["corner_density"].astype(np.float64)[o["corner_idx"]].T
            n_loc = F.voxel_normal(g8)
            ent = dict(active=active, R=R, p=p, P=P, vmin=vmin, h=h,
                       vmax=vmin + h[:, None], col=col, raw=raw, wdir=wdir,
                       r=r, g8=g8, n_loc=n_loc, n_w=n_loc @ R.T)
            if k > 0:
                ent["box"] = G.actor_box(o)
            self.oct.append(ent)


def subtract(s, e, ss, se, blockers):
    """[s, e) minus the union of blocker intervals.  Each interval carries
    the sources of its two ends (octree index, axis) for the adjoint."""
    out = []
    cur, csrc = s, ss
    for bs, be, bss, bse in sorted(blockers, key=lambda x: x[0]):
        if be <= cur:
            continue
        if bs >= e:
            break
        if bs > cur:
            out.append((cur, bs, csrc, bss))
        if be > cur:
            cur, csrc = be, bse
        if cur >= e:
            break
    if cur < e:
        out.append((cur, e, csrc, se))
    return out


def ray_frames(ctx, o, d):
    """Ray in every octree frame: list of (o_k, d_k)."""
    fr = []
    for ent in ctx.oct:
        R, p = ent["R"], ent["p"]
        fr.append((R.T @ (o - p), R.T @ d))
    return fr


def owned_intervals(ctx, frames):
    """Ownership of the ray parameter: dict octree -> list of intervals
    (s, e, src_s, src_e); src = (octree whose box face it is, axis)."""
    boxes = []
    for k in range(1, len(ctx.oct)):
        ent = ctx.oct[k]
        if not ent["active"]:
            continue
        ok, dk = frames[k]
        t0, t1, a0, a1 = G.slab(ok, dk, *ent["box"])
        s0 = (k, a0)
        if t0 < ctx.tau_near:
            t0, s0 = ctx.tau_near, NO_SRC
        if t1 > t0:
            boxes.append((k, t0, t1, s0, (k, a1)))
    own = {}
    for idx, (k, A, B, sA, sB) in enumerate(boxes):
        lower = [(b[1], b[2], b[3], b[4]) for b in boxes[:idx]]
        own[k] = subtract(A, B, sA, sB, lower)
    own[0] = subtract(ctx.tau_near, np.inf, NO_SRC, NO_SRC,
                      [(b[1], b[2], b[3], b[4]) for b in boxes])
    return own, boxes


def ray_pieces(ctx, o, d):
    """All positive-length pieces along the ray, sorted by entry distance.

    Returns a dict of arrays: octree k, leaf v, a, b, and the sources of a
    and b as (octree, axis) (axis -1: constant end)."""
    frames = ray_frames(ctx, o, d)
    own, _ = owned_intervals(ctx, frames)
    ks, vs, As, Bs, sa, sb = [], [], [], [], [], []
    for k, ivs in own.items():
        if not ivs:
            continue
        ent = ctx.oct[k]
        ok, dk = frames[k]
        t0, t1, ax0, ax1 = G.slab_many(ok, dk, ent["vmin"], ent["vmax"])
        near = t0 < ctx.tau_near
        t0 = np.where(near, ctx.tau_near, t0)
        hit = np.nonzero(t1 > t0)[0]
        if hit.size == 0:
            continue
        t0h, t1h = t0[hit], t1[hit]
        src0 = np.where(near[hit], -1, ax0[hit])
        for (s, e, ss, se) in ivs:
            a = np.maximum(t0h, s)
            b = np.minimum(t1h, e)
            keep = b > a
            if not keep.any():
                continue
            a_vox = t0h[keep] >= s
            b_vox = t1h[keep] <= e
            n = int(keep.sum())
            ks.append(np.full(n, k))
            vs.append(hit[keep])
            As.append(a[keep])
            Bs.append(b[keep])
            sa.append(np.stack([np.where(a_vox, np.where(src0[keep] >= 0, k, -1), ss[0]),
                                np.where(a_vox, src0[keep], ss[1])], 1))
            sb.append(np.stack([np.where(b_vox, k, se[0]),
                                np.where(b_vox, ax1[hit][keep], se[1])], 1))
    if not ks:
        z = np.zeros(0)
        return dict(k=z.astype(int), v=z.astype(int), a=z, b=z,
                    sa=np.zeros((0, 2), int), sb=np.zeros((0, 2), int),
                    frames=frames)
    k = np.concatenate(ks)
    order = np.argsort(np.concatenate(As), kind="stable")
    return dict(k=k[order], v=np.concatenate(vs)[order],
                a=np.concatenate(As)[order], b=np.concatenate(Bs)[order],
                sa=np.concatenate(sa)[order], sb=np.concatenate(sb)[order],
                frames=frames)


def piece_samples(ctx, pc):
    """Midpoint samples of every piece: tau_q [n,K], x_q [n,K,3] (octree
    frame), u_q [n,K,3], g_q [n,K] (raw), sigma_q [n,K], tau_opt [n]."""
    K = ctx.K
    n = pc["a"].shape[0]
    a, b = pc["a"], pc["b"]
    l = b - a
    frac = (np.arange(K) + 0.5) / K
    tq = a[:, None] + frac[None, :] * l[:, None]
    o_k = np.array([pc["frames"][k][0] for k in pc["k"]]).reshape(n, 3)
    d_k = np.array([pc["frames"][k][1] for k in pc["k"]]).reshape(n, 3)
    vmin = np.array([ctx.oct[k]["vmin"][v] for k, v in zip(pc["k"], pc["v"])]).reshape(n, 3)
    h = np.array([ctx.oct[k]["h"][v] for k, v in zip(pc["k"], pc["v"])])
    g8 = np.array([ctx.oct[k]["g8"][v] for k, v in zip(pc["k"], pc["v"])]).reshape(n, 8)
    x = o_k[:, None, :] + tq[:, :, None] * d_k[:, None, :]
    u = np.clip((x - vmin[:, None, :]) / h[:, None, None], 0.0, 1.0)
    W = F.trilinear_weights(u)                        # [n,K,8]
    g = np.einsum("nkm,nm->nk", W, g8)
    sig = F.explin(g, ctx.c)
    tau = (l / K) * sig.sum(axis=1)
    return dict(l=l, tq=tq, x=x, u=u, W=W, g=g, sig=sig, tau=tau, o_k=o_k,
                d_k=d_k, vmin=vmin, h=h, g8=g8)


def composite(ctx, pc, smp, c_sky=None):
    """Front-to-back compositing of sorted pieces with the stop test, then
    the sky behind them (Eq. 2): c_sky, else the constant bg."""
    c_sky = ctx.bg if c_sky is None else c_sky
    n = pc["a"].shape[0]
    e = np.exp(-smp["tau"])
    Tb = np.ones(n)
    T = 1.0
    nproc = n
    for i in range(n):
        Tb[i] = T
        T = T * e[i]
        if T < ctx.eps:
            nproc = i + 1
            break
    sl = slice(0, nproc)
    w = Tb[sl] * (1.0 - e[sl])
    col = np.array([ctx.oct[k]["col"][v] for k, v in zip(pc["k"][sl], pc["v"][sl])]).reshape(-1, 3)
    nw = np.array([ctx.oct[k]["n_w"][v] for k, v in zip(pc["k"][sl], pc["v"][sl])]).reshape(-1, 3)
    mid = 0.5 * (pc["a"][sl] + pc["b"][sl])
    C = (w[:, None] * col).sum(0)
    D = float((w * mid).sum())
    N = (w[:, None] * nw).sum(0)
    return dict(rgb=C + T * c_sky, C=C, depth=D, normal=N, T=T,
                nproc=nproc, e=e[sl], Tb=Tb[sl], w=w, col=col, nw=nw,
                mid=mid)


def render_ray(ctx, o, d):
    pc = ray_pieces(ctx, o, d)
    smp = piece_samples(ctx, pc)
    c_sky = None if ctx.sky is None else SKY.sample(ctx.sky, d)
    return composite(ctx, pc, smp, c_sky), pc, smp


def window_pixels(view):
    ys, xs = np.mgrid[0:view["h"], 0:view["w"]]
    return np.stack([xs.ravel() + view["x0"], ys.ravel() + view["y0"]], 1)


def _render_list(ctx, pix):
    out = np.zeros((len(pix), 8))
    for i, (px, py) in enumerate(pix):
        o, d = G.camera_ray(ctx.view, px, py)
        r, _, _ = render_ray(ctx, o, d)
        out[i, 0:3] = r["rgb"]
        out[i, 3] = r["depth"]
        out[i, 4:7] = r["normal"]
        out[i, 7] = r["T"]
    return out


_POOL_CTX = None


def _pool_work(pix):
    return _render_list(_POOL_CTX, pix)


def render_pixels(scene, view, opts, pixels, pose_override=None, procs=1,
                  ctx=None):
    """Render listed image pixels [n,2]; returns [n,8] = rgb, depth,
    normal, T.  ``procs`` > 1 splits the rays over forked processes."""
    global _POOL_CTX
    ctx = ctx or ViewContext(scene, view, opts, pose_override)
    pixels = np.asarray(pixels).reshape(-1, 2)
    if procs <= 1 or len(pixels) < 2 * procs:
        return _render_list(ctx, pixels)
    import multiprocessing as mp
    _POOL_CTX = ctx
    chunks = np.array_split(pixels, procs * 4)
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_pool_work, chunks)
    _POOL_CTX = None
    return np.concatenate(parts, 0)


def render_image(scene, view, opts, pose_override=None, procs=1):
    """Render the view's window: dict rgb [3,h,w], depth [h,w],
    normal [3,h,w], T [h,w]."""
    pix = window_pixels(view)
    out = render_pixels(scene, view, opts, pix, pose_override, procs)
    h, w = view["h"], view["w"]
    return dict(rgb=out[:, 0:3].T.reshape(3, h, w),
                depth=out[:, 3].reshape(h, w),
                normal=out[:, 4:7].T.reshape(3, h, w),
                T=out[:, 7].reshape(h, w))


def default_procs():
    return max(1, min(16, os.cpu_count() or 1))
