"""Hand-derived FP64 reverse pass of the forward in ``render``.

Sec. 3.4 says gradients flow through each voxel segment independently; the
paper keeps tracks fixed (Sec. 5) and names pose optimisation as future
work, so the pose gradient here goes beyond it.  With per-piece value
v_i = G_C.c_i + G_D (a_i+b_i)/2 + G_N.n_i and the scalar
L = G_C.(C + T C_sky) + G_D D + G_N.N + G_T T, the derivative of L with
respect to the optical depth of piece i is
    dL/dtau_i = T_{i+1} v_i - (L - sum_{j<=i} w_j v_j),
which needs no division by (1 - alpha).  Pose enters through the ray in
the actor frame (o_k = R^T (o - p), d_k = R^T d): sample positions, leaf
faces, box faces that end background or asset pieces, the SH direction
from the camera position o_k, and the rotation of normals.  Binning and
ordering are piecewise constant and carry no gradient.
"""
import numpy as np

from . import geometry as G
from . import field as F
from . import sh as SH
from . import render as RD
from . import sky as SKY

_GW_CENTRE = F.trilinear_weight_grads(np.full(3, 0.5))       # [8,3]


def new_accumulators(ctx):
    # corner_abs: sum of |per-piece contribution| per corner, the scale of
    # the summands behind each corner gradient (bookkeeping for error bars)
    # dR_abs / dp_abs: the same for the pose entries
    acc = dict(corner=[], corner_abs=[], dcol=[], dcol_abs=[], dnw=[], dR=[],
               dp=[], dR_abs=[], dp_abs=[])
    for k, o in enumerate(ctx.scene["octrees"]):
        acc["corner"].append(np.zeros(o["corner_density"].shape[0]))
        acc["corner_abs"].append(np.zeros(o["corner_density"].shape[0]))
        n = o["level"].shape[0]
        acc["dcol"].append(np.zeros((n, 3)))
        acc["dcol_abs"].append(np.zeros((n, 3)))
        acc["dnw"].append(np.zeros((n, 3)))
        acc["dR"].append(np.zeros((3, 3)))
        acc["dp"].append(np.zeros(3))
        acc["dR_abs"].append(np.zeros((3, 3)))
        acc["dp_abs"].append(np.zeros(3))
    # sky texture gradient (the map is sampled per ray, Eq. 2)
    acc["sky"] = None if ctx.sky is None else np.zeros_like(ctx.sky)
    return acc


def ray_adjoint(ctx, o, d, gC, gD, gN, gT, acc):
    res, pc, smp = RD.render_ray(ctx, o, d)
    if ctx.sky is not None:
        # dL/dC_sky = T_final G_C, spread over the four bilinear taps
        SKY.scatter_grad(acc["sky"], d, res["T"] * np.asarray(gC, np.float64))
    n = res["nproc"]
    if n == 0:
        return res
    K = ctx.K
    gC, gN = np.asarray(gC, np.float64), np.asarray(gN, np.float64)
    v = res["col"] @ gC + gD * res["mid"] + res["nw"] @ gN
    L = gC @ res["rgb"] + gD * res["depth"] + gN @ res["normal"] + gT * res["T"]
    w = res["w"]
    pref = np.cumsum(w * v)
    Tn = res["Tb"] * res["e"]
    dtau = Tn * v - (L - pref)
    ks, vs = pc["k"][:n], pc["v"][:n]
    sig = smp["sig"][:n]
    g = smp["g"][:n]
    W = smp["W"][:n]
    l = smp["l"][:n]
    dsig = F.explin_grad(g, ctx.c)                    # [n,K]
    dgq = dtau[:, None] * (l / K)[:, None] * dsig     # dL/dg_q
    frac = (np.arange(K) + 0.5) / K
    frames = pc["frames"]
    go = [np.zeros(3) for _ in ctx.oct]
    gd = [np.zeros(3) for _ in ctx.oct]
    go_abs = [np.zeros(3) for _ in ctx.oct]
    gd_abs = [np.zeros(3) for _ in ctx.oct]
    for i in range(n):
        k, vv = int(ks[i]), int(vs[i])
        ent = ctx.oct[k]
        oct_ = ctx.scene["octrees"][k]
        # corner densities through the samples
        dg8 = W[i].T @ dgq[i]                          # [8]
        np.add.at(acc["corner"][k], oct_["corner_idx"][:, vv], dg8)
        np.add.at(acc["corner_abs"][k], oct_["corner_idx"][:, vv], np.abs(dg8))
        acc["dcol"][k][vv] += w[i] * gC
        acc["dcol_abs"][k][vv] += np.abs(w[i] * gC)
        acc["dnw"][k][vv] += w[i] * gN
        # geometry: samples and piece ends
        gw = F.trilinear_weight_grads(smp["u"][i])     # [K,8,3]
        dgdu = np.einsum("m,kma->ka", ent["g8"][vv], gw)
        dtdx = (l[i] / K) * dsig[i][:, None] * dgdu / ent["h"][vv]  # [K,3]
        dk = frames[k][1]
        s_sig = sig[i].sum() / K
        dta = -s_sig + ((dtdx @ dk) * (1.0 - frac)).sum()
        dtb = s_sig + ((dtdx @ dk) * frac).sum()
        ga = dtau[i] * dta + 0.5 * w[i] * gD
        gb = dtau[i] * dtb + 0.5 * w[i] * gD
        if k >= 1:
            go[k] += dtau[i] * dtdx.sum(0)
            gd[k] += dtau[i] * (smp["tq"][i][:, None] * dtdx).sum(0)
            go_abs[k] += np.abs(dtau[i] * dtdx).sum(0)
            gd_abs[k] += np.abs(dtau[i] * smp["tq"][i][:, None] * dtdx).sum(0)
        for (src, t, gg) in ((pc["sa"][i], pc["a"][i], ga),
                             (pc["sb"][i], pc["b"][i], gb)):
            j, ax = int(src[0]), int(src[1])
            if j >= 1 and ax >= 0:
                dj = frames[j][1]
                go[j][ax] += gg * (-1.0 / dj[ax])
                gd[j][ax] += gg * (-t / dj[ax])
                go_abs[j][ax] += abs(gg / dj[ax])
                gd_abs[j][ax] += abs(gg * t / dj[ax])
    for k in range(1, len(ctx.oct)):
        if not go[k].any() and not gd[k].any():
            continue
        R, p = ctx.oct[k]["R"], ctx.oct[k]["p"]
        acc["dR"][k] += np.outer(o - p, go[k]) + np.outer(d, gd[k])
        acc["dp"][k] += -R @ go[k]
        acc["dR_abs"][k] += (np.outer(np.abs(o - p), go_abs[k])
                             + np.outer(np.abs(d), gd_abs[k]))
        acc["dp_abs"][k] += np.abs(R) @ go_abs[k]
    return res


def finalize(ctx, acc):
    """Per-leaf colour and normal gradients -> SH coefficients, corners
    (through normals) and poses (SH direction, normal rotation)."""
    out = dict(corner=[], corner_abs=[], sh=[], sh_abs=[], dR=[], dp=[],
               dR_abs=[], dp_abs=[], sky=acc.get("sky"))
    for k, o in enumerate(ctx.scene["octrees"]):
        ent = ctx.oct[k]
        dcol = acc["dcol"][k] * (ent["raw"] > 0)
        deg = o["sh_degree"]
        Y = SH.basis(ent["wdir"], deg)                  # [N,S]
        out["sh"].append(np.einsum("ns,nc->scn", Y, dcol))
        dcol_abs = acc["dcol_abs"][k] * (ent["raw"] > 0)
        out["sh_abs"].append(np.einsum("ns,nc->scn", np.abs(Y), dcol_abs))
        corner = acc["corner"][k].copy()
        corner_abs = acc["corner_abs"][k].copy()
        dR, dp = acc["dR"][k].copy(), acc["dp"][k].copy()
        dR_abs, dp_abs = acc["dR_abs"][k].copy(), acc["dp_abs"][k].copy()
        R, p = ent["R"], ent["p"]
        # normals: n_w = R n_loc, n_loc = -v/|v|, v = grad of trilinear
        dnw = acc["dnw"][k]
        nz = np.nonzero(np.abs(dnw).sum(1) > 0)[0]
        if nz.size:
            nl = ent["n_loc"][nz]
            if k >= 1:
                dR += np.einsum("na,nb->ab", dnw[nz], nl)
                dR_abs += np.einsum("na,nb->ab", np.abs(dnw[nz]), np.abs(nl))
            dnl = dnw[nz] @ R                           # R^T dnw
            vv = F.centre_gradient(ent["g8"][nz])
            nrm = np.linalg.norm(vv, axis=1)
            ok = nrm > 0
            proj = dnl - nl * (nl * dnl).sum(1, keepdims=True)
            dv = np.where(ok[:, None], -proj / np.where(ok, nrm, 1.0)[:, None], 0.0)
            dg8 = dv @ _GW_CENTRE.T                     # [n,8]
            np.add.at(corner, o["corner_idx"][:, nz].T.ravel(), dg8.ravel())
            np.add.at(corner_abs, o["corner_idx"][:, nz].T.ravel(),
                      np.abs(dg8).ravel())
        # the SH colour depends on the viewing direction (camera position in
        # the actor frame); a view-independent per-leaf value (the feature
        # render's) does not
        if k >= 1 and not getattr(ctx, "view_independent", False):
            cz = np.nonzero(np.abs(dcol).sum(1) > 0)[0]
            if cz.size:
                gY = SH.basis_grad(ent["wdir"][cz], deg)   # [n,S,3]
                shc = o["sh"][:, :, cz].astype(np.float64)  # [S,3,n]
                dw = np.einsum("nc,scn,nsa->na", dcol[cz], shc, gY)
                dP = -(dw / ent["r"][cz][:, None]).sum(0)
                dR += np.outer(ctx.cam - p, dP)
                dp += -R @ dP
                dP_abs = np.abs(dw / ent["r"][cz][:, None]).sum(0)
                dR_abs += np.outer(np.abs(ctx.cam - p), dP_abs)
                dp_abs += np.abs(R) @ dP_abs
        out["corner"].append(corner)
        out["corner_abs"].append(corner_abs)
        out["dR"].append(dR)
        out["dp"].append(dp)
        out["dR_abs"].append(dR_abs)
        out["dp_abs"].append(dp_abs)
    return out


def render_and_grad(scene, view, opts, grads, pixels, pose_override=None):
    """Forward + adjoint over listed pixels.  ``grads`` [n,8] holds
    (G_RGB, G_D, G_N, G_T) per pixel.  Returns (outputs [n,8], gradients)
    with gradients for corner densities, SH and actor (R, p)."""
    ctx = RD.ViewContext(scene, view, opts, pose_override)
    acc = new_accumulators(ctx)
    pixels = np.asarray(pixels).reshape(-1, 2)
    out = np.zeros((len(pixels), 8))
    for i, (px, py) in enumerate(pixels):
        o, d = G.camera_ray(view, px, py)
        gg = grads[i]
        r = ray_adjoint(ctx, o, d, gg[0:3], gg[3], gg[4:7], gg[7], acc)
        out[i, 0:3], out[i, 3], out[i, 4:7], out[i, 7] = (
            r["rgb"], r["depth"], r["normal"], r["T"])
    return out, finalize(ctx, acc)
