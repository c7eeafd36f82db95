"""Tile-binning and depth-order contracts (reference definitions in FP64).

The paper inherits a tile rasterizer with per-tile depth-sorted voxel lists
(Sec. 2 and Sec. 3.4: Morton-ordered traversal) but states neither the
binning predicate nor the sort key.  These readings fix both so that tile
lists and orders can be compared exactly:

Binning.  Per (view, octree), a = R_c^T R_k and b = R_c^T (p_k - o) take
octree-frame points to the camera frame.  For a leaf, each corner
x = root_min + (ijk + m) h goes to X = a x + b (every sum taken left to
right, no fused multiply-add).  All Z <= 0: culled.  Any Z < 1e-3: the
leaf covers the whole window.  Otherwise u = cx + fx (X/Z),
v = cy + fy (Y/Z); pixel column px is covered iff px >= ceil(umin - 9/16)
and px <= floor(umax - 7/16) (pixel centre within 1/16 px of the box of
projected corners), both bounds clamped to the window before rounding;
rows likewise.  Tiles are 16x16 over the window.

Order.  The rank of a leaf is a BSP painter's order from the camera
position P (octree frame): at every ancestor depth d < l the child bit of
each axis is XOR-ed with [P >= that parent's splitting plane], the three
bits form digit z<<2 | y<<1 | x, and digits are packed from the most
significant end for max_level levels.  P is quantised to 2^-24 of the root
side (floor of the clamped value), so the comparisons are exact integer
tests.  Along any ray from P the flipped bits only go 0 -> 1, hence leaves
hit by the ray appear in increasing rank exactly in increasing entry
distance.
"""
import numpy as np

Z_EPS = 1e-3
QBITS = 24


def _mat_t_mul(Rc, Rk):
    """A[i][j] = sum_r Rc[r][i] Rk[r][j], summed r = 0, 1, 2 in order."""
    A = np.empty((3, 3))
    for i in range(3):
        for j in range(3):
            A[i, j] = (Rc[0, i] * Rk[0, j] + Rc[1, i] * Rk[1, j]) + Rc[2, i] * Rk[2, j]
    return A


def camera_transform(view, R, p):
    Rc = view["c2w"][:, :3]
    o = view["c2w"][:, 3]
    A = _mat_t_mul(Rc, R)
    q = (p[0] - o[0], p[1] - o[1], p[2] - o[2])
    b = np.array([(Rc[0, i] * q[0] + Rc[1, i] * q[1]) + Rc[2, i] * q[2]
                  for i in range(3)])
    return A, b


def camera_in_octree(view, R, p):
    o = view["c2w"][:, 3]
    q = (o[0] - p[0], o[1] - p[1], o[2] - p[2])
    return np.array([(R[0, j] * q[0] + R[1, j] * q[1]) + R[2, j] * q[2]
                     for j in range(3)])


def leaf_rects(o, view, R, p):
    """Per leaf: status (0 culled, 1 rect, 2 whole window) and the covered
    window-relative pixel bounds (x_lo, x_hi, y_lo, y_hi), inclusive;
    an empty rect has lo > hi."""
    A, b = camera_transform(view, R, p)
    lv = o["level"].astype(np.int64)
    h = np.ldexp(np.full(lv.shape, o["root_size"]), -lv)
    ijk = o["ijk"].astype(np.int64)
    n = lv.shape[0]
    Xs = np.empty((8, 3, n))
    for m in range(8):
        x = [o["root_min"][a] + (ijk[a] + ((m >> a) & 1)).astype(np.float64) * h
             for a in range(3)]
        for i in range(3):
            Xs[m, i] = ((A[i, 0] * x[0] + A[i, 1] * x[1]) + A[i, 2] * x[2]) + b[i]
    Z = Xs[:, 2]
    culled = np.all(Z <= 0.0, axis=0)
    full = (~culled) & np.any(Z < Z_EPS, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = view["cx"] + view["fx"] * (Xs[:, 0] / Z)
        v = view["cy"] + view["fy"] * (Xs[:, 1] / Z)
    x0, y0, w, hh = view["x0"], view["y0"], view["w"], view["h"]

    def bounds(lo_val, hi_val, org, size):
        lo = np.ceil(np.clip(lo_val - 0.5625, org - 1.0, org + size))
        hi = np.floor(np.clip(hi_val - 0.4375, org - 1.0, org + size))
        lo = np.maximum(lo, org) - org
        hi = np.minimum(hi, org + size - 1) - org
        return lo.astype(np.int64), hi.astype(np.int64)

    rect = ~(culled | full)
    umin = np.where(rect, u.min(0), 0.0)
    umax = np.where(rect, u.max(0), 0.0)
    vmin = np.where(rect, v.min(0), 0.0)
    vmax = np.where(rect, v.max(0), 0.0)
    xl, xh = bounds(umin, umax, x0, w)
    yl, yh = bounds(vmin, vmax, y0, hh)
    xl = np.where(full, 0, xl)
    xh = np.where(full, w - 1, xh)
    yl = np.where(full, 0, yl)
    yh = np.where(full, hh - 1, yh)
    status = np.where(culled, 0, np.where(full, 2, 1))
    xl = np.where(culled, 1, xl)
    xh = np.where(culled, 0, xh)
    return status, xl, xh, yl, yh


def quantised_camera(o, view, R, p):
    P = camera_in_octree(view, R, p)
    Q = np.empty(3, np.int64)
    for a in range(3):
        q = (P[a] - o["root_min"][a]) / o["root_size"]
        q = min(max(q, -1.0), 2.0)
        Q[a] = int(np.floor(np.ldexp(q, QBITS)))
    return Q


def leaf_ranks(o, view, R, p):
    """BSP rank of every leaf (uint64), max_level digits of 3 bits."""
    Q = quantised_camera(o, view, R, p)
    L = int(o["max_level"])
    lv = o["level"].astype(np.int64)
    ijk = o["ijk"].astype(np.int64)
    rank = np.zeros(lv.shape[0], np.int64)
    for d in range(L):
        act = d < lv
        sh_child = np.maximum(lv - d - 1, 0)
        sh_par = np.maximum(lv - d, 0)
        digit = np.zeros_like(lv)
        for a in range(3):
            parent = ijk[a] >> sh_par
            plane = (2 * parent + 1) << (QBITS - d - 1)
            flip = (Q[a] >= plane).astype(np.int64)
            bit = (ijk[a] >> sh_child) & 1
            digit |= (bit ^ flip) << a
        rank |= np.where(act, digit << (3 * (L - 1 - d)), 0)
    return rank.astype(np.uint64)


def expected_tile_lists(scene, view, poses):
    """Reference tile lists: dict (tile id) -> list of (octree, leaf) in
    (octree, rank) order.  ``poses`` as from geometry.octree_poses."""
    ntx = (view["w"] + 15) // 16
    lists = {}
    for k, o in enumerate(scene["octrees"]):
        active, R, p = poses[k]
        if not active:
            continue
        st, xl, xh, yl, yh = leaf_rects(o, view, R, p)
        rk = leaf_ranks(o, view, R, p)
        vis = np.nonzero((st > 0) & (xl <= xh) & (yl <= yh))[0]
        vis = vis[np.argsort(rk[vis], kind="stable")]
        for vv in vis:
            for ty in range(yl[vv] >> 4, (yh[vv] >> 4) + 1):
                for tx in range(xl[vv] >> 4, (xh[vv] >> 4) + 1):
                    lists.setdefault(ty * ntx + tx, []).append((k, int(vv)))
    return lists


def actor_tile_lists(scene, view, poses):
    """Reference per-tile actor lists (ascending actor octree index) from
    the binning of each active actor's box as a single box."""
    ntx = (view["w"] + 15) // 16
    lists = {}
    for k in range(1, len(scene["octrees"])):
        active, R, p = poses[k]
        if not active:
            continue
        o = scene["octrees"][k]
        bmin = o.get("box_min", o["root_min"])
        bmax = o.get("box_max", o["root_min"] + o["root_size"])
        st, xl, xh, yl, yh = box_rect(bmin, bmax, view, R, p)
        if st == 0 or xl > xh or yl > yh:
            continue
        for ty in range(yl >> 4, (yh >> 4) + 1):
            for tx in range(xl >> 4, (xh >> 4) + 1):
                lists.setdefault(ty * ntx + tx, []).append(k)
    return lists


def box_rect(bmin, bmax, view, R, p):
    """The binning rule above applied to one box given by min/max corners
    (corner m takes max on axis a iff bit a of m is set)."""
    A, b = camera_transform(view, R, p)
    Xs = np.empty((8, 3))
    for m in range(8):
        x = [bmax[a] if (m >> a) & 1 else bmin[a] for a in range(3)]
        for i in range(3):
            Xs[m, i] = ((A[i, 0] * x[0] + A[i, 1] * x[1]) + A[i, 2] * x[2]) + b[i]
    Z = Xs[:, 2]
    x0, y0, w, hh = view["x0"], view["y0"], view["w"], view["h"]
    if np.all(Z <= 0.0):
        return 0, 1, 0, 1, 0
    if np.any(Z < Z_EPS):
        return 2, 0, w - 1, 0, hh - 1
    u = view["cx"] + view["fx"] * (Xs[:, 0] / Z)
    v = view["cy"] + view["fy"] * (Xs[:, 1] / Z)

    def bounds(lo_val, hi_val, org, size):
        lo = np.ceil(np.clip(lo_val - 0.5625, org - 1.0, org + size))
        hi = np.floor(np.clip(hi_val - 0.4375, org - 1.0, org + size))
        return int(max(lo, org) - org), int(min(hi, org + size - 1) - org)

    xl, xh = bounds(u.min(), u.max(), x0, w)
    yl, yh = bounds(v.min(), v.max(), y0, hh)
    return 1, xl, xh, yl, yh
