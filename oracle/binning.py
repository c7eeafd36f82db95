"""Tile-binning and depth-order contracts (reference definitions in FP64).

The paper inherits a tile rasterizer with per-tile depth-sorted voxel lists
(Sec. 2 and Sec. 3.4: Morton-ordered traversal) but states neither the
binning predicate nor the sort key.  These readings fix both so that tile
lists and orders can be compared exactly:

Binning.  Per (view, octree), a = R_c^T R_k and b = R_c^T (p_k - o) take
octree-frame points to the camera frame.  For a leaf, each corner
x = root_min + (ijk + m) h goes to X = a x + b (every sum taken left to
right, no fused multiply-add).  All Z <= 0: culled.  If every Z >= e
(e = 1e-3) the corners are projected, u = cx + fx (X/Z),
v = cy + fy (Y/Z).  Otherwise the box straddles the plane Z = e: if the
axis-aligned (camera-frame) bound of its corners comes closer to the
camera than r_near (twice e times the largest |(x, y, 1)| of a window
pixel-centre direction) it covers the whole window; else the projected
points are the corners with Z >= e plus, on each of the 12 edges whose
ends lie on both sides of the plane, the crossing point
X_i = X_m + t (X_m' - X_m), t = (e - Z_m) / (Z_m' - Z_m), projected as
u = cx + fx (X_i / e).  (A ray that meets the box only where Z < e does so
within r_near / 2 of the camera, so the rule stays conservative.)  Pixel
column px is covered iff px >= ceil(umin - 9/16) and
px <= floor(umax - 7/16) (pixel centre within 1/16 px of the box of
projected points), both bounds clamped to the window before rounding;
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


def near_radius2(view):
    """r_near^2 = (2 e)^2 max over window corner pixel centres of
    (1 + x^2 + y^2), x = (px + 1/2 - cx) / fx, y likewise."""
    m2 = 0.0
    for px in (view["x0"], view["x0"] + view["w"] - 1):
        for py in (view["y0"], view["y0"] + view["h"] - 1):
            x = (px + 0.5 - view["cx"]) / view["fx"]
            y = (py + 0.5 - view["cy"]) / view["fy"]
            m2 = max(m2, (1.0 + x * x) + y * y)
    return (2.0 * Z_EPS) * (2.0 * Z_EPS) * m2


def _rects_from_corners(Xs, view):
    """Xs [8,3,n] camera-frame corners -> (status, xl, xh, yl, yh)."""
    Z = Xs[:, 2]
    n = Z.shape[1]
    culled = np.all(Z <= 0.0, axis=0)
    near = (~culled) & np.any(Z < Z_EPS, axis=0)
    lo = Xs.min(0)                                   # [3,n]
    hi = Xs.max(0)
    dd = np.maximum(np.maximum(lo, 0.0), -hi)
    dist2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
    full = near & (dist2 < near_radius2(view))
    with np.errstate(divide="ignore", invalid="ignore"):
        u = view["cx"] + view["fx"] * (Xs[:, 0] / Z)
        v = view["cy"] + view["fy"] * (Xs[:, 1] / Z)
    ok = Z >= Z_EPS                                  # [8,n]
    big = np.inf
    umin = np.where(ok, u, big).min(0)
    umax = np.where(ok, u, -big).max(0)
    vmin = np.where(ok, v, big).min(0)
    vmax = np.where(ok, v, -big).max(0)
    for bit in (1, 2, 4):
        for m in range(8):
            if m & bit:
                continue
            m2 = m | bit
            cross = (Z[m] < Z_EPS) != (Z[m2] < Z_EPS)
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (Z_EPS - Z[m]) / (Z[m2] - Z[m])
                xi = Xs[m, 0] + t * (Xs[m2, 0] - Xs[m, 0])
                yi = Xs[m, 1] + t * (Xs[m2, 1] - Xs[m, 1])
                ui = view["cx"] + view["fx"] * (xi / Z_EPS)
                vi = view["cy"] + view["fy"] * (yi / Z_EPS)
            umin = np.where(cross, np.minimum(umin, ui), umin)
            umax = np.where(cross, np.maximum(umax, ui), umax)
            vmin = np.where(cross, np.minimum(vmin, vi), vmin)
            vmax = np.where(cross, np.maximum(vmax, vi), vmax)
    x0, y0, w, hh = view["x0"], view["y0"], view["w"], view["h"]

    def bounds(lo_val, hi_val, org, size):
        lo_ = np.ceil(np.clip(lo_val - 0.5625, org - 1.0, org + size))
        hi_ = np.floor(np.clip(hi_val - 0.4375, org - 1.0, org + size))
        lo_ = np.maximum(lo_, org) - org
        hi_ = np.minimum(hi_, org + size - 1) - org
        return lo_.astype(np.int64), hi_.astype(np.int64)

    rect = ~(culled | full)
    xl, xh = bounds(np.where(rect, umin, 0.0), np.where(rect, umax, 0.0), x0, w)
    yl, yh = bounds(np.where(rect, vmin, 0.0), np.where(rect, vmax, 0.0), y0, hh)
    xl = np.where(full, 0, xl)
    xh = np.where(full, w - 1, xh)
    yl = np.where(full, 0, yl)
    yh = np.where(full, hh - 1, yh)
    status = np.where(culled, 0, np.where(full, 2, 1))
    xl = np.where(culled, 1, xl)
    xh = np.where(culled, 0, xh)
    return status, xl, xh, yl, yh


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
    return _rects_from_corners(Xs, view)


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


def expected_tile_lists(scene, view, poses, tiles=None):
    """Reference tile lists: dict (tile id) -> list of (octree, leaf) in
    (octree, rank) order.  ``poses`` as from geometry.octree_poses.  With
    ``tiles`` (iterable of tile ids) only those lists are built."""
    ntx = (view["w"] + 15) // 16
    if tiles is not None:
        return _tile_lists_subset(scene, view, poses, sorted(set(tiles)), ntx)
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


def _tile_lists_subset(scene, view, poses, tiles, ntx):
    lists = {t: [] for t in tiles}
    for k, o in enumerate(scene["octrees"]):
        active, R, p = poses[k]
        if not active:
            continue
        st, xl, xh, yl, yh = leaf_rects(o, view, R, p)
        vis = (st > 0) & (xl <= xh) & (yl <= yh)
        rk = leaf_ranks(o, view, R, p)
        for t in tiles:
            tx, ty = t % ntx, t // ntx
            sel = np.nonzero(vis & ((xl >> 4) <= tx) & ((xh >> 4) >= tx) &
                             ((yl >> 4) <= ty) & ((yh >> 4) >= ty))[0]
            sel = sel[np.argsort(rk[sel], kind="stable")]
            lists[t].extend((k, int(v)) for v in sel)
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
    Xs = np.empty((8, 3, 1))
    for m in range(8):
        x = [bmax[a] if (m >> a) & 1 else bmin[a] for a in range(3)]
        for i in range(3):
            Xs[m, i, 0] = ((A[i, 0] * x[0] + A[i, 1] * x[1]) + A[i, 2] * x[2]) + b[i]
    st, xl, xh, yl, yh = _rects_from_corners(Xs, view)
    return int(st[0]), int(xl[0]), int(xh[0]), int(yl[0]), int(yh[0])
