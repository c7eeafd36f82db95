"""Structure edits of the octrees (Sec. 3.3 'Initialization'; Supp.
'Adaptive Optimization Schedule'), FP64 brute force.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may use it.  It shares no code with the HIP
path.

* Soft density prior: each grid corner gets Eq. 1 of its distance to the
  nearest LiDAR point (``prior.soft_prior`` of
  ``prior.nearest_distance_bruteforce``).
* Proximity subdivision (initialisation step 2): a leaf is split into its
  8 children when a LiDAR point lies within tau of its box.  Reading: the
  distance is the Euclidean distance from the point to the leaf's closed
  box (0 inside), and tau = ratio * h with h the leaf's side (the paper
  names a distance threshold without a value).  Rounds repeat until the
  finest leaves are smaller than the minimum size.
* Subdivide with corner remapping (training-time edits): a child corner at
  a new position gets the value of the parent's trilinear field there;
  corners at positions that already exist (the parent's own, or a finer
  neighbour's on a shared face) keep their value.  The field inside a split
  leaf is unchanged wherever no finer neighbour already holds a corner at a
  child's corner position (always, on a uniform grid).
* Prune: leaves are removed; corners no longer used are dropped.
* Refinement (initialisation step 2, all rounds): while the finest leaf is
  not yet below the minimum size, the leaves near a point (proximity rule
  above) that are above the maximum level are split; it stops early when a
  round flags none.
* Bookkeeping for the optimiser state: every new leaf names its source
  leaf (itself when kept, its parent when a child) and every new corner
  the old corner at its position (-1 for a new position).  A child takes
  its parent's SH coefficients (the colour does not change under a split,
  reading).

Canonical order, so lists can be compared exactly: leaves that stay, in
their order, then the children of the split leaves, parent by parent,
child m = mx + 2 my + 4 mz in order; corners sorted by their integer
position on the finest grid (i, then j, then k), as the generators do.
"""
import numpy as np

from . import prior as PR


def leaf_boxes(o):
    h = o["root_size"] / np.exp2(np.asarray(o["level"], np.float64))
    lo = np.asarray(o["root_min"], np.float64)[None, :] + \
        np.asarray(o["ijk"], np.float64).T * h[:, None]
    return lo, lo + h[:, None], h


def point_box_distance(points, lo, hi):
    """Distance from every point to the closed box [lo, hi] (0 inside):
    [n_points]."""
    q = np.maximum(np.maximum(lo[None, :] - points, 0.0), points - hi[None, :])
    return np.sqrt((q * q).sum(1))


def proximity_flags(o, points, ratio):
    """Leaves with a LiDAR point within ratio * h of their box."""
    lo, hi, h = leaf_boxes(o)
    pts = np.asarray(points, np.float64)
    out = np.zeros(len(h), bool)
    for v in range(len(h)):
        out[v] = point_box_distance(pts, lo[v], hi[v]).min() <= ratio * h[v]
    return out


def _corner_keys(level, ijk, max_level):
    """Integer finest-grid positions of the 8 corners of every leaf:
    [8, N, 3] (corner m = mx + 2 my + 4 mz)."""
    sh = (max_level - np.asarray(level, np.int64))[:, None]
    base = np.asarray(ijk, np.int64).T
    out = np.empty((8, base.shape[0], 3), np.int64)
    for m in range(8):
        off = np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1], np.int64)
        out[m] = (base + off[None, :]) << sh
    return out


def _trilinear(g8, u):
    """Trilinear interpolation of 8 corner values at local coordinates u."""
    val = 0.0
    for m in range(8):
        wgt = 1.0
        for a in range(3):
            wgt *= u[a] if (m >> a) & 1 else 1.0 - u[a]
        val += wgt * g8[m]
    return val


def subdivide(o, split):
    """Split the flagged leaves; returns a new octree dict (level, ijk,
    corner_idx, corner_density in canonical order; other fields copied)."""
    split = np.asarray(split, bool)
    L = int(o["max_level"])
    lv, ijk = np.asarray(o["level"], np.int64), np.asarray(o["ijk"], np.int64)
    if np.any(lv[split] >= L):
        raise ValueError("a split leaf is already at the maximum level")
    keep = np.nonzero(~split)[0]
    par = np.nonzero(split)[0]
    new_lv = [lv[keep]]
    new_ijk = [ijk[:, keep]]
    src = [keep]
    ch_lv, ch_ijk, ch_par, ch_m = [], [], [], []
    for p in par:
        for m in range(8):
            ch_lv.append(lv[p] + 1)
            ch_ijk.append([2 * ijk[0, p] + (m & 1), 2 * ijk[1, p] + ((m >> 1) & 1),
                           2 * ijk[2, p] + ((m >> 2) & 1)])
            ch_par.append(p)
            ch_m.append(m)
    if par.size:
        new_lv.append(np.array(ch_lv, np.int64))
        new_ijk.append(np.array(ch_ijk, np.int64).T)
        src.append(np.array(ch_par, np.int64))
    leaf_src = np.concatenate(src)
    level = np.concatenate(new_lv)
    cells = np.concatenate(new_ijk, axis=1)
    # corner table: old positions keep their value; new ones come from the
    # parent's trilinear field
    old_pos = _corner_keys(lv, ijk, L)
    old_val = np.asarray(o["corner_density"], np.float64)
    cidx = np.asarray(o["corner_idx"], np.int64)
    value, origin = {}, {}
    for m in range(8):
        for v in range(len(lv)):
            value[tuple(old_pos[m, v])] = old_val[cidx[m, v]]
            origin[tuple(old_pos[m, v])] = cidx[m, v]
    pos = _corner_keys(level, cells, L)
    for j in range(par.size * 8):
        v = len(keep) + j
        p, mc = ch_par[j], ch_m[j]
        g8 = np.array([old_val[cidx[m, p]] for m in range(8)])
        for m in range(8):
            key = tuple(pos[m, v])
            if key in value:
                continue
            # local coordinates of the child's corner m in the parent
            u = np.array([((mc >> a) & 1) + ((m >> a) & 1) for a in range(3)]) / 2.0
            value[key] = _trilinear(g8, u)
    return _finish(o, level, cells, pos, value, origin, leaf_src)


def prune(o, keep_mask):
    """Remove the leaves not in keep_mask; drop unused corners."""
    keep = np.nonzero(np.asarray(keep_mask, bool))[0]
    L = int(o["max_level"])
    lv, ijk = np.asarray(o["level"], np.int64), np.asarray(o["ijk"], np.int64)
    old_pos = _corner_keys(lv, ijk, L)
    old_val = np.asarray(o["corner_density"], np.float64)
    cidx = np.asarray(o["corner_idx"], np.int64)
    value, origin = {}, {}
    for m in range(8):
        for v in keep:
            value[tuple(old_pos[m, v])] = old_val[cidx[m, v]]
            origin[tuple(old_pos[m, v])] = cidx[m, v]
    level, cells = lv[keep], ijk[:, keep]
    return _finish(o, level, cells, _corner_keys(level, cells, L), value,
                   origin, keep)


def refine(o, points, ratio, min_size, max_rounds=32):
    """Proximity subdivision rounds until the finest leaf is smaller than
    min_size (or no leaf is flagged, or max_rounds).  The result is in
    canonical order even after no round; leaf_src and corner_src refer to
    the input octree.  Each round is one subdivision edit of the stored
    octree, whose corner densities are FP32 parameters: a round
    interpolates (in FP64) from the previous round's values as stored,
    i.e. rounded to float32."""
    # the input in canonical corner order (an all-keep prune)
    cur = prune(o, np.ones(len(o["level"]), bool))
    leaf_src = cur["leaf_src"]
    corner_src = cur["corner_src"]
    rounds = 0
    L = int(o["max_level"])
    while rounds < max_rounds:
        lv = np.asarray(cur["level"], np.int64)
        if lv.size == 0 or cur["root_size"] / 2.0 ** lv.max() < min_size:
            break
        flags = proximity_flags(cur, points, ratio) & (lv < L)
        if not flags.any():
            break
        nxt = subdivide(cur, flags)
        nxt["corner_density"] = np.asarray(nxt["corner_density"],
                                           np.float32).astype(np.float64)
        leaf_src = leaf_src[nxt["leaf_src"]]
        cs = nxt["corner_src"]
        corner_src = np.where(cs >= 0, corner_src[np.maximum(cs, 0)], -1)
        cur = nxt
        rounds += 1
    out = dict(cur)
    out["leaf_src"] = leaf_src
    out["corner_src"] = corner_src
    out["rounds"] = rounds
    return out


def _finish(o, level, cells, pos, value, origin, leaf_src):
    n = len(level)
    keys = sorted({tuple(pos[m, v]) for m in range(8) for v in range(n)})
    index = {k: i for i, k in enumerate(keys)}
    cidx = np.array([[index[tuple(pos[m, v])] for v in range(n)] for m in range(8)],
                    np.int64).reshape(8, n)
    out = dict(o)
    out["level"] = np.asarray(level, np.int64)
    out["ijk"] = np.asarray(cells, np.int64).reshape(3, n)
    out["corner_idx"] = cidx
    out["corner_density"] = np.array([value[k] for k in keys], np.float64)
    out["corner_pos"] = np.array(keys, np.int64).reshape(-1, 3)
    out["corner_src"] = np.array([origin.get(k, -1) for k in keys], np.int64)
    out["leaf_src"] = np.asarray(leaf_src, np.int64)
    if "sh" in o:
        out["sh"] = np.asarray(o["sh"])[:, :, np.asarray(leaf_src, np.int64)]
    return out


def field_at(o, x):
    """The octree's trilinear raw density at point x (brute-force leaf
    search; None outside every leaf)."""
    lo, hi, h = leaf_boxes(o)
    inside = np.all((x[None, :] >= lo) & (x[None, :] <= hi), axis=1)
    idx = np.nonzero(inside)[0]
    if idx.size == 0:
        return None
    v = idx[0]
    u = (x - lo[v]) / h[v]
    g8 = np.asarray(o["corner_density"], np.float64)[np.asarray(o["corner_idx"])[:, v]]
    return _trilinear(g8, u)


def corner_world_positions(o):
    """World position of every corner (finest-grid integer positions)."""
    L = int(o["max_level"])
    pos = o.get("corner_pos")
    if pos is None:
        lv, ijk = np.asarray(o["level"], np.int64), np.asarray(o["ijk"], np.int64)
        keys = _corner_keys(lv, ijk, L)
        cidx = np.asarray(o["corner_idx"], np.int64)
        pos = np.zeros((int(cidx.max()) + 1, 3), np.int64)
        for m in range(8):
            pos[cidx[m]] = keys[m]
    return np.asarray(o["root_min"], np.float64)[None, :] + \
        pos.astype(np.float64) * (o["root_size"] / 2.0 ** L)


def corner_prior(o, points, s, v_close=PR.V_CLOSE, v_far=PR.V_FAR):
    """Eq. 1 for every corner of the octree."""
    d = PR.nearest_distance_bruteforce(points, corner_world_positions(o))
    return PR.soft_prior(d, s, v_close, v_far)
