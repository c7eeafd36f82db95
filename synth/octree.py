"""Leaf-set construction for sparse-voxel octrees (structure only).

An octree is stored as its leaves only: each leaf has a level ``l`` and an
integer cell ``ijk`` in [0, 2^l)^3.  Corners are identified by their exact
integer position on the finest grid, so neighbouring leaves share corner
entries (one raw density per grid corner, as in the paper's initialisation
section where densities are assigned "for each grid corner").
"""
import numpy as np


def leaves_from_grid(level, ijk):
    """Return (level u8[N], ijk i32[3,N]) for cells given as an [N,3] array."""
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    lv = np.full(ijk.shape[0], level, dtype=np.uint8)
    return lv, np.ascontiguousarray(ijk.T.astype(np.int32))


def full_grid(level):
    n = 1 << level
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij"), -1).reshape(-1, 3)
    return leaves_from_grid(level, g)


def children(level, ijk):
    """Children of a set of cells: level+1, 8 per cell (m = mx+2my+4mz)."""
    ijk = np.asarray(ijk, dtype=np.int64).reshape(3, -1)
    out = []
    for m in range(8):
        off = np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1])[:, None]
        out.append(2 * ijk + off)
    ch = np.concatenate(out, axis=1)
    return np.full(ch.shape[1], level + 1, np.uint8), ch.astype(np.int32)


def random_subdivide(level, ijk, n_sub, max_level, rng):
    """Apply ``n_sub`` subdivisions, each of a leaf drawn uniformly among
    the leaves whose level is below ``max_level``.  Order of the returned
    leaves: the surviving originals, then children in creation order."""
    lv = list(np.asarray(level, dtype=np.int64))
    cells = [tuple(c) for c in np.asarray(ijk).T.tolist()]
    for _ in range(n_sub):
        cand = [i for i, l in enumerate(lv) if l < max_level]
        if not cand:
            break
        k = cand[int(rng.integers(len(cand)))]
        l, c = lv.pop(k), cells.pop(k)
        for m in range(8):
            lv.append(l + 1)
            cells.append((2 * c[0] + (m & 1), 2 * c[1] + ((m >> 1) & 1),
                          2 * c[2] + ((m >> 2) & 1)))
    return (np.array(lv, np.uint8),
            np.ascontiguousarray(np.array(cells, np.int64).T.astype(np.int32)))


def corner_positions(level, ijk, max_level):
    """Integer finest-grid positions of the 8 corners: int64[8,3,N]."""
    lv = np.asarray(level, np.int64)
    ijk = np.asarray(ijk, np.int64)
    sh = (max_level - lv)[None, :]
    out = np.empty((8, 3, lv.shape[0]), np.int64)
    for m in range(8):
        off = np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1])[:, None]
        out[m] = (ijk + off) << sh
    return out


def dedup_corners(level, ijk, max_level):
    """Shared-corner table: corner_idx i32[8,N] and the unique integer
    positions int64[Nc,3] (finest grid) in first-appearance-sorted order."""
    lv = np.asarray(level, np.int64)
    c = np.asarray(ijk, np.int64)
    n = lv.shape[0]
    sh = max_level - lv
    side = (1 << max_level) + 1
    # corner m of a leaf sits at ((ijk + (mx, my, mz)) << (max_level - l));
    # key = (x * side + y) * side + z, built per axis without the [8,3,N]
    # position array
    ax = [[(c[a] + o) << sh for o in (0, 1)] for a in range(3)]
    key = np.empty((8, n), np.int64)
    for m in range(8):
        np.multiply(ax[0][m & 1], side, out=key[m])
        key[m] += ax[1][(m >> 1) & 1]
        key[m] *= side
        key[m] += ax[2][(m >> 2) & 1]
    uniq, inv = np.unique(key.reshape(-1), return_inverse=True)
    cidx = inv.reshape(8, n).astype(np.int32)
    upos = np.stack([uniq // (side * side), (uniq // side) % side,
                     uniq % side], -1)
    return np.ascontiguousarray(cidx), upos


def _spread3(x):
    """Spread the low 21 bits of x (uint64 array) to every third bit."""
    x = np.asarray(x, np.uint64) & np.uint64(0x1FFFFF)
    for sh, m in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF),
                  (8, 0x100F00F00F00F00F), (4, 0x10C30C30C30C30C3),
                  (2, 0x1249249249249249)):
        x = (x | (x << np.uint64(sh))) & np.uint64(m)
    return x


def morton_codes(pos):
    """Morton (Z-order) codes of integer positions int64[n, 3]."""
    pos = np.asarray(pos, np.int64).reshape(-1, 3)
    return (_spread3(pos[:, 0]) | (_spread3(pos[:, 1]) << np.uint64(1)) |
            (_spread3(pos[:, 2]) << np.uint64(2)))


def morton_order_leaves(level, ijk, max_level):
    """Leaves sorted by the Morton code of their cell's low corner on the
    finest grid (leaves never overlap, so the codes are distinct): each run
    of consecutive leaves is a compact piece of space."""
    lv = np.asarray(level, np.int64)
    c = np.asarray(ijk, np.int64)
    pos = (c << (max_level - lv)[None, :]).T
    order = np.argsort(morton_codes(pos), kind="stable")
    return (np.ascontiguousarray(np.asarray(level)[order]),
            np.ascontiguousarray(np.asarray(ijk)[:, order]))


def morton_order_corners(cidx, upos):
    """Renumber a shared-corner table so corners are in Morton order of
    their finest-grid position: returns (corner_idx, positions)."""
    order = np.argsort(morton_codes(upos), kind="stable")
    rank = np.empty(len(order), np.int64)
    rank[order] = np.arange(len(order))
    return (np.ascontiguousarray(rank[cidx].astype(np.int32)),
            np.ascontiguousarray(np.asarray(upos)[order]))


def make_octree(root_min, root_size, max_level, level, ijk, corner_idx,
                corner_density, sh, box_min=None, box_max=None):
    level = np.ascontiguousarray(level, dtype=np.uint8)
    ijk = np.ascontiguousarray(ijk, dtype=np.int32)
    sh = np.ascontiguousarray(sh, dtype=np.float32)
    s = sh.shape[0]
    deg = int(round(np.sqrt(s))) - 1
    assert (deg + 1) ** 2 == s and sh.shape[1] == 3
    o = dict(root_min=np.asarray(root_min, np.float64).copy(),
             root_size=float(root_size), max_level=int(max_level),
             level=level, ijk=ijk,
             corner_idx=np.ascontiguousarray(corner_idx, dtype=np.int32),
             corner_density=np.ascontiguousarray(corner_density,
                                                 dtype=np.float32),
             sh_degree=deg, sh=sh)
    if box_min is not None:
        o["box_min"] = np.asarray(box_min, np.float64).copy()
        o["box_max"] = np.asarray(box_max, np.float64).copy()
    return o


def n_voxels(o):
    return int(o["level"].shape[0])
