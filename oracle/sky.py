"""FP64 sky environment map (Sec. 3.1 sky modeling, Eq. 2). Test
infrastructure only: nothing on the product path imports it.

The sky is a 2D spherical texture: a ray's world direction is mapped to 2D
map coordinates and the texture is sampled bilinearly; the sampled colour
is the C_sky of the final composite C = C_voxels + T_final C_sky, and the
texture receives gradients by backpropagation. The paper does not fix the
mapping; this reading (shared with the kernels, written separately there)
is the equirectangular one in the world frame with z up:
    longitude phi = atan2(d_y, d_x) in (-pi, pi], colatitude
    theta = acos(d_z) in [0, pi],
    u = (phi + pi) / (2 pi) W - 1/2,  v = theta / pi H - 1/2
(texel (i, j) has its centre at u = i, v = j), bilinear between columns
floor(u), floor(u) + 1 taken modulo W (the map wraps in longitude) and rows
floor(v), floor(v) + 1 clamped to [0, H - 1] (no wrap over the poles).
The texture is [3][H][W].
"""
import numpy as np


def taps(d, W, H):
    """The four (row, column, weight) taps of direction d (any length > 0)."""
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    phi = np.arctan2(d[1], d[0])
    theta = np.arccos(np.clip(d[2], -1.0, 1.0))
    u = (phi + np.pi) / (2.0 * np.pi) * W - 0.5
    v = theta / np.pi * H - 0.5
    i0 = int(np.floor(u))
    j0 = int(np.floor(v))
    fu, fv = u - i0, v - j0
    cols = (i0 % W, (i0 + 1) % W)
    rows = (min(max(j0, 0), H - 1), min(max(j0 + 1, 0), H - 1))
    return [(rows[0], cols[0], (1.0 - fu) * (1.0 - fv)),
            (rows[0], cols[1], fu * (1.0 - fv)),
            (rows[1], cols[0], (1.0 - fu) * fv),
            (rows[1], cols[1], fu * fv)]


def sample(sky, d):
    """C_sky for direction d from the texture sky [3][H][W]."""
    sky = np.asarray(sky, np.float64)
    _, H, W = sky.shape
    c = np.zeros(3)
    for j, i, w in taps(d, W, H):
        c += w * sky[:, j, i]
    return c


def scatter_grad(grad, d, g):
    """Adjoint of sample: add g (dL/dC_sky, 3 channels) into grad [3][H][W]."""
    _, H, W = grad.shape
    for j, i, w in taps(d, W, H):
        grad[:, j, i] += w * np.asarray(g, np.float64)


def texel_direction(i, j, W, H):
    """Unit direction through the centre of texel (column i, row j)."""
    phi = (i + 0.5) / W * 2.0 * np.pi - np.pi
    theta = (j + 0.5) / H * np.pi
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                     np.cos(theta)])
