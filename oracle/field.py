"""Density field inside one leaf (Sec. 3.1 and Sec. 3.4).

Readings: the eight raw corner densities are interpolated trilinearly
*before* activation, and the exp-linear activation with knee c is
    explin_c(x) = x                for x > c,
                = c * exp(x/c - 1) otherwise  (continuous and C^1 at c).
Corner m = mx + 2 my + 4 mz sits at offset (mx, my, mz) in the leaf.
"""
import numpy as np

CORNER_OFFSETS = np.array([[m & 1, (m >> 1) & 1, (m >> 2) & 1]
                           for m in range(8)], np.float64)


def trilinear_weights(u):
    """W [..,8] at local coordinates u [..,3] in [0,1]^3."""
    u = np.asarray(u, np.float64)
    w = np.ones(u.shape[:-1] + (8,))
    for m in range(8):
        for a in range(3):
            if (m >> a) & 1:
                w[..., m] *= u[..., a]
            else:
                w[..., m] *= 1.0 - u[..., a]
    return w


def trilinear_weight_grads(u):
    """dW_m/du_a  [..,8,3]."""
    u = np.asarray(u, np.float64)
    g = np.ones(u.shape[:-1] + (8, 3))
    for m in range(8):
        for a in range(3):
            for b in range(3):
                bit = (m >> b) & 1
                if a == b:
                    g[..., m, a] *= 1.0 if bit else -1.0
                else:
                    g[..., m, a] *= u[..., b] if bit else 1.0 - u[..., b]
    return g


def explin(x, c):
    x = np.asarray(x, np.float64)
    return np.where(x > c, x, c * np.exp(np.minimum(x, c) / c - 1.0))


def explin_grad(x, c):
    x = np.asarray(x, np.float64)
    return np.where(x > c, 1.0, np.exp(np.minimum(x, c) / c - 1.0))


def centre_gradient(g8):
    """Gradient of the trilinear field w.r.t. u at the leaf centre, [..,3];
    g8 [..,8] corner values."""
    return np.einsum("...m,ma->...a", g8, trilinear_weight_grads(
        np.full(3, 0.5)))


def voxel_normal(g8):
    """Reading of App. A ('N aggregates voxel normals'): one constant normal
    per leaf, n = -grad g(centre) / |grad g(centre)| in the octree frame,
    zero where the gradient vanishes."""
    v = centre_gradient(g8)
    nrm = np.linalg.norm(v, axis=-1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        n = np.where(nrm > 0, -v / np.where(nrm > 0, nrm, 1.0), 0.0)
    return n
