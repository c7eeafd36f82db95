"""Real spherical harmonics of degree <= 3, written from their definition.

Sec. 3.1 stores view-dependent colour as SH coefficients.  Reading: the
real orthonormal basis built from complex Y_l^m (with Condon-Shortley phase)
as  Y_{l,m} = sqrt2 (-1)^m Re Y_l^m (m>0),  Y_l^0 (m=0),
sqrt2 (-1)^m Im Y_l^|m| (m<0);  coefficient index l^2 + l + m.  With this
sign choice Y_{1,-1}, Y_{1,0}, Y_{1,1} are positive multiples of y, z, x.
Colour: c = max(0, sum_lm Y_lm(w) k_lm + 1/2), w = unit(voxel centre -
camera) in the octree's frame.
"""
import math
import numpy as np


def _assoc_legendre(l, m, x):
    """P_l^m(x), m >= 0, with the Condon-Shortley phase (-1)^m."""
    pmm = np.ones_like(x)
    if m > 0:
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
        fact = 1.0
        for _ in range(m):
            pmm = -pmm * fact * s
            fact += 2.0
    if l == m:
        return pmm
    pm1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pm1
    pll = pm1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pm1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pm1 = pm1, pll
    return pll


def basis(dirs, degree):
    """Y [.., (degree+1)^2] at unit directions ``dirs`` [..,3]."""
    dirs = np.asarray(dirs, np.float64)
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    phi = np.arctan2(y, x)
    out = np.zeros(dirs.shape[:-1] + ((degree + 1) ** 2,))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            p = _assoc_legendre(l, am, z)
            if m == 0:
                val = norm * p
            elif m > 0:
                val = math.sqrt(2.0) * (-1) ** m * norm * p * np.cos(m * phi)
            else:
                val = math.sqrt(2.0) * (-1) ** am * norm * p * np.sin(am * phi)
            out[..., l * l + l + m] = val
    return out


def basis_grad(dirs, degree):
    """d Y / d w [.., S, 3] at unit w, for the unconstrained function
    Y(w/|w|) (used for the camera-position term of pose gradients).

    Analytic.  With P_l^m(z) = (-1)^m (1 - z^2)^(m/2) P_l^(m)(z), P_l^(m)
    the m-th derivative of the Legendre polynomial, and
    (1 - z^2)^(m/2) e^(i m phi) = (x + i y)^m on the unit sphere, the
    basis above equals on the sphere
        F = sqrt2 N Re((x + i y)^m) P_l^(m)(z)      (m > 0)
        F = N P_l(z)                                (m = 0)
        F = sqrt2 N Im((x + i y)^|m|) P_l^(|m|)(z)  (m < 0).
    The derivative of w -> w/|w| at unit w is the projection I - w w^T and
    F agrees with Y on the sphere, so dY/dw = (I - w w^T) grad F(w)."""
    dirs = np.asarray(dirs, np.float64)
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    u = x + 1j * y
    gF = np.zeros(dirs.shape[:-1] + ((degree + 1) ** 2, 3))
    for l in range(degree + 1):
        leg = np.polynomial.legendre.Legendre.basis(l)
        for m in range(-l, l + 1):
            k = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - k) / math.factorial(l + k))
            q = leg.deriv(k)(z) if k > 0 else leg(z)
            dq = leg.deriv(k + 1)(z)
            if m == 0:
                a, ax, ay = np.ones_like(x), np.zeros_like(x), np.zeros_like(x)
                c = norm
            else:
                uk, duk = u ** k, k * u ** (k - 1)
                c = math.sqrt(2.0) * norm
                if m > 0:
                    a, ax, ay = uk.real, duk.real, -duk.imag
                else:
                    a, ax, ay = uk.imag, duk.imag, duk.real
            i = l * l + l + m
            gF[..., i, 0] = c * ax * q
            gF[..., i, 1] = c * ay * q
            gF[..., i, 2] = c * a * dq
    # project out the radial part: (I - w w^T) grad F
    radial = np.einsum("...sa,...a->...s", gF, dirs)
    return gF - radial[..., None] * dirs[..., None, :]


def basis_polynomial_form(dirs, degree):
    """F of ``basis_grad`` evaluated at ``dirs`` (equals ``basis`` on the
    unit sphere; kept so the identity behind the gradient can be checked)."""
    dirs = np.asarray(dirs, np.float64)
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    u = x + 1j * y
    out = np.zeros(dirs.shape[:-1] + ((degree + 1) ** 2,))
    for l in range(degree + 1):
        leg = np.polynomial.legendre.Legendre.basis(l)
        for m in range(-l, l + 1):
            k = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - k) / math.factorial(l + k))
            q = leg.deriv(k)(z) if k > 0 else leg(z)
            if m == 0:
                v = norm * q
            elif m > 0:
                v = math.sqrt(2.0) * norm * (u ** k).real * q
            else:
                v = math.sqrt(2.0) * norm * (u ** k).imag * q
            out[..., l * l + l + m] = v
    return out


def colour(sh, dirs):
    """Clamped colour [..,3] from coefficients sh [S,3,..] (f32 -> f64)."""
    S = sh.shape[0]
    deg = int(round(math.sqrt(S))) - 1
    Y = basis(dirs, deg)                             # [N,S]
    raw = np.einsum("ns,scn->nc", Y, sh.astype(np.float64)) + 0.5
    return np.maximum(raw, 0.0), raw
