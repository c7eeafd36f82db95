"""Training losses and the optimiser step (Supp. 'Optimization Details',
Training Losses; Sec. 3.5), FP64, with their gradients with respect to the
rendered planes.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may use it.  It shares no code with the HIP
path.

L = l_color L_color + l_depth L_depth + l_normal L_normal + l_sky L_sky:
* L_color = (1 - l_ssim) mean|C - C_gt| + l_ssim (1 - SSIM(C, C_gt)).
  Reading: the printed colour term is garbled; the text names an L1 pixel
  loss and an SSIM term, combined here with weight l_ssim on SSIM.  SSIM
  (Wang et al. 2004): 11 x 11 Gaussian window, sigma 1.5, C1 = 0.01^2,
  C2 = 0.03^2 (dynamic range 1), zero padding at the image border ("same"
  size), mean over pixels and channels.
* L_depth = mean over pixels with LiDAR depth (D_lidar > 0) of |D - D_lidar|.
* L_normal = mean over pixels with a pseudo normal of 1 - cos(N, N_pseudo);
  reading: cos = N . Np / (max(|N|, 1e-8) |Np|) (a rendered normal is 0
  where nothing was hit).
* L_sky = mean over sky-mask pixels of (T_final - 1)^2.
The weights are options (the paper gives none).

Adam (the optimiser the paper inherits from SVRaster's pipeline; reading):
m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import numpy as np
from scipy.signal import convolve2d

SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def gaussian_window(size=11, sigma=1.5):
    """Normalised 2D Gaussian window (outer product of the 1D one)."""
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _blur(img, w):
    return convolve2d(img, w, mode="same", boundary="fill", fillvalue=0.0)


def ssim_map(x, y, w):
    """Per-pixel SSIM of one channel and the blurred moments."""
    mx, my = _blur(x, w), _blur(y, w)
    exx, eyy, exy = _blur(x * x, w), _blur(y * y, w), _blur(x * y, w)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A1, A2 = 2 * mx * my + SSIM_C1, 2 * sxy + SSIM_C2
    B1, B2 = mx * mx + my * my + SSIM_C1, sxx + syy + SSIM_C2
    S = A1 * A2 / (B1 * B2)
    return S, dict(mx=mx, my=my, A1=A1, A2=A2, B1=B1, B2=B2)


def ssim(x, y, w=None):
    """Mean SSIM over pixels and channels of [C, H, W] images."""
    w = gaussian_window() if w is None else w
    return float(np.mean([ssim_map(x[c], y[c], w)[0] for c in range(x.shape[0])]))


def ssim_grad(x, y, w=None):
    """d mean-SSIM / d x, [C, H, W].  With m = w * x (blur), e_xx = w * x^2,
    e_xy = w * (x y): S depends on x through m_x, e_xx, e_xy, and the
    adjoint of the zero-padded blur is the blur itself (w is symmetric):
    dS/dx = w * G_m + 2 x (w * G_xx) + y (w * G_xy)."""
    w = gaussian_window() if w is None else w
    C = x.shape[0]
    n = float(x.size)
    out = np.zeros_like(x, dtype=np.float64)
    for c in range(C):
        S, q = ssim_map(x[c], y[c], w)
        mx, my, A1, A2, B1, B2 = q["mx"], q["my"], q["A1"], q["A2"], q["B1"], q["B2"]
        dm = 2 * my * (A2 - A1) / (B1 * B2) - 2 * mx * S * (1.0 / B1 - 1.0 / B2)
        dxx = -S / B2
        dxy = 2 * A1 / (B1 * B2)
        out[c] = (_blur(dm / n, w) + 2 * x[c] * _blur(dxx / n, w)
                  + y[c] * _blur(dxy / n, w))
    return out


def training_loss(out, tgt, lam):
    """Loss terms and gradients.  out: rgb [3,H,W], depth [H,W],
    normal [3,H,W], T [H,W]; tgt: rgb, depth (0 = no LiDAR return),
    normal (0 = none), sky (mask, 1 = sky); lam: color, ssim, depth,
    normal, sky.  Returns (terms dict, total, grads dict of the planes)."""
    C, Cg = out["rgb"].astype(np.float64), tgt["rgb"].astype(np.float64)
    D, Dl = out["depth"].astype(np.float64), tgt["depth"].astype(np.float64)
    N, Np = out["normal"].astype(np.float64), tgt["normal"].astype(np.float64)
    T, sky = out["T"].astype(np.float64), tgt["sky"].astype(np.float64)
    l_ssim = lam["ssim"]
    # colour
    l1 = np.abs(C - Cg).mean()
    s = ssim(C, Cg)
    L_color = (1 - l_ssim) * l1 + l_ssim * (1 - s)
    gC = lam["color"] * ((1 - l_ssim) * np.sign(C - Cg) / C.size
                         - l_ssim * ssim_grad(C, Cg))
    # sparse depth
    md = Dl > 0
    nd = max(int(md.sum()), 1)
    L_depth = np.abs(D - Dl)[md].sum() / nd
    gD = lam["depth"] * np.where(md, np.sign(D - Dl), 0.0) / nd
    # normals
    nN = np.linalg.norm(N, axis=0)
    nP = np.linalg.norm(Np, axis=0)
    mn = nP > 0
    nn = max(int(mn.sum()), 1)
    den = np.maximum(nN, 1e-8) * np.where(mn, nP, 1.0)
    cos = (N * Np).sum(0) / den
    L_normal = (1 - cos)[mn].sum() / nn
    big = nN > 1e-8
    dcos = np.where(big, (Np / np.where(mn, nP, 1.0) - cos * N / np.where(big, nN, 1.0))
                    / np.where(big, nN, 1.0),
                    Np / (1e-8 * np.where(mn, nP, 1.0)))
    gN = lam["normal"] * np.where(mn, -dcos, 0.0) / nn
    # sky transmittance
    ms = sky > 0
    ns = max(int(ms.sum()), 1)
    L_sky = ((T - 1) ** 2)[ms].sum() / ns
    gT = lam["sky"] * np.where(ms, 2 * (T - 1), 0.0) / ns
    terms = dict(color=L_color, l1=l1, ssim=s, depth=L_depth, normal=L_normal,
                 sky=L_sky)
    total = (lam["color"] * L_color + lam["depth"] * L_depth
             + lam["normal"] * L_normal + lam["sky"] * L_sky)
    return terms, total, dict(rgb=gC, depth=gD, normal=gN, T=gT)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1) on FP64 copies; returns
    (p, m, v)."""
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
