"""FP64 reference of the D-SSIM term of the photometric energy (Sec. 3.4, eq. 8).

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's oracle leg; it
never imports the HIP package.

E_pho = (1 - lambda) |I - I_ref|_1 + lambda L_D-SSIM(I, I_ref), lambda = 0.2.  The paper does
not spell L_D-SSIM out (it cites an optimised implementation of the usual structural
similarity); the reading taken here is the standard one:

    L_D-SSIM = 1 - mean over channels and pixels of SSIM(p),
    SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),

with mu, s the Gaussian-weighted local means, variances and covariance over an 11 x 11
window (standard deviation 1.5, weights summing to 1), pixels outside the image counting as
0 (the window is not renormalised at the border), C1 = 0.01^2, C2 = 0.03^2, and
s_x^2 = E[x^2] - mu_x^2, s_xy = E[xy] - mu_x mu_y.

Everything is computed from its definition: each window sum is the explicit sum of the 121
shifted, weighted images, and the gradient is the chain rule written out term by term.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """size x size weights exp(-(dx^2 + dy^2) / (2 sigma^2)), normalised to sum 1."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(r ** 2) / (2.0 * sigma ** 2))
    g /= g.sum()
    return np.outer(g, g)


def window_sum(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """out(p) = sum_{d} w(d) img(p + d - c), zero outside the image (c = window centre)."""
    k = w.shape[0]
    c = (k - 1) // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * c, W + 2 * c))
    pad[c:c + H, c:c + W] = img
    out = np.zeros((H, W))
    for i in range(k):
        for j in range(k):
            out += w[i, j] * pad[i:i + H, j:j + W]
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray, w: np.ndarray):
    """Per-pixel SSIM of one channel and the local statistics it is made of."""
    mx, my = window_sum(x, w), window_sum(y, w)
    sxx = window_sum(x * x, w) - mx * mx
    syy = window_sum(y * y, w) - my * my
    sxy = window_sum(x * y, w) - mx * my
    n1, n2 = 2 * mx * my + C1, 2 * sxy + C2
    d1, d2 = mx * mx + my * my + C1, sxx + syy + C2
    s = (n1 * n2) / (d1 * d2)
    return s, mx, my, n1, n2, d1, d2


def dssim(color: np.ndarray, target: np.ndarray) -> float:
    """L_D-SSIM of a colour image [3, H, W] against its target."""
    w = gaussian_window()
    tot = 0.0
    for ch in range(color.shape[0]):
        s = ssim_terms(np.asarray(color[ch], np.float64), np.asarray(target[ch], np.float64), w)[0]
        tot += s.sum()
    return 1.0 - tot / color.size


def dssim_grad(color: np.ndarray, target: np.ndarray) -> np.ndarray:
    """d L_D-SSIM / d color, [3, H, W].

    With S(q) = n1 n2 / (d1 d2) at window centre q, the image value x(p) enters mu_x(q) with
    weight w(p - q), E[x^2](q) with 2 w x(p) and E[xy](q) with w y(p), so
        dS(q)/dx(p) = w(p - q) (A(q) + 2 B(q) x(p) + C(q) y(p)),
        B = dS/ds_xx = -S / d2,  C = dS/ds_xy = 2 n1 / (d1 d2),
        A = dS/dmu_x - 2 mu_x B - mu_y C,  dS/dmu_x = 2 mu_y n2 / (d1 d2) - 2 mu_x S / d1,
    and dL/dx(p) = -(1/N) sum_q dS(q)/dx(p) (N = all channels and pixels).  The window is
    symmetric, so the sum over q is the same window sum as in the forward pass."""
    w = gaussian_window()
    N = color.size
    out = np.zeros(color.shape)
    for ch in range(color.shape[0]):
        x = np.asarray(color[ch], np.float64)
        y = np.asarray(target[ch], np.float64)
        s, mx, my, n1, n2, d1, d2 = ssim_terms(x, y, w)
        B = -s / d2
        Cc = 2.0 * n1 / (d1 * d2)
        dmu = 2.0 * my * n2 / (d1 * d2) - 2.0 * mx * s / d1
        A = dmu - 2.0 * mx * B - my * Cc
        out[ch] = -(window_sum(A, w) + 2.0 * x * window_sum(B, w) + y * window_sum(Cc, w)) / N
    return out
