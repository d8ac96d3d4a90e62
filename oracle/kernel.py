"""Kaiser-Bessel interpolation kernel c(u), its derivative, and its
continuous Fourier transform (oracle; test infrastructure only).

The paper uses an interpolation kernel c(x) in image space with transform
C(k) (notation table) and divides by the transform to undo the kernel's
weighting (deapodization, section "k-space Gridding"; Eq. 7-9).  It names
no kernel family, width or oversampling.  The reading used here: the
Kaiser-Bessel kernel of the gridding reference the paper adapts its notation
from (Beatty et al. 2005), width W = 4 on a 2x oversampled grid, with
beta = pi * sqrt((W/alpha)^2 (alpha - 1/2)^2 - 0.8).

Support is OPEN: c(u) = 0 for |u| >= W/2, so an integer coordinate has three
non-zero taps and the fourth tap gets weight exactly 0.
"""
import math

import numpy as np
from scipy.special import i0, i1

WIDTH = 4
ALPHA = 2


def kb_beta(width: int = WIDTH, alpha: float = ALPHA) -> float:
    return math.pi * math.sqrt((width / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


BETA = kb_beta()


def kb(u, width: int = WIDTH, beta: float = BETA) -> np.ndarray:
    """c(u) = I0(beta * sqrt(1 - (2u/W)^2)) for |u| < W/2, else 0."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    m = np.abs(u) < width / 2.0
    out[m] = i0(beta * np.sqrt(1.0 - (2.0 * u[m] / width) ** 2))
    return out


def kb_deriv(u, width: int = WIDTH, beta: float = BETA) -> np.ndarray:
    """dc/du.  With s = sqrt(1 - (2u/W)^2): dc/du = I1(beta s) * beta * ds/du
    and ds/du = -(4u/W^2)/s, so dc/du = -(4 beta u / W^2) I1(beta s)/s.
    As s -> 0, I1(beta s)/s -> beta/2."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    m = np.abs(u) < width / 2.0
    s = np.sqrt(1.0 - (2.0 * u[m] / width) ** 2)
    ratio = np.where(s > 1e-12, i1(beta * s) / np.where(s > 1e-12, s, 1.0), beta / 2.0)
    out[m] = -(4.0 * beta * u[m] / width ** 2) * ratio
    return out


def kb_ft(f, width: int = WIDTH, beta: float = BETA) -> np.ndarray:
    """Continuous Fourier transform of c:  C(f) = int c(u) e^{-2 pi i f u} du
    = W sinh(z)/z with z = sqrt(beta^2 - (pi W f)^2)  (sin(|z|)/|z| branch
    when the radicand is negative).  Real and even, so C* = C."""
    f = np.asarray(f, dtype=np.float64)
    z2 = beta ** 2 - (math.pi * width * f) ** 2
    out = np.empty_like(f)
    pos = z2 > 0
    neg = z2 < 0
    zero = ~(pos | neg)
    z = np.sqrt(z2[pos])
    out[pos] = width * np.sinh(z) / z
    zn = np.sqrt(-z2[neg])
    out[neg] = width * np.sin(zn) / zn
    out[zero] = width
    return out
