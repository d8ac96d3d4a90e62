"""Wavelet-FISTA for the l1-regularised problems of the paper, and the power
iteration that gives its step size (oracle; test infrastructure only).

Eq. 11 (nonrigid motion-corrected reconstruction) and Eq. 13 (inverting a
nonrigid transform, Appendix 1) both read

    min_x  F(x) = ||y - A x||_2^2 + lambda ||W x||_1

with A the stacked nonrigid SENSE operator (Eq. 11) or the warp T (Eq. 13)
and W the orthonormal wavelet transform of ``wavelet``.  The paper solves them
with wavelet-FISTA (Beck and Teboulle 2009; 400 iterations, lambda = 1e-6 in
Appendix 1).  The steps, in the notation of that method with constant step
size 1/L, L >= the Lipschitz constant 2 lambda_max(A^H A) of grad f,
f(x) = ||y - A x||^2:

    x_k     = p_L(z_k),  p_L(v) = W^H S_{lambda/L}(W (v - grad f(v) / L)),
              grad f(v) = 2 (A^H A v - A^H y)
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
    z_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1})

from z_1 = x_0, t_1 = 1.  S_tau is the soft threshold of a complex value,
S_tau(c) = c max(0, 1 - tau/|c|), applied to every detail coefficient; the
approximation coefficients (the coarsest low-pass band) are not penalised
(a reading: the paper does not say).  The prox is exact because W is
orthonormal.
"""
import numpy as np

from . import wavelet


def soft_threshold(c: np.ndarray, tau: float) -> np.ndarray:
    """c max(0, 1 - tau/|c|) elementwise (0 where c = 0)."""
    c = np.asarray(c, dtype=np.complex128)
    mag = np.abs(c)
    scale = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    return c * scale


def prox(v: np.ndarray, tau: float, levels: int) -> np.ndarray:
    """argmin_x tau ||W x||_1 (details only) + 1/2 ||x - v||^2 = W^H S_tau(W v)."""
    w = wavelet.forward(v, levels)
    keep = wavelet.approximation_mask(v.shape, levels)
    w = np.where(keep, w, soft_threshold(w, tau))
    return wavelet.inverse(w, levels)


def objective(Ax_minus_y_sq: float, x: np.ndarray, lam: float, levels: int) -> float:
    """F(x) given ||A x - y||^2."""
    w = wavelet.forward(x, levels)
    keep = wavelet.approximation_mask(x.shape, levels)
    return float(Ax_minus_y_sq + lam * np.sum(np.abs(w[~keep])))


def fista(apply_AhA, b: np.ndarray, lam: float, L: float, iters: int, levels: int,
          x0: np.ndarray | None = None) -> np.ndarray:
    """FISTA with constant step 1/L for F(x) = ||y - A x||^2 + lam ||W x||_1
    given b = A^H y and apply_AhA(v) = A^H A v; returns x_iters."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    z = x.copy()
    t = 1.0
    for _ in range(iters):
        grad = 2.0 * (apply_AhA(z) - b)
        x_new = prox(z - grad / L, lam / L, levels)
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
    return x


def power_iteration(apply_N, x0: np.ndarray, iters: int):
    """Largest eigenvalue of the Hermitian positive semidefinite N by the
    power method from x0: v_0 = x0/||x0||, w_j = N v_{j-1}, v_j = w_j/||w_j||;
    returns (||w_iters||, v_iters).  ||N v|| over unit v converges to the
    largest eigenvalue from below."""
    v = np.asarray(x0, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply_N(v)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam, v
