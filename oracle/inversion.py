"""Inverting a nonrigid transform in image space (Appendix 1; oracle; test
infrastructure only).

Given an image p and a displacement field d, q = T{p} (Eq. 12) with T the
forward image-space gridding T_d (Eq. 9).  Recovering p from q:

* naive: apply the negated field, T_{-d} q (Fig. 10a);
* iterative: min_p ||q - T p||^2 + lambda ||W p||_1 (Eq. 13) with wavelet-FISTA
  (``fista``; 400 iterations, lambda = 1e-6 in the paper), or its l2 form
  min_p ||q - T p||^2 + lambda ||p||^2, i.e. (T^H T + lambda I) p = T^H q,
  with conjugate gradients (``cg``).
"""
import numpy as np

from .warp import warp, warp_adjoint


def naive(q: np.ndarray, d: np.ndarray) -> np.ndarray:
    """T_{-d} q."""
    return warp(q, -np.asarray(d, dtype=np.float64))


def normal(p: np.ndarray, d: np.ndarray, lam: float) -> np.ndarray:
    """(T^H T + lambda I) p."""
    return warp_adjoint(warp(p, d), d) + lam * np.asarray(p, dtype=np.complex128)
