"""Conjugate gradients for the l2 form of the inverse problem (oracle; test
infrastructure only).

Eq. 11 poses min ||y - A x||^2 + lambda R(x) over the stacked nonrigid SENSE
operators.  With R(x) = ||x||^2 the minimiser solves the Hermitian positive
definite system (sum_p A_p^H A_p + lambda I) x = sum_p A_p^H y_p, solved
here with plain Hestenes-Stiefel conjugate gradients: a fixed number of
iterations, no early exit, no preconditioner, inner products
<a, b> = sum conj(a) b.
"""
import numpy as np


def cg(apply_normal, b: np.ndarray, iters: int, x0: np.ndarray | None = None):
    """Return (x_iters, [||r_0||, ..., ||r_iters||])."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    r = b - apply_normal(x) if x0 is not None else b.copy()
    p = r.copy()
    rho = np.vdot(r, r).real
    hist = [np.sqrt(rho)]
    for _ in range(iters):
        q = apply_normal(p)
        alpha = rho / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_new = np.vdot(r, r).real
        p = r + (rho_new / rho) * p
        rho = rho_new
        hist.append(np.sqrt(rho))
    return x, hist
