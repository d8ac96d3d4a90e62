"""Nonrigid registration of a reference image to a moving one by gradient
descent on the displacement field, with image-space gridding as the warp
(oracle; test infrastructure only).

The paper estimates the displacement field of each respiratory phase
relative to a reference self-iNAV with a demons registration (section
"Nonrigid Respiratory Motion Correction"); the warp model it then uses is
T_d (Eq. 5, 9), which is differentiable in d.  This module states the
gradient-based alternative: minimise

    E(d) = ||T_d m_ref - m_mov||^2 + mu sum_i sum_a ||D_a d_i||^2

over the field d (voxels, pull convention: T_d m_ref at r is m_ref at
r + d(r)), D_a the periodic forward difference along axis a,
(D_a f)[r] = f[r + e_a] - f[r].  Its gradient is

    dE/dd_i[r] = 2 Re(conj(T_d m_ref - m_mov)[r] d(T_d m_ref)[r]/dd_i[r])
                 + 2 mu (-Lap d_i)[r],

-Lap f = sum_a D_a^T D_a f = sum_a (2 f[r] - f[r + e_a] - f[r - e_a]), and the
iteration is plain gradient descent with a fixed step:
d_{k+1} = d_k - step grad E(d_k), k = 0 .. iters - 1.
"""
import numpy as np

from .warp import warp, warp_jacobian


def neg_laplacian(f: np.ndarray) -> np.ndarray:
    """sum_a (2 f - f[+e_a] - f[-e_a]) with periodic neighbours."""
    out = np.zeros_like(f)
    for a in range(f.ndim):
        out += 2.0 * f - np.roll(f, -1, axis=a) - np.roll(f, 1, axis=a)
    return out


def smoothness(d: np.ndarray) -> float:
    """sum_i sum_a ||D_a d_i||^2."""
    d = np.asarray(d, dtype=np.float64)
    return float(sum(np.sum((np.roll(d[i], -1, axis=a) - d[i]) ** 2)
                     for i in range(d.shape[0]) for a in range(d.ndim - 1)))


def energy(d, ref, mov, mu: float) -> float:
    r = warp(ref, d) - np.asarray(mov, dtype=np.complex128)
    return float(np.vdot(r, r).real + mu * smoothness(d))


def energy_grad(d, ref, mov, mu: float) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    r = warp(ref, d) - np.asarray(mov, dtype=np.complex128)
    J = warp_jacobian(ref, d)
    return 2.0 * np.real(np.conj(r)[None] * J) + 2.0 * mu * np.stack([neg_laplacian(d[i]) for i in range(d.shape[0])])


def gradient_descent(ref, mov, d0, mu: float, step: float, iters: int):
    """Returns (d_iters, [E(d_0), ..., E(d_iters)])."""
    d = np.asarray(d0, dtype=np.float64).copy()
    hist = [energy(d, ref, mov, mu)]
    for _ in range(iters):
        d = d - step * energy_grad(d, ref, mov, mu)
        hist.append(energy(d, ref, mov, mu))
    return d, hist
