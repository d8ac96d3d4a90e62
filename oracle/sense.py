"""Nonrigid SENSE operators and the stacked multi-state model (oracle; test
infrastructure only).

Section "Nonrigid SENSE Operators" (Eq. 10; Figs. 2-3): the operator for
state p is the forward image-space gridding T_p, then multiplication by each
coil sensitivity S_c, then inverse k-space gridding G_p on that state's
share of the trajectory:

  A_p x      = [ G_p (S_c . T_p x) ]_c
  A_p^H y_p  = T_p^H ( sum_c conj(S_c) . G_p^H y_{p,c} )

Stacking the states gives the data model of Eq. 10 and the inverse problem of
Eq. 11.  With the l2 (Tikhonov) regulariser in place of the paper's
l1-wavelet term, the normal equations are (sum_p A_p^H A_p + lambda I) x =
sum_p A_p^H y_p.
"""
import numpy as np

from .kspace import nufft_adjoint, nufft_forward
from .warp import warp, warp_adjoint, warp_jacobian


def coil_forward(m: np.ndarray, S: np.ndarray, k: np.ndarray) -> np.ndarray:
    """[G_p (S_c . m)]_c -> [C][M]."""
    return np.stack([nufft_forward(S[c].astype(np.complex128) * m, k) for c in range(S.shape[0])])


def coil_adjoint(y: np.ndarray, S: np.ndarray, k: np.ndarray, shape) -> np.ndarray:
    """sum_c conj(S_c) . G_p^H y_c."""
    out = np.zeros(shape, dtype=np.complex128)
    for c in range(S.shape[0]):
        out += np.conj(S[c].astype(np.complex128)) * nufft_adjoint(y[c], k, shape)
    return out


def sense_forward(x, ds, S, ks):
    """Stacked forward model (Eq. 10): list over states of [C][M_p]."""
    x = np.asarray(x, dtype=np.complex128)
    return [coil_forward(warp(x, d), S, k) for d, k in zip(ds, ks)]


def sense_adjoint(ys, ds, S, ks, shape):
    """sum_p A_p^H y_p."""
    out = np.zeros(shape, dtype=np.complex128)
    for y, d, k in zip(ys, ds, ks):
        out += warp_adjoint(coil_adjoint(y, S, k, shape), d)
    return out


def normal(x, lam, ds, S, ks):
    """(sum_p A_p^H A_p + lambda I) x."""
    x = np.asarray(x, dtype=np.complex128)
    return sense_adjoint(sense_forward(x, ds, S, ks), ds, S, ks, x.shape) + lam * x


def loss(x, ds, S, ks, ys) -> float:
    """L = sum_p 1/2 ||A_p x - y_p||^2."""
    r = [a - np.asarray(y, dtype=np.complex128) for a, y in zip(sense_forward(x, ds, S, ks), ys)]
    return 0.5 * float(sum(np.vdot(ri, ri).real for ri in r))


def loss_grads(x, ds, S, ks, ys):
    """Gradients of ``loss``.

    grad_x = sum_p A_p^H (A_p x - y_p)  (d L/d Re x + i d L/d Im x).
    grad_{d_p,i}[r] = Re(conj(v_p[r]) * d(T_p x)[r]/d d_{p,i}[r]) with
    v_p = sum_c conj(S_c) G_p^H (A_p x - y_p)_c: the chain rule through the
    linear maps S and G_p.
    """
    x = np.asarray(x, dtype=np.complex128)
    shape = x.shape
    gx = np.zeros(shape, dtype=np.complex128)
    gds = []
    for d, k, y in zip(ds, ks, ys):
        r = coil_forward(warp(x, d), S, k) - np.asarray(y, dtype=np.complex128)
        v = coil_adjoint(r, S, k, shape)
        gx += warp_adjoint(v, d)
        J = warp_jacobian(x, d)
        gds.append(np.real(np.conj(v)[None] * J))
    return gx, gds
