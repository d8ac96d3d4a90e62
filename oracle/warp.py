"""Image-space gridding T_d and its adjoint T_d^H (oracle; test
infrastructure only).

Warp by a displacement field (Eq. 5): the warped image at voxel r is the
object at r + d(r) (pull convention, d in voxels, component i along array
axis i).  Those warped positions are non-Cartesian points on the reference
grid, so T is computed like inverse k-space gridding but in image space
(section "Image-space Gridding"):

  forward (Eq. 9):  F -> 1/C*[k] -> Z -> F^H -> B_d
  adjoint (Eq. 8):  P_d -> F -> Z^H -> 1/C[k] -> F^H

Readings of what the paper leaves open:
* oversampling alpha = 2, so voxel r sits at grid coordinate alpha*r;
* F is the unnormalised DFT; the inverse DFT onto the oversampled grid is
  scaled so that u[g] = (1/|N|) sum_k U[k] exp(+2 pi i k.g/G), which makes
  T_0 equal the identity up to the kernel's approximation error;
* the spectrum of an even-length axis is K = {-n/2, ..., n/2 - 1} placed at
  index k mod G (no Hermitian symmetrisation of the Nyquist bin);
* the oversampled grid is periodic (wrap-around);
* C is the continuous transform of the kernel; it is real, so C* = C.
"""
import numpy as np
import scipy.fft as sfft

from .grid import gather, gather_deriv, spread
from .kernel import ALPHA, kb_ft

WORKERS = -1  # scipy.fft: use every host core


def _freqs(n: int) -> np.ndarray:
    """Signed frequencies of the DFT bins 0..n-1: K = {-n/2..n/2-1}."""
    j = np.arange(n)
    return np.where(j < n - n // 2, j, j - n)


def _deapod_k(shape, gshape) -> np.ndarray:
    """prod_i C(k_i / G_i) on the n-point spectrum, in DFT bin order."""
    out = np.ones(shape)
    for i, (n, G) in enumerate(zip(shape, gshape)):
        sh = [1] * len(shape)
        sh[i] = n
        out = out * kb_ft(_freqs(n) / G).reshape(sh)
    return out


def oversampled_shape(shape, alpha: int = ALPHA):
    return tuple(alpha * int(n) for n in shape)


def upsample(x: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """The d-independent front end of Eq. 9: F, divide by C, zero-pad Z,
    then F^H onto the oversampled grid with the 1/|N| scale."""
    shape = x.shape
    gshape = oversampled_shape(shape, alpha)
    X = sfft.fftn(np.asarray(x, dtype=np.complex128), workers=WORKERS)
    X = X / _deapod_k(shape, gshape)
    U = np.zeros(gshape, dtype=np.complex128)
    U[np.ix_(*[np.mod(_freqs(n), G) for n, G in zip(shape, gshape)])] = X
    # ifftn carries 1/|G|; the wanted scale is 1/|N|.
    return sfft.ifftn(U, workers=WORKERS) * (np.prod(gshape) / np.prod(shape))


def warp_coords(d: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """Oversampled-grid coordinates alpha*(r + d(r)) of every voxel, [npts][ndim],
    computed in FP64 from the (float32) field."""
    d = np.asarray(d, dtype=np.float64)
    ndim = d.shape[0]
    shape = d.shape[1:]
    r = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return np.stack([alpha * r[i].reshape(-1) + alpha * d[i].reshape(-1)
                     for i in range(ndim)], axis=-1)


def warp(x: np.ndarray, d: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """T_d x (Eq. 9)."""
    u = upsample(x, alpha)
    return gather(u, warp_coords(d, alpha)).reshape(x.shape)


def warp_at(x: np.ndarray, d: np.ndarray, voxels: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """T_d x evaluated only at the listed flat voxel indices (same definition,
    restricted output)."""
    u = upsample(x, alpha)
    coords = warp_coords(d, alpha)[np.asarray(voxels)]
    return gather(u, coords)


def warp_adjoint(v: np.ndarray, d: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """T_d^H v (Eq. 7-8): spread onto the oversampled grid, F, crop the
    central spectrum Z^H, divide by C, then F^H with the 1/|N| scale."""
    shape = v.shape
    gshape = oversampled_shape(shape, alpha)
    Up = spread(v.reshape(-1), warp_coords(d, alpha), gshape)
    Uh = sfft.fftn(Up, workers=WORKERS)
    V = Uh[np.ix_(*[np.mod(_freqs(n), G) for n, G in zip(shape, gshape)])]
    V = V / _deapod_k(shape, gshape)
    return sfft.ifftn(V, workers=WORKERS)


def warp_multi_adjoint(vs, ds, alpha: int = ALPHA) -> np.ndarray:
    """sum_p T_{d_p}^H v_p."""
    return sum(warp_adjoint(v, d, alpha) for v, d in zip(vs, ds))


def warp_jacobian(x: np.ndarray, d: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """d(T_d x)[r] / d d_i[r] for every axis i, [ndim][*shape] complex.
    y_i = alpha (r_i + d_i), so the chain rule brings a factor alpha."""
    u = upsample(x, alpha)
    coords = warp_coords(d, alpha)
    return np.stack([alpha * gather_deriv(u, coords, i).reshape(x.shape)
                     for i in range(x.ndim)])


def warp_grad_d(x: np.ndarray, d: np.ndarray, v: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """Gradient of Re<v, T_d x> with respect to d:
    grad_i[r] = Re(conj(v[r]) * d(T_d x)[r]/d d_i[r]), [ndim][*shape] float64."""
    J = warp_jacobian(x, d, alpha)
    return np.real(np.conj(v)[None] * J)
