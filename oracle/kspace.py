"""Inverse k-space gridding G (type-2 NUFFT) and k-space gridding G^H
(type-1 NUFFT), plus the direct NDFT they approximate (oracle; test
infrastructure only).

  G^H (Eq. 1-2):  P^(k) -> F^H -> Z^H -> 1/c[x]
  G   (Eq. 3):    1/c*[x] -> Z -> F -> B^(k)

Readings of what the paper leaves open:
* k in cycles/voxel, in [-0.5, 0.5); grid coordinate kappa = G k (FP64);
* image voxel n sits at the centred position x = n - n/2 and is zero-padded
  to grid index x mod G;
* the approximated operator is the orthonormally scaled NDFT
  y(k) = |N|^{-1/2} sum_x z[x] exp(-2 pi i k.x);
* no density compensation: the "density corrected" data of the notation
  table belongs to direct gridding reconstruction, not to the inverse
  problem of Eq. 11.
"""
import numpy as np
import scipy.fft as sfft

from .grid import gather, spread
from .kernel import ALPHA, kb_ft

WORKERS = -1


def centred_positions(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - n // 2


def _deapod_x(shape, gshape) -> np.ndarray:
    """prod_i C(x_i / G_i) over the centred image positions."""
    out = np.ones(shape)
    for i, (n, G) in enumerate(zip(shape, gshape)):
        sh = [1] * len(shape)
        sh[i] = n
        out = out * kb_ft(centred_positions(n) / G).reshape(sh)
    return out


def grid_coords(k: np.ndarray, gshape) -> np.ndarray:
    """kappa = G * k in FP64 from the (float32) trajectory, [M][ndim]."""
    return np.asarray(k, dtype=np.float64) * np.asarray(gshape, dtype=np.float64)[None, :]


def _pad_index(shape, gshape):
    return np.ix_(*[np.mod(centred_positions(n).astype(np.int64), G)
                    for n, G in zip(shape, gshape)])


def nufft_forward(z: np.ndarray, k: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    """G z: deapodize by 1/C(x/G), zero-pad (centred), unnormalised DFT
    scaled by |N|^{-1/2}, then interpolate at kappa = G k."""
    shape = z.shape
    gshape = tuple(alpha * n for n in shape)
    Z = np.zeros(gshape, dtype=np.complex128)
    Z[_pad_index(shape, gshape)] = np.asarray(z, dtype=np.complex128) / _deapod_x(shape, gshape)
    Zh = sfft.fftn(Z, workers=WORKERS) / np.sqrt(np.prod(shape))
    return gather(Zh, grid_coords(k, gshape))


def nufft_adjoint(y: np.ndarray, k: np.ndarray, shape, alpha: int = ALPHA) -> np.ndarray:
    """G^H y: spread at kappa = G k, unnormalised inverse DFT scaled by
    |N|^{-1/2}, crop the centred image, divide by C(x/G)."""
    shape = tuple(shape)
    gshape = tuple(alpha * n for n in shape)
    Y = spread(np.asarray(y, dtype=np.complex128), grid_coords(k, gshape), gshape)
    # ifftn carries 1/|G|; the unnormalised inverse is ifftn * |G|.
    Yh = sfft.ifftn(Y, workers=WORKERS) * (np.prod(gshape) / np.sqrt(np.prod(shape)))
    return Yh[_pad_index(shape, gshape)] / _deapod_x(shape, gshape)


def ndft(z: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Direct NDFT y_j = |N|^{-1/2} sum_x z[x] exp(-2 pi i k_j . x) with
    centred x.  O(M |N|): tiny problems only."""
    shape = z.shape
    pos = np.stack(np.meshgrid(*[centred_positions(n) for n in shape], indexing="ij"),
                   axis=-1).reshape(-1, len(shape))
    E = np.exp(-2j * np.pi * (np.asarray(k, dtype=np.float64) @ pos.T))
    return (E @ np.asarray(z, dtype=np.complex128).reshape(-1)) / np.sqrt(np.prod(shape))


def ndft_adjoint(y: np.ndarray, k: np.ndarray, shape) -> np.ndarray:
    pos = np.stack(np.meshgrid(*[centred_positions(n) for n in shape], indexing="ij"),
                   axis=-1).reshape(-1, len(shape))
    E = np.exp(+2j * np.pi * (pos @ np.asarray(k, dtype=np.float64).T))
    return (E @ np.asarray(y, dtype=np.complex128)).reshape(shape) / np.sqrt(np.prod(shape))
