"""Bulk-translation correction by a linear phase, density compensation and
direct k-space gridding reconstruction (oracle; test infrastructure only).

Section "Motion Capturing for Segmented Data Acquisitions": low-resolution
3D iNAVs are reconstructed from data near the k-space origin, translational
motion is estimated per heartbeat, and the estimated bulk translation is
corrected "by applying linear phase shifts to the k-space data"; direct
gridding reconstructs from density-corrected data M(k) (notation table;
Eq. 1-2).

Readings (the paper gives no formulas for these steps):
* translation t (voxels, component i along array axis i) of the object
  during sample j multiplies that sample by exp(-2 pi i k_j . t_j) (with the
  NDFT convention y(k) = |N|^{-1/2} sum_x z[x] exp(-2 pi i k.x), a shifted
  object z[x - t] has exactly this factor); correcting data multiplies by
  the conjugate.  The translated forward model is ph o G z, its adjoint
  G^H(conj(ph) o y);
* density compensation by the iteration of Pipe and Menon (MRM 1999) with
  the gridding kernel itself: w_0 = 1, w_{i+1} = w_i / (P w_i),
  (P w)_j = sum_l w_l sum_q c~(kappa_j - q) c~(kappa_l - q), i.e. a spread
  of the weights onto the oversampled grid followed by a gather at the
  samples, with the Kaiser-Bessel kernel of ``kernel`` scaled to unit
  integral per axis, c~ = c / C(0), so that w_j is about the reciprocal of
  the number of samples per grid cell around sample j;
* direct gridding reconstruction of multi-coil data:
  x = sum_c conj(S_c) o G^H(w o conj(ph) o y_c).
"""
import numpy as np

from .grid import gather, spread
from .kernel import kb_ft
from .kspace import grid_coords, nufft_adjoint, nufft_forward


def phase(k: np.ndarray, t: np.ndarray) -> np.ndarray:
    """exp(-2 pi i k_j . t_j) per sample; k [M][ndim] cycles/voxel, t [M][ndim]
    voxels (or one [ndim] shift for every sample)."""
    k = np.asarray(k, dtype=np.float64)
    t = np.broadcast_to(np.asarray(t, dtype=np.float64), k.shape)
    return np.exp(-2j * np.pi * np.sum(k * t, axis=1))


def translated_forward(z, k, t):
    """ph o G z: the forward model of the object translated by t."""
    return phase(k, t) * nufft_forward(z, k)


def translated_adjoint(y, k, t, shape):
    """G^H(conj(ph) o y)."""
    return nufft_adjoint(np.conj(phase(k, t)) * np.asarray(y, dtype=np.complex128), k, shape)


def dcf(k: np.ndarray, shape, iters: int, alpha: int = 2) -> np.ndarray:
    """Pipe-Menon density compensation weights after `iters` iterations."""
    gshape = tuple(alpha * n for n in shape)
    kap = grid_coords(k, gshape)
    unit = kb_ft(0.0) ** (2 * len(shape))  # two kernel factors per axis, each divided by C(0)
    w = np.ones(k.shape[0])
    for _ in range(iters):
        pw = gather(spread(w.astype(np.complex128), kap, gshape), kap).real / unit
        w = w / pw
    return w


def dcf_apply(w: np.ndarray, k: np.ndarray, shape, alpha: int = 2) -> np.ndarray:
    """P w with the unit-integral kernel (the quantity the iteration drives to 1)."""
    gshape = tuple(alpha * n for n in shape)
    kap = grid_coords(k, gshape)
    unit = kb_ft(0.0) ** (2 * len(shape))
    return gather(spread(np.asarray(w, dtype=np.complex128), kap, gshape), kap).real / unit


def grid_recon(y: np.ndarray, k: np.ndarray, S: np.ndarray, shape, w=None, t=None) -> np.ndarray:
    """sum_c conj(S_c) o G^H(w o conj(ph) o y_c); y [C][M]; w, t optional."""
    y = np.asarray(y, dtype=np.complex128)
    M = k.shape[0]
    wt = np.ones(M) if w is None else np.asarray(w, dtype=np.float64)
    ph = np.ones(M) if t is None else np.conj(phase(k, t))
    out = np.zeros(shape, dtype=np.complex128)
    for c in range(y.shape[0]):
        out += np.conj(np.asarray(S[c], dtype=np.complex128)) * nufft_adjoint(wt * ph * y[c], k, shape)
    return out
