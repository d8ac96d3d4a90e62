"""Orthonormal multi-level Haar wavelet transform of a 1D, 2D or 3D array
(oracle; test infrastructure only).

Eq. 11 and Eq. 13 regularise with ||W x||_1, W "a sparsifying operator, such
as a wavelet transform" (the paper names no wavelet family, no level count
and no boundary rule).  The reading used here: the orthonormal Haar wavelet
(Daubechies' wavelet of one vanishing moment), applied separably along
every axis, `levels` times on the low-pass band (the Mallat pyramid), on
axes whose lengths are divisible by 2^levels, so W^H = W^{-1}.

One level along one axis maps the pair (a, b) at positions 2j, 2j + 1 to
the low-pass value (a + b)/sqrt(2) at position j and the high-pass value
(a - b)/sqrt(2) at position j + n/2.  A level of the separable transform
applies this along axis 0, then axis 1, then axis 2 to the current low-pass
box [0, n_0/2^l) x ...; the coarsest low-pass box (all axes low-pass at the
last level) holds the approximation coefficients, everything else detail
coefficients.
"""
import numpy as np


def _haar_axis(a: np.ndarray, axis: int) -> np.ndarray:
    a = np.moveaxis(a, axis, 0)
    lo = (a[0::2] + a[1::2]) / np.sqrt(2.0)
    hi = (a[0::2] - a[1::2]) / np.sqrt(2.0)
    return np.moveaxis(np.concatenate([lo, hi], axis=0), 0, axis)


def _ihaar_axis(a: np.ndarray, axis: int) -> np.ndarray:
    a = np.moveaxis(a, axis, 0)
    h = a.shape[0] // 2
    lo, hi = a[:h], a[h:]
    out = np.empty_like(a)
    out[0::2] = (lo + hi) / np.sqrt(2.0)
    out[1::2] = (lo - hi) / np.sqrt(2.0)
    return np.moveaxis(out, 0, axis)


def check_levels(shape, levels: int) -> None:
    if levels < 1 or any(n % (1 << levels) for n in shape):
        raise ValueError(f"every length must be divisible by 2^{levels}")


def forward(x: np.ndarray, levels: int) -> np.ndarray:
    """W x: Mallat layout, same shape as x."""
    x = np.asarray(x, dtype=np.complex128)
    check_levels(x.shape, levels)
    w = x.copy()
    box = list(x.shape)
    for _ in range(levels):
        sl = tuple(slice(0, b) for b in box)
        sub = w[sl]
        for ax in range(x.ndim):
            sub = _haar_axis(sub, ax)
        w[sl] = sub
        box = [b // 2 for b in box]
    return w


def inverse(w: np.ndarray, levels: int) -> np.ndarray:
    """W^H w = W^{-1} w."""
    w = np.asarray(w, dtype=np.complex128)
    check_levels(w.shape, levels)
    x = w.copy()
    boxes = []
    box = list(w.shape)
    for _ in range(levels):
        boxes.append(list(box))
        box = [b // 2 for b in box]
    for box in reversed(boxes):
        sl = tuple(slice(0, b) for b in box)
        sub = x[sl]
        for ax in reversed(range(w.ndim)):
            sub = _ihaar_axis(sub, ax)
        x[sl] = sub
    return x


def approximation_mask(shape, levels: int) -> np.ndarray:
    """True on the approximation coefficients (the coarsest low-pass box)."""
    m = np.zeros(shape, dtype=bool)
    m[tuple(slice(0, n >> levels) for n in shape)] = True
    return m
