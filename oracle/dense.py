"""Brute-force dense matrices of T_d and G from explicit double sums, with no
FFT anywhere (oracle; test infrastructure only).  Tiny problems only.

They restate the same definitions as ``warp`` and ``kspace`` term by term, so
any slip in the FFT-based functions (a wrong scale, a misplaced pad or crop
index, a flipped exponent sign) shows up as a mismatch.

T_d (Eq. 9) entry for output voxel r and input voxel s:
  T[r, s] = sum_taps prod_i c(y_i(r) - g_i) * h_i(g_i, s_i),
  h_i(g, s) = (1/n_i) sum_{k in K_i} exp(+2 pi i k g / G_i) exp(-2 pi i k s / n_i) / C(k / G_i)
with y(r) = alpha (r + d(r)) and the taps of the tap rule.

G (Eq. 3) entry for sample j and centred voxel x:
  G[j, x] = |N|^{-1/2} sum_taps prod_i c(kappa_ji - q_i) exp(-2 pi i q_i x_i / G_i) / C(x_i / G_i).
"""
import itertools

import numpy as np

from .kernel import ALPHA, WIDTH, kb, kb_ft


def _taps(y: float):
    base = np.floor(y) - WIDTH // 2 + 1
    return [(base + t, float(kb(np.array(y - (base + t))))) for t in range(WIDTH)]


def warp_matrix(d: np.ndarray, alpha: int = ALPHA) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    ndim = d.shape[0]
    shape = d.shape[1:]
    gshape = tuple(alpha * n for n in shape)
    # h_i[g][s] for g in 0..G-1 (periodic, so any integer g reduces mod G)
    h = []
    for n, G in zip(shape, gshape):
        K = np.array([k if k < n - n // 2 else k - n for k in range(n)], dtype=np.float64)
        hk = np.zeros((G, n), dtype=np.complex128)
        for g in range(G):
            for s in range(n):
                hk[g, s] = np.sum(np.exp(2j * np.pi * K * g / G) * np.exp(-2j * np.pi * K * s / n)
                                  / kb_ft(K / G)) / n
        h.append(hk)
    size = int(np.prod(shape))
    T = np.zeros((size, size), dtype=np.complex128)
    for row, r in enumerate(itertools.product(*[range(n) for n in shape])):
        y = [alpha * r[i] + alpha * d[(i,) + r] for i in range(ndim)]
        per_axis = []
        for i in range(ndim):
            acc = np.zeros(shape[i], dtype=np.complex128)
            for g, w in _taps(y[i]):
                acc += w * h[i][int(g) % gshape[i]]
            per_axis.append(acc)
        full = per_axis[0]
        for a in per_axis[1:]:
            full = np.multiply.outer(full, a)
        T[row] = full.reshape(-1)
    return T


def nufft_matrix(k: np.ndarray, shape, alpha: int = ALPHA) -> np.ndarray:
    k = np.asarray(k, dtype=np.float64)
    shape = tuple(shape)
    ndim = len(shape)
    gshape = tuple(alpha * n for n in shape)
    M = k.shape[0]
    A = np.zeros((M, int(np.prod(shape))), dtype=np.complex128)
    xs = [np.arange(n, dtype=np.float64) - n // 2 for n in shape]
    for j in range(M):
        per_axis = []
        for i in range(ndim):
            kap = gshape[i] * k[j, i]
            acc = np.zeros(shape[i], dtype=np.complex128)
            for q, w in _taps(kap):
                acc += w * np.exp(-2j * np.pi * q * xs[i] / gshape[i])
            per_axis.append(acc / kb_ft(xs[i] / gshape[i]))
        full = per_axis[0]
        for a in per_axis[1:]:
            full = np.multiply.outer(full, a)
        A[j] = full.reshape(-1) / np.sqrt(np.prod(shape))
    return A
