"""Projection Core (spread) and Backprojection Core (gather) on a periodic
oversampled Cartesian grid (oracle; test infrastructure only).

The Projection Core convolves non-Cartesian values with the kernel and
samples the result on the oversampled grid (Eq. 1 and its process diagram
Eq. 2; Fig. 1a).  The Backprojection Core is its adjoint: it interpolates the
grid at the non-Cartesian points (Eq. 3; Fig. 1b).  The image-space
versions (Eq. 7-9) use the same two cores with the warped voxel positions
as the non-Cartesian points.

Tap rule (a reading; the paper gives none).  For a coordinate y in grid units
the taps along one axis are g = floor(y) - W/2 + 1 + t, t = 0..W-1, and the
weight of the tap is c(y - g).  The grid is periodic (implied by the DFTs
around the cores), so tap g reads/writes index g mod G.
"""
import numpy as np

from .kernel import WIDTH, kb, kb_deriv


def taps_1d(y, G: int, width: int = WIDTH):
    """For coordinates y [npts] return (indices [W][npts] in 0..G-1,
    offsets y - g [W][npts])."""
    y = np.asarray(y, dtype=np.float64)
    base = np.floor(y) - width // 2 + 1
    idx, off = [], []
    for t in range(width):
        g = base + t
        off.append(y - g)
        idx.append(np.mod(g, G).astype(np.int64))
    return np.stack(idx), np.stack(off)


def _tap_loop(coords, gshape, width):
    """Yield (flat grid index, per-axis offsets) for every one of the W^ndim
    tap combinations."""
    ndim = len(gshape)
    per_axis = [taps_1d(coords[..., i], gshape[i], width) for i in range(ndim)]
    strides = [int(np.prod(gshape[i + 1:])) for i in range(ndim)]
    for combo in np.ndindex(*([width] * ndim)):
        flat = np.zeros(coords.shape[0], dtype=np.int64)
        offs = []
        for i, t in enumerate(combo):
            flat += per_axis[i][0][t] * strides[i]
            offs.append(per_axis[i][1][t])
        yield flat, offs


def gather(grid: np.ndarray, coords: np.ndarray, width: int = WIDTH) -> np.ndarray:
    """Backprojection Core B: out[j] = sum_taps prod_i c(y_ji - g_i) grid[g mod G].
    coords is [npts][ndim] in grid units."""
    coords = np.asarray(coords, dtype=np.float64)
    flat_grid = grid.reshape(-1)
    out = np.zeros(coords.shape[0], dtype=np.complex128)
    for flat, offs in _tap_loop(coords, grid.shape, width):
        w = np.ones(coords.shape[0])
        for o in offs:
            w = w * kb(o, width)
        out += w * flat_grid[flat]
    return out


def gather_deriv(grid: np.ndarray, coords: np.ndarray, axis: int,
                 width: int = WIDTH) -> np.ndarray:
    """Derivative of ``gather`` with respect to coordinate ``axis``:
    sum_taps c'(y_axis - g_axis) prod_{i != axis} c(y_i - g_i) grid[g]."""
    coords = np.asarray(coords, dtype=np.float64)
    flat_grid = grid.reshape(-1)
    out = np.zeros(coords.shape[0], dtype=np.complex128)
    for flat, offs in _tap_loop(coords, grid.shape, width):
        w = np.ones(coords.shape[0])
        for i, o in enumerate(offs):
            w = w * (kb_deriv(o, width) if i == axis else kb(o, width))
        out += w * flat_grid[flat]
    return out


def spread(values: np.ndarray, coords: np.ndarray, gshape, width: int = WIDTH) -> np.ndarray:
    """Projection Core P (adjoint of ``gather``):
    grid[g mod G] += prod_i c(y_ji - g_i) values[j] over all points and taps.
    The scatter-add uses bincount, which sums duplicate indices."""
    coords = np.asarray(coords, dtype=np.float64)
    values = np.asarray(values, dtype=np.complex128)
    size = int(np.prod(gshape))
    re = np.zeros(size)
    im = np.zeros(size)
    for flat, offs in _tap_loop(coords, gshape, width):
        w = np.ones(coords.shape[0])
        for o in offs:
            w = w * kb(o, width)
        re += np.bincount(flat, weights=w * values.real, minlength=size)
        im += np.bincount(flat, weights=w * values.imag, minlength=size)
    return (re + 1j * im).reshape(gshape)
