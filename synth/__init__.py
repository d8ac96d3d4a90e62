"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws inputs: phantoms, displacement fields, coil
sensitivities, non-Cartesian trajectories and noise.  It holds none of the
method's arithmetic (no kernel, no FFT, no gridding), so the oracle and the
HIP path can both take their inputs from here without sharing any of the
computation that is being checked.

The paper measures on in-vivo free-breathing coronary data (section
"Nonrigid Respiratory Motion Correction"); none of that data exists here, so
every workload is synthetic with the structure of that experiment: a 3D
object, several respiratory states with smooth nonrigid displacement fields,
smooth multi-coil sensitivities and a 3D non-Cartesian trajectory whose
interleaves are dealt out to the respiratory states.

Every generator is driven by ``numpy.random.default_rng`` seeded from
``SeedSequence([16713, cfg, purpose, index])`` so that any test, the smoke
check and the benchmark see identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 16713
# purpose ids of the seed sequence
P_PHANTOM, P_MOTION, P_COILS, P_NOISE, P_SEGMENTS, P_MISC = 0, 1, 2, 3, 4, 5

# Multidimensional golden means for 3D golden-angle radial ordering
# (Chan, Ramsay, Ramanujam, MRM 2009).
GOLDEN_3D = (0.4656, 0.6823)
# 2D golden angle in radians (111.246... degrees).
GOLDEN_2D = math.pi * (3.0 - math.sqrt(5.0))


def rng(cfg: int, purpose: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, cfg, purpose, index]))


# ----------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------

def _random_rotation(g: np.random.Generator, ndim: int) -> np.ndarray:
    if ndim == 2:
        a = g.uniform(0.0, math.pi)
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s], [s, c]])
    # uniform random unit quaternion (Shoemake)
    u1, u2, u3 = g.uniform(0.0, 1.0, 3)
    q = np.array([
        math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
        math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
        math.sqrt(u1) * math.sin(2 * math.pi * u3),
        math.sqrt(u1) * math.cos(2 * math.pi * u3),
    ])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_phantom(shape, count: int = 10, g: np.random.Generator | None = None) -> np.ndarray:
    """Sum of ``count`` solid ellipses (2D) or ellipsoids (3D) with random
    complex amplitudes, as complex128.

    Centres are uniform in [0.2 n, 0.8 n], semi-axes uniform in
    [0.05 n, 0.25 n], orientation uniform, amplitude rho*exp(i theta) with
    rho ~ U[0.2, 1] and theta ~ U[-pi, pi).
    """
    g = g if g is not None else rng(0, P_PHANTOM)
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    n = np.array(shape, dtype=np.float64)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    pos = np.stack(grids, axis=-1)
    img = np.zeros(shape, dtype=np.complex128)
    for _ in range(count):
        c = g.uniform(0.2, 0.8, ndim) * n
        ax = g.uniform(0.05, 0.25, ndim) * n
        R = _random_rotation(g, ndim)
        rho = g.uniform(0.2, 1.0)
        th = g.uniform(-math.pi, math.pi)
        q = (pos - c) @ R  # coordinates in the ellipsoid frame
        inside = np.sum((q / ax) ** 2, axis=-1) <= 1.0
        img[inside] += rho * np.exp(1j * th)
    return img


# ----------------------------------------------------------------------------
# displacement fields
# ----------------------------------------------------------------------------

def bump_displacement(shape, bumps: int, sigma: float, dmax: float,
                      g: np.random.Generator | None = None) -> np.ndarray:
    """Smooth displacement field, float32 [ndim][*shape], in voxels.

    d(r) = sum_b a_b exp(-|r - c_b|^2 / (2 sigma^2)) with the periodic
    (minimum-image) distance, a_b ~ N(0, I), centres uniform over the volume,
    then rescaled so that max_r ||d(r)||_2 == dmax.  Component i displaces
    along array axis i.
    """
    g = g if g is not None else rng(0, P_MOTION)
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    d = np.zeros((ndim,) + shape, dtype=np.float64)
    for _ in range(bumps):
        c = g.uniform(0.0, 1.0, ndim) * np.array(shape)
        a = g.standard_normal(ndim)
        r2 = np.zeros(shape, dtype=np.float64)
        for i, n in enumerate(shape):
            t = np.arange(n, dtype=np.float64) - c[i]
            t = t - n * np.round(t / n)  # minimum image
            sh = [1] * ndim
            sh[i] = n
            r2 = r2 + (t ** 2).reshape(sh)
        bump = np.exp(-r2 / (2.0 * sigma * sigma))
        for i in range(ndim):
            d[i] += a[i] * bump
    mag = np.sqrt(np.sum(d ** 2, axis=0)).max()
    if mag > 0:
        d *= dmax / mag
    return d.astype(np.float32)


# ----------------------------------------------------------------------------
# coil sensitivities
# ----------------------------------------------------------------------------

def _fibonacci_directions(count: int, ndim: int) -> np.ndarray:
    if ndim == 2:
        a = 2 * math.pi * np.arange(count) / count
        return np.stack([np.cos(a), np.sin(a)], axis=-1)
    i = np.arange(count) + 0.5
    z = 1.0 - 2.0 * i / count
    r = np.sqrt(1.0 - z * z)
    phi = math.pi * (1.0 + math.sqrt(5.0)) * i
    return np.stack([z, r * np.cos(phi), r * np.sin(phi)], axis=-1)


def coil_maps(shape, ncoils: int, g: np.random.Generator | None = None,
              dtype=np.complex64) -> np.ndarray:
    """Smooth complex coil sensitivities [C][*shape] with sum_c |S_c|^2 == 1.

    Coil c sits at p_c on a Fibonacci sphere (circle in 2D) of radius 0.6 n
    around the centre; S_c = exp(-|r-p_c|^2 / (2 (0.5 n)^2)) *
    exp(i (phi_c + 2 pi g_c . (r - n/2) / n)), phi_c ~ U[-pi, pi),
    |g_c| <= 0.5, then normalised voxelwise by sqrt(sum_c |S_c|^2).
    """
    g = g if g is not None else rng(0, P_COILS)
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    n = np.array(shape, dtype=np.float64)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    pos = np.stack(grids, axis=-1)
    dirs = _fibonacci_directions(ncoils, ndim)
    out = np.zeros((ncoils,) + shape, dtype=np.complex128)
    for c in range(ncoils):
        p = n / 2 + 0.6 * n * dirs[c]
        mag = np.exp(-np.sum(((pos - p) / (0.5 * n)) ** 2, axis=-1) / 2.0)
        phi = g.uniform(-math.pi, math.pi)
        gv = g.standard_normal(ndim)
        gv *= g.uniform(0.0, 0.5) / max(np.linalg.norm(gv), 1e-12)
        ph = phi + 2 * math.pi * np.sum(gv * (pos - n / 2) / n, axis=-1)
        out[c] = mag * np.exp(1j * ph)
    out /= np.sqrt(np.sum(np.abs(out) ** 2, axis=0))
    return out.astype(dtype)


# ----------------------------------------------------------------------------
# trajectories (cycles/voxel, in [-0.5, 0.5))
# ----------------------------------------------------------------------------

def radial_spokes_3d(first: int, count: int, readout: int) -> np.ndarray:
    """Spokes first..first+count-1 of a 3D golden-angle radial sequence,
    float32 [count*readout][3].  Spoke s has direction
    (sqrt(1-u^2) cos a, sqrt(1-u^2) sin a, u) with u = frac(s*0.4656) and
    a = 2 pi frac(s*0.6823); sample j of a spoke sits at (j - L/2)/L along
    it (component i is along array axis i)."""
    s = np.arange(first, first + count, dtype=np.float64)
    u = np.mod(s * GOLDEN_3D[0], 1.0)
    a = 2 * math.pi * np.mod(s * GOLDEN_3D[1], 1.0)
    rho = np.sqrt(1.0 - u * u)
    dirs = np.stack([rho * np.cos(a), rho * np.sin(a), u], axis=-1)
    t = (np.arange(readout, dtype=np.float64) - readout / 2) / readout
    k = dirs[:, None, :] * t[None, :, None]
    return k.reshape(-1, 3).astype(np.float32)


def radial_spokes_2d(first: int, count: int, readout: int) -> np.ndarray:
    s = np.arange(first, first + count, dtype=np.float64)
    a = s * GOLDEN_2D
    dirs = np.stack([np.cos(a), np.sin(a)], axis=-1)
    t = (np.arange(readout, dtype=np.float64) - readout / 2) / readout
    k = dirs[:, None, :] * t[None, :, None]
    return k.reshape(-1, 2).astype(np.float32)


def uniform_samples(count: int, ndim: int, g: np.random.Generator) -> np.ndarray:
    """Uniformly random k-space points in [-0.5, 0.5)^ndim, float32."""
    k = g.uniform(-0.5, 0.5, (count, ndim)).astype(np.float32)
    return np.where(k >= 0.5, np.float32(-0.5), k)


def binned_radial_phases(spokes_per_phase, readout: int, segment: int,
                         g: np.random.Generator) -> list:
    """Deal heartbeat segments of ``segment`` consecutive spokes of ONE
    global golden-angle sequence to respiratory phases at random, giving each
    phase exactly ``spokes_per_phase[p]`` spokes.  This imitates binning
    heartbeats into respiratory phases by their navigator position."""
    counts = [int(s) // segment for s in spokes_per_phase]
    assert all(c * segment == s for c, s in zip(counts, spokes_per_phase))
    order = g.permutation(sum(counts))
    out, pos = [], 0
    for c in counts:
        segs = np.sort(order[pos:pos + c])
        pos += c
        out.append(np.concatenate([radial_spokes_3d(int(sg) * segment, segment, readout)
                                   for sg in segs], axis=0))
    return out


def complex_noise(shape, g: np.random.Generator, dtype=np.complex64) -> np.ndarray:
    """(N(0,1) + i N(0,1)) / sqrt(2)."""
    z = (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / math.sqrt(2.0)
    return z.astype(dtype)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    cfg: int
    shape: tuple
    ncoils: int
    nphases: int
    dmax: float
    bumps: int
    sigma: float
    spokes: list = field(default_factory=list)   # per phase
    readout: int = 0
    segment: int = 0
    lam: float = 0.0
    cg_iters: int = 0


WORKLOADS = {
    # 2D warp only: 64x64, 10 ellipses, 4 bumps sigma 8 px, max |d| 3 px
    "warp2d_64": Workload("warp2d_64", 1, (64, 64), 1, 1, 3.0, 4, 8.0),
    # 3D nonrigid SENSE, 1 phase, 96^3, 8 coils, 2000 spokes x 96
    "sense3d_96": Workload("sense3d_96", 2, (96, 96, 96), 8, 1, 8.0, 6, 12.0,
                           [2000], 96, 25, 1e-3, 20),
    # batched phases: 160^3, 12 coils, 6 phases, 80k..600k samples per phase
    "batched_160": Workload("batched_160", 3, (160, 160, 160), 12, 6, 10.0, 6, 20.0,
                            [500, 1125, 1750, 2375, 3000, 3750], 160, 25, 1e-3, 20),
    # differentiation: 128^3, 8 coils, 4 phases
    "grad_128": Workload("grad_128", 4, (128, 128, 128), 8, 4, 8.0, 6, 16.0,
                         [2000] * 4, 128, 25, 1e-3, 0),
    # mixed precision at scale: 256^3, 16 coils, 8 phases, ~1.5M samples/phase
    "mixed_256": Workload("mixed_256", 5, (256, 256, 256), 16, 8, 10.0, 6, 32.0,
                          [5860] * 8, 256, 20, 1e-3, 30),
    # the same at 128^3 (16 coils, 8 phases, a quarter of the spokes: the same
    # radial sampling density), small enough for a 30-iteration FP64 CG
    "mixed_128": Workload("mixed_128", 6, (128, 128, 128), 16, 8, 10.0, 6, 16.0,
                          [1460] * 8, 128, 20, 1e-3, 30),
}


def small_workload(shape=(16, 16, 16), ncoils=3, nphases=2, spokes=(40, 60),
                   readout=None, dmax=2.5, cfg=100) -> Workload:
    readout = readout or shape[0]
    return Workload(f"small_{'x'.join(map(str, shape))}", cfg, tuple(shape), ncoils,
                    nphases, dmax, 3, shape[0] / 6.0, list(spokes), readout, 1, 1e-2, 8)


def make_inputs(w: Workload, with_traj: bool = True) -> dict:
    """All inputs of a workload: image x (complex64), displacement fields
    d_p (float32 [ndim][n]), coil maps S (complex64 [C][n]) and trajectories
    k_p (float32 [M_p][ndim])."""
    shape = w.shape
    ndim = len(shape)
    x = ellipsoid_phantom(shape, 10, rng(w.cfg, P_PHANTOM)).astype(np.complex64)
    ds = [bump_displacement(shape, w.bumps, w.sigma, w.dmax, rng(w.cfg, P_MOTION, p))
          for p in range(w.nphases)]
    S = coil_maps(shape, w.ncoils, rng(w.cfg, P_COILS))
    ks = []
    if with_traj and w.spokes:
        if ndim == 3 and w.segment > 1:
            ks = binned_radial_phases(w.spokes, w.readout, w.segment, rng(w.cfg, P_SEGMENTS))
        elif ndim == 3:
            first = 0
            for s in w.spokes:
                ks.append(radial_spokes_3d(first, s, w.readout))
                first += s
        else:
            first = 0
            for s in w.spokes:
                ks.append(radial_spokes_2d(first, s, w.readout))
                first += s
    return {"x": x, "d": ds, "S": S, "k": ks}
