"""Python binding of the HIP library: plans, prepared motions and
trajectories, and the operators.  Torch tensors supply device memory and
the stream; every arithmetic step runs in libisg.so.

Layouts follow include/isg.h: images complex64 [n0][n1](/[n2]); fields
float32 [ndim][*shape]; coils complex64 [C][*shape]; trajectories float32
[M][ndim]; data complex64 with the states packed one after another, state
p holding [M_p][C].
"""
from __future__ import annotations

import ctypes as C
import weakref

import torch

from . import _lib
from ._lib import check, isg_plan_desc


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _require(t: torch.Tensor, dtype, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


def device_count() -> int:
    c = C.c_int(0)
    check(_lib.load().isg_device_count(C.byref(c)))
    return c.value


def version() -> str:
    return _lib.load().isg_version().decode()


class Motion:
    """A displacement field prepared for T_d / T_d^H (Eq. 5)."""

    def __init__(self, plan: "Plan", d: torch.Tensor):
        self.plan = plan
        d = _require(d, torch.float32, (plan.ndim,) + plan.shape, "d")
        h = C.c_void_p()
        check(plan.lib.isg_motion_create(plan.handle, _ptr(d), C.byref(h)))
        self.handle = h
        self.d = d
        plan._dependents.add(self)

    def close(self):
        if getattr(self, "handle", None):
            self.plan.lib.isg_motion_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Traj:
    """A trajectory prepared for the k-space pair (Eq. 1-3)."""

    def __init__(self, plan: "Plan", k: torch.Tensor):
        self.plan = plan
        if k.dim() != 2 or k.shape[1] != plan.ndim:
            raise ValueError(f"k must be [M][{plan.ndim}]")
        k = _require(k, torch.float32, None, "k")
        self.M = int(k.shape[0])
        h = C.c_void_p()
        check(plan.lib.isg_traj_create(plan.handle, _ptr(k), self.M, C.byref(h)))
        self.handle = h
        plan._dependents.add(self)

    def info(self) -> dict:
        """{"visits": (sample, tile) spread visits, "tiles": touched spread
        tiles, "tile_points": grid points per tile, "touched_cells": grid
        cells of the touched runs the axis-0 passes move, "active_columns":
        grid columns along axis 0 holding such a run}"""
        a, b, c, f, g = (C.c_int64(0) for _ in range(5))
        check(self.plan.lib.isg_traj_info(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        check(self.plan.lib.isg_traj_touched_cells(self.handle, C.byref(f)))
        check(self.plan.lib.isg_traj_active_columns(self.handle, C.byref(g)))
        return {"visits": a.value, "tiles": b.value, "tile_points": c.value, "touched_cells": f.value,
                "active_columns": g.value}

    def set_shift(self, t: torch.Tensor | None) -> None:
        """Translate the object by t (float32 [M][ndim], voxels) during the
        samples: forward models gain exp(-2 pi i k.t), adjoints its conjugate;
        None removes the translation."""
        self.plan._sync_stream()
        if t is None:
            check(self.plan.lib.isg_traj_set_shift(self.handle, None))
            return
        t = _require(t, torch.float32, (self.M, self.plan.ndim), "t")
        check(self.plan.lib.isg_traj_set_shift(self.handle, _ptr(t)))

    def close(self):
        if getattr(self, "handle", None):
            self.plan.lib.isg_traj_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Shape, tables and scratch for one image geometry.

    shape: image shape (2D or 3D, even lengths 8..512 with factors 2, 3, 5, 7);
    ncoils / nphases: coil count and most states per call; storage: element
    type of the coil-expanded k-space grids ("fp32", "bf16", "fp16");
    alpha / width / beta: oversampling, kernel width and Kaiser-Bessel shape
    (only 2, 4 and the default beta, given as <= 0, are supported).
    """

    def __init__(self, shape, ncoils: int = 1, nphases: int = 1, storage: str = "fp32",
                 device=None, alpha: int = 2, width: int = 4, beta: float = 0.0):
        self.lib = _lib.load()
        self._dependents = weakref.WeakSet()  # live Motion / Traj objects
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.ncoils = int(ncoils)
        self.nphases = int(nphases)
        self.storage = storage
        self.device = torch.device("cuda" if device is None else device)
        desc = isg_plan_desc()
        desc.ndim = self.ndim
        for i, s in enumerate(self.shape):
            desc.n[i] = s
        desc.alpha = int(alpha)
        desc.width = int(width)
        desc.beta = float(beta)
        desc.ncoils = self.ncoils
        desc.nphases = self.nphases
        desc.storage = _lib.STORAGE[storage]
        with torch.cuda.device(self.device):
            desc.stream = torch.cuda.current_stream().cuda_stream
            h = C.c_void_p()
            check(self.lib.isg_plan_create(C.byref(desc), C.byref(h)))
        self.handle = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        """Destroy the plan, after the motions and trajectories still open on it."""
        if getattr(self, "handle", None):
            for dep in list(getattr(self, "_dependents", ())):
                dep.close()
            self.lib.isg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        b = C.c_int64(0)
        check(self.lib.isg_plan_device_bytes(self.handle, C.byref(b)))
        return b.value

    def set_timing(self, enable: bool, prefix: str = "") -> None:
        """Bracket kernel launches whose tag starts with `prefix` with HIP
        events on the plan's stream (clears the totals)."""
        self._sync_stream()
        check(self.lib.isg_plan_set_timing(self.handle, int(enable), prefix.encode()))

    def read_timing(self) -> dict:
        """{tag: (launches, total_ms)} of the launches timed so far."""
        import json
        buf = C.create_string_buffer(1 << 16)
        check(self.lib.isg_plan_read_timing(self.handle, buf, len(buf)))
        return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}

    def set_option(self, name: str, value: int) -> None:
        """Set an execution option: "spread_chunk", "phase_batch" or "graph"
        (include/isg.h, isg_option)."""
        check(self.lib.isg_plan_set_option(self.handle, _lib.OPTIONS[name], int(value)))

    def get_option(self, name: str) -> int:
        v = C.c_int64(0)
        check(self.lib.isg_plan_get_option(self.handle, _lib.OPTIONS[name], C.byref(v)))
        return v.value

    def tune(self, x, lam, motions, S, trajs, reps: int = 3) -> dict:
        """Autotune spread chunk, phase batch and graph replay on these
        inputs; keeps the fastest setting and returns the timing report."""
        import json
        x = self._image(x)
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        buf = C.create_string_buffer(1 << 16)
        self._sync_stream()
        check(self.lib.isg_plan_tune(self.handle, P, _ptr(x), dm, _ptr(S), km, float(lam), int(reps), buf, len(buf)))
        return json.loads(buf.value.decode())

    def _sync_stream(self):
        check(self.lib.isg_plan_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream))

    # -- prepared inputs ----------------------------------------------------
    def motion(self, d: torch.Tensor) -> Motion:
        self._sync_stream()
        return Motion(self, d)

    def traj(self, k: torch.Tensor) -> Traj:
        self._sync_stream()
        return Traj(self, k)

    # -- helpers ------------------------------------------------------------
    def _image(self, x, name="x"):
        return _require(x, torch.complex64, self.shape, name)

    def _empty_image(self):
        return torch.empty(self.shape, dtype=torch.complex64, device=self.device)

    def _handles(self, motions, trajs):
        P = len(motions)
        if P != len(trajs):
            raise ValueError("one trajectory per motion")
        for m in motions:
            if m.plan is not self:
                raise ValueError("motion belongs to another plan")
        for t in trajs:
            if t.plan is not self:
                raise ValueError("trajectory belongs to another plan")
        dm = (C.c_void_p * P)(*[m.handle for m in motions])
        km = (C.c_void_p * P)(*[t.handle for t in trajs])
        return P, dm, km

    def data_rows(self, trajs) -> int:
        return sum(t.M for t in trajs)

    # -- operators ----------------------------------------------------------
    def warp(self, x: torch.Tensor, motion: Motion, out: torch.Tensor | None = None) -> torch.Tensor:
        """T_d x (Eq. 9)."""
        x = self._image(x)
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_warp(self.handle, motion.handle, _ptr(x), _ptr(out)))
        return out

    def warp_adjoint(self, y: torch.Tensor, motion: Motion, out: torch.Tensor | None = None) -> torch.Tensor:
        """T_d^H y (Eq. 7-8)."""
        y = self._image(y, "y")
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_warp_adjoint(self.handle, motion.handle, _ptr(y), _ptr(out)))
        return out

    def warp_adjoint_noalloc(self, y: torch.Tensor, motion: Motion, out: torch.Tensor) -> torch.Tensor:
        """T_d^H y into a caller-supplied `out`, with the library's fixed
        device scratch instead of plan memory (allocates nothing; shapes up to
        the scratch's 64 MiB, see include/isg.h)."""
        y = self._image(y, "y")
        out = self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_warp_adjoint_noalloc(self.handle, motion.handle, _ptr(y), _ptr(out)))
        return out

    def warp_grad_d(self, x: torch.Tensor, v: torch.Tensor, motion: Motion,
                    out: torch.Tensor | None = None) -> torch.Tensor:
        """Re(conj(v) * d(T_d x)/dd), float32 [ndim][*shape]."""
        x = self._image(x)
        v = self._image(v, "v")
        if out is None:
            out = torch.empty((self.ndim,) + self.shape, dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(self.lib.isg_warp_grad_d(self.handle, motion.handle, _ptr(x), _ptr(v), _ptr(out)))
        return out

    def sense_forward(self, x, motions, S, trajs, out=None) -> torch.Tensor:
        """Stacked nonrigid SENSE model (Eq. 10); returns [sum_p M_p][C]."""
        x = self._image(x)
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        rows = self.data_rows(trajs)
        if out is None:
            out = torch.empty((rows, self.ncoils), dtype=torch.complex64, device=self.device)
        else:
            out = _require(out, torch.complex64, (rows, self.ncoils), "out")
        self._sync_stream()
        check(self.lib.isg_sense_forward(self.handle, P, _ptr(x), dm, _ptr(S), km, _ptr(out)))
        return out

    def sense_adjoint(self, y, motions, S, trajs, out=None) -> torch.Tensor:
        """sum_p A_p^H y_p (Fig. 3b)."""
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        y = _require(y, torch.complex64, (self.data_rows(trajs), self.ncoils), "y")
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_sense_adjoint(self.handle, P, _ptr(y), dm, _ptr(S), km, _ptr(out)))
        return out

    def normal(self, x, lam, motions, S, trajs, out=None) -> torch.Tensor:
        """sum_p A_p^H A_p x + lam x."""
        x = self._image(x)
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_normal(self.handle, P, _ptr(x), float(lam), dm, _ptr(S), km, _ptr(out)))
        return out

    def sense_grad(self, x, motions, S, trajs, r, want_x: bool = True, want_d: bool = True):
        """Gradients of sum_p 1/2 ||A_p x - y_p||^2 from the residual r = A x - y:
        (grad_x complex64 [*shape] or None, grad_d float32 [P][ndim][*shape] or None)."""
        x = self._image(x)
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        r = _require(r, torch.complex64, (self.data_rows(trajs), self.ncoils), "r")
        gx = self._empty_image() if want_x else None
        gd = torch.empty((P, self.ndim) + self.shape, dtype=torch.float32, device=self.device) if want_d else None
        self._sync_stream()
        check(self.lib.isg_sense_grad(self.handle, P, _ptr(x), dm, _ptr(S), km, _ptr(r),
                                      _ptr(gx) if gx is not None else None,
                                      _ptr(gd) if gd is not None else None))
        return gx, gd

    def cg_solve(self, y, motions, S, trajs, lam: float, iters: int, x0=None):
        """CG on (sum_p A_p^H A_p + lam I) x = sum_p A_p^H y_p; returns
        (x, residual norms [iters + 1])."""
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        y = _require(y, torch.complex64, (self.data_rows(trajs), self.ncoils), "y")
        x = torch.zeros(self.shape, dtype=torch.complex64, device=self.device) if x0 is None \
            else self._image(x0, "x0").clone()
        hist = (C.c_double * (iters + 1))()
        self._sync_stream()
        check(self.lib.isg_cg_solve(self.handle, P, _ptr(y), dm, _ptr(S), km, float(lam), int(iters),
                                    _ptr(x), hist))
        return x, list(hist)

    def warp_cg_solve(self, q, motion: Motion, lam: float, iters: int, p0=None):
        """CG on (T_d^H T_d + lam I) p = T_d^H q (Appendix 1, l2 form);
        returns (p, residual norms [iters + 1])."""
        q = self._image(q, "q")
        p = torch.zeros(self.shape, dtype=torch.complex64, device=self.device) if p0 is None \
            else self._image(p0, "p0").clone()
        hist = (C.c_double * (iters + 1))()
        self._sync_stream()
        check(self.lib.isg_warp_cg_solve(self.handle, motion.handle, _ptr(q), float(lam), int(iters), _ptr(p), hist))
        return p, list(hist)

    # -- sparsity-regularised reconstruction (Eq. 11, Eq. 13) ----------------
    def wavelet_forward(self, x, levels: int, out=None) -> torch.Tensor:
        """W x: orthonormal Haar, `levels` levels, Mallat layout."""
        x = self._image(x)
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_wavelet_forward(self.handle, int(levels), _ptr(x), _ptr(out)))
        return out

    def wavelet_inverse(self, w, levels: int, out=None) -> torch.Tensor:
        """W^H w."""
        w = self._image(w, "w")
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_wavelet_inverse(self.handle, int(levels), _ptr(w), _ptr(out)))
        return out

    def power_iteration(self, motions, S, trajs, iters: int, v0):
        """Largest eigenvalue of sum_p A_p^H A_p from start vector v0;
        returns (lambda_max estimate, last unit iterate)."""
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        v = self._image(v0, "v0").clone()
        lmax = C.c_double(0.0)
        self._sync_stream()
        check(self.lib.isg_power_iteration(self.handle, P, dm, _ptr(S), km, int(iters), _ptr(v), C.byref(lmax)))
        return lmax.value, v

    def warp_power_iteration(self, motion: Motion, iters: int, v0):
        """Largest eigenvalue of T_d^H T_d; returns (estimate, last unit iterate)."""
        v = self._image(v0, "v0").clone()
        lmax = C.c_double(0.0)
        self._sync_stream()
        check(self.lib.isg_warp_power_iteration(self.handle, motion.handle, int(iters), _ptr(v), C.byref(lmax)))
        return lmax.value, v

    def fista_solve(self, y, motions, S, trajs, lam: float, lipschitz: float, levels: int, iters: int, x0=None):
        """Wavelet-FISTA for ||y - A x||^2 + lam ||W x||_1 (Eq. 11); returns
        (x, [||x_k - x_{k-1}||, k = 1..iters])."""
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        P, dm, km = self._handles(motions, trajs)
        y = _require(y, torch.complex64, (self.data_rows(trajs), self.ncoils), "y")
        x = torch.zeros(self.shape, dtype=torch.complex64, device=self.device) if x0 is None \
            else self._image(x0, "x0").clone()
        hist = (C.c_double * max(iters, 1))()
        self._sync_stream()
        check(self.lib.isg_fista_solve(self.handle, P, _ptr(y), dm, _ptr(S), km, float(lam), float(lipschitz),
                                       int(levels), int(iters), _ptr(x), hist))
        return x, list(hist)[:iters]

    def warp_fista_solve(self, q, motion: Motion, lam: float, lipschitz: float, levels: int, iters: int, p0=None):
        """Wavelet-FISTA for ||q - T_d p||^2 + lam ||W p||_1 (Eq. 13)."""
        q = self._image(q, "q")
        p = torch.zeros(self.shape, dtype=torch.complex64, device=self.device) if p0 is None \
            else self._image(p0, "p0").clone()
        hist = (C.c_double * max(iters, 1))()
        self._sync_stream()
        check(self.lib.isg_warp_fista_solve(self.handle, motion.handle, _ptr(q), float(lam), float(lipschitz),
                                            int(levels), int(iters), _ptr(p), hist))
        return p, list(hist)[:iters]

    # -- registration, density compensation, gridding ------------------------
    def register(self, ref, mov, mu: float, step: float, iters: int, d0=None):
        """Gradient descent on ||T_d ref - mov||^2 + mu sum ||D_a d_i||^2;
        returns (d float32 [ndim][*shape], energies [iters + 1])."""
        ref = self._image(ref, "ref")
        mov = self._image(mov, "mov")
        d = torch.zeros((self.ndim,) + self.shape, dtype=torch.float32, device=self.device) if d0 is None \
            else _require(d0, torch.float32, (self.ndim,) + self.shape, "d0").clone()
        hist = (C.c_double * (iters + 1))()
        self._sync_stream()
        check(self.lib.isg_register(self.handle, _ptr(ref), _ptr(mov), float(mu), float(step), int(iters),
                                    _ptr(d), hist))
        return d, list(hist)

    def dcf(self, traj: Traj, iters: int) -> torch.Tensor:
        """Pipe-Menon density compensation weights, float32 [M]."""
        if traj.plan is not self:
            raise ValueError("trajectory belongs to another plan")
        w = torch.empty(traj.M, dtype=torch.float32, device=self.device)
        self._sync_stream()
        check(self.lib.isg_traj_dcf(self.handle, traj.handle, int(iters), _ptr(w)))
        return w

    def grid_recon(self, traj: Traj, y, S, w=None, out=None) -> torch.Tensor:
        """sum_c conj(S_c) G^H(w conj(ph) y_c); y complex64 [M][C]."""
        if traj.plan is not self:
            raise ValueError("trajectory belongs to another plan")
        y = _require(y, torch.complex64, (traj.M, self.ncoils), "y")
        S = _require(S, torch.complex64, (self.ncoils,) + self.shape, "S")
        if w is not None:
            w = _require(w, torch.float32, (traj.M,), "w")
        out = self._empty_image() if out is None else self._image(out, "out")
        self._sync_stream()
        check(self.lib.isg_grid_recon(self.handle, traj.handle, _ptr(y), _ptr(w) if w is not None else None,
                                      _ptr(S), _ptr(out)))
        return out
