"""MI355X-native image-space gridding and nonrigid SENSE.

Operators of "Image-Space Gridding for Nonrigid Motion-Corrected MR Image
Reconstruction" (arXiv:2501.16713): the warp T_d and its adjoint (Eq. 7-9),
the nonrigid SENSE operator A_p = G_p S T_p (Eq. 10) and its adjoint, the l2
normal operator of Eq. 11, and CG on it, all computed by hand-written HIP
kernels for gfx950 behind the C ABI in include/isg.h.
"""
from ._lib import IsgError, STORAGE  # noqa: F401

__all__ = ["Plan", "Motion", "Traj", "IsgError", "device_count", "version"]


def __getattr__(name):
    # importing the operators needs torch; keep `import paper_2501_16713_amd`
    # cheap for the build step
    if name in ("Plan", "Motion", "Traj", "device_count", "version"):
        from . import ops
        return getattr(ops, name)
    if name in ("autograd",):
        import importlib
        return importlib.import_module(".autograd", __name__)
    raise AttributeError(name)
