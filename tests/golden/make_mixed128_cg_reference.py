"""Writes mixed128_cg.json: an FP64 oracle conjugate-gradient solve on the
128^3, 16-coil, 8-state workload (the 256^3 mixed-precision workload at a
size whose 30-iteration FP64 solve finishes in hours), used by
tests/test_gpu_mixed128.py to state the error of the FP32, FP16 and BF16
grid forms of the GPU solve against FP64.

Problem: (sum_p A_p^H A_p + lambda I) x = sum_p A_p^H y_p (l2 form of Eq. 11),
x0 = 0, 30 Hestenes-Stiefel iterations (oracle.cg), with y the seeded complex
noise of synth (all states packed, [sum_p M_p][C]).  lambda = 1e-3 (the
workload's; CG does not converge in 30 iterations there, a stress case) is
written to mixed128_cg.json, lambda = 0.5 (--lam 0.5) to
mixed128_cg_lam0.5.json.  Stored: the residual norms ||r_0|| .. ||r_30||, the
iterate x_30 at 4096 seeded voxels and its norm, and sum_p A_p^H y_p at the
same voxels.

It calls only oracle/ and synth/; the states of every normal-operator
application run in parallel worker processes (one per state, single-threaded
FFTs, about 2 GB each):

    python tests/golden/make_mixed128_cg_reference.py [--workers 8] [--lam 0.5]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import P_MISC, WORKLOADS, complex_noise, make_inputs, rng  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed128_cg.json")
N_VOXELS = 4096
W = WORKLOADS["mixed_128"]


def selections(N: int):
    """seeded voxel subset (shared with the test)"""
    return np.sort(rng(W.cfg, P_MISC, 7).choice(N, N_VOXELS, replace=False))


def data(Mtot: int, C: int) -> np.ndarray:
    """the seeded y of the solve, [sum_p M_p][C] complex64"""
    return complex_noise((Mtot, C), rng(W.cfg, P_MISC, 8))


_inp = None


def _init():
    global _inp
    oracle.kspace.WORKERS = 1  # one process per state: single-threaded FFTs
    oracle.warp.WORKERS = 1
    _inp = make_inputs(W)


def _adjoint(p):
    """A_p^H y_p"""
    ks = _inp["k"]
    Ms = [k.shape[0] for k in ks]
    off = int(np.sum(Ms[:p]))
    y = data(int(np.sum(Ms)), W.ncoils)[off:off + Ms[p]]
    return oracle.warp.warp_adjoint(oracle.sense.coil_adjoint(y.T, _inp["S"], ks[p], W.shape), _inp["d"][p])


def _normal_state(args):
    """A_p^H A_p v"""
    p, v = args
    S, d, k = _inp["S"], _inp["d"][p], _inp["k"][p]
    ya = oracle.sense.coil_forward(oracle.warp.warp(v, d), S, k)
    return oracle.warp.warp_adjoint(oracle.sense.coil_adjoint(ya, S, k, W.shape), d)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--lam", type=float, default=W.lam)
    args = ap.parse_args()
    lam = args.lam
    out_path = OUT if lam == W.lam else OUT.replace(".json", f"_lam{lam:g}.json")
    t0 = time.time()
    vs = selections(int(np.prod(W.shape)))
    with get_context("spawn").Pool(args.workers, initializer=_init) as pool:
        b = np.zeros(W.shape, dtype=np.complex128)
        for a in pool.map(_adjoint, range(W.nphases)):
            b = b + a
        print(f"b = A^H y {time.time() - t0:.0f}s", flush=True)
        count = [0]

        def normal(v):
            out = lam * v
            for a in pool.map(_normal_state, [(p, v) for p in range(W.nphases)]):
                out = out + a
            count[0] += 1
            print(f"  normal operator {count[0]} {time.time() - t0:.0f}s", flush=True)
            return out

        x, hist = oracle.cg.cg(normal, b, W.cg_iters)
    rec = {
        "workload": W.name,
        "lambda": lam,
        "iters": W.cg_iters,
        "note": "FP64 oracle CG written by tests/golden/make_mixed128_cg_reference.py",
        "voxels": vs.tolist(),
        "resnorm": [float(h) for h in hist],
        "x_final": [[float(z.real), float(z.imag)] for z in x.reshape(-1)[vs]],
        "b": [[float(z.real), float(z.imag)] for z in b.reshape(-1)[vs]],
        "norms": {"x_final": float(np.linalg.norm(x)), "b": float(np.linalg.norm(b))},
    }
    with open(out_path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {out_path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
