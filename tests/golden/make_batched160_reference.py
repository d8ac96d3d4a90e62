"""Writes batched160.json: FP64 oracle values for the benchmarked workload
(160^3 image, 12 coils, 6 respiratory states with 80k..600k radial samples,
lambda = 1e-3), used by tests/test_gpu_batched160.py and by bench.py to state
each timed form's error against FP64.

* forward: (A_p x)[j][c] = G_p(S_c . T_p x)_j (Eq. 10) for every state p at
  256 seeded sample indices j, all 12 coils, x the workload's phantom;
* normal: (sum_p A_p^H A_p x + lambda x)[v] (l2 form of Eq. 11) at 4096 seeded
  voxels v;
* adjoint: (sum_p A_p^H y_p)[v] (Fig. 3b) at the same voxels for the seeded
  complex noise y of synth (all states packed, [sum_p M_p][C]).

It calls only oracle/ and synth/.  The states run in parallel worker
processes (about 4 GB of memory each); with 3 workers on 8 cores it takes
about an hour:

    python tests/golden/make_batched160_reference.py [--workers 3]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched160.json")
N_SAMPLES, N_VOXELS = 256, 4096
CFG = 3


def selections(Ms, N: int):
    """seeded sample subsets (one per state) and voxel subset (shared with
    the test and the benchmark)"""
    g = rng(CFG, P_MISC, 7)
    js = [np.sort(g.choice(M, N_SAMPLES, replace=False)) for M in Ms]
    v = np.sort(g.choice(N, N_VOXELS, replace=False))
    return js, v


def adjoint_data(Mtot: int, C: int) -> np.ndarray:
    """the seeded y of the adjoint check, [sum_p M_p][C] complex64"""
    return complex_noise((Mtot, C), rng(CFG, P_MISC, 8))


def _state(p):
    """state p's share: sampled A_p x, A_p^H A_p x and A_p^H y_p"""
    t0 = time.time()
    w = WORKLOADS["batched_160"]
    inp = make_inputs(w)
    x = inp["x"].astype(np.complex128)
    S, ks, shape = inp["S"], inp["k"], w.shape
    Ms = [k.shape[0] for k in ks]
    js, _ = selections(Ms, int(np.prod(shape)))
    off = int(np.sum(Ms[:p]))
    y = adjoint_data(int(np.sum(Ms)), w.ncoils)[off:off + Ms[p]]
    d, k = inp["d"][p], ks[p]
    ya = oracle.sense.coil_forward(oracle.warp.warp(x, d), S, k)  # [C][M_p]
    fwd = ya[:, js[p]].T.copy()                                    # [256][C]
    print(f"  state {p}: forward {time.time() - t0:.0f}s", flush=True)
    nrm = oracle.warp.warp_adjoint(oracle.sense.coil_adjoint(ya, S, k, shape), d)
    del ya
    print(f"  state {p}: A^H A x {time.time() - t0:.0f}s", flush=True)
    adj = oracle.warp.warp_adjoint(oracle.sense.coil_adjoint(y.T, S, k, shape), d)
    print(f"  state {p}: A^H y {time.time() - t0:.0f}s", flush=True)
    return p, fwd, nrm, adj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=3)
    args = ap.parse_args()
    w = WORKLOADS["batched_160"]
    t0 = time.time()
    inp = make_inputs(w)
    x = inp["x"].astype(np.complex128)
    Ms = [k.shape[0] for k in inp["k"]]
    js, vs = selections(Ms, int(np.prod(w.shape)))
    nrm = w.lam * x
    adj = np.zeros(w.shape, dtype=np.complex128)
    fwd = [None] * w.nphases
    with get_context("spawn").Pool(args.workers) as pool:
        for p, f, n, a in pool.imap_unordered(_state, range(w.nphases)):
            fwd[p] = f
            nrm = nrm + n
            adj = adj + a
            print(f"state {p} done {time.time() - t0:.0f}s", flush=True)
    rec = {
        "workload": w.name,
        "lambda": w.lam,
        "note": "FP64 oracle values written by tests/golden/make_batched160_reference.py",
        "sample_indices": [j.tolist() for j in js],
        "forward": [[[[float(z.real), float(z.imag)] for z in row] for row in f] for f in fwd],
        "voxels": vs.tolist(),
        "normal": [[float(z.real), float(z.imag)] for z in nrm.reshape(-1)[vs]],
        "adjoint": [[float(z.real), float(z.imag)] for z in adj.reshape(-1)[vs]],
        "norms": {"normal_full": float(np.linalg.norm(nrm)), "adjoint_full": float(np.linalg.norm(adj))},
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
