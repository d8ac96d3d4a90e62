"""Writes mixed256_state0.json: FP64 oracle values for the 256^3, 16-coil,
8-state workload (state 0 only), used by tests/test_gpu_scale.py.

* forward: (A_0 x)[j][c] = G_0(S_c . T_0 x)_j (Eq. 10) at 512 seeded sample
  indices j of state 0, all 16 coils;
* adjoint: (A_0^H y)[v] = T_0^H sum_c conj(S_c) . G_0^H y_c (Fig. 3b) at 4096
  seeded voxels v, for the seeded complex noise y of synth.

It calls only oracle/ and synth/ (about 20-40 minutes on one CPU core, about
10 GB of memory):

    python tests/golden/make_mixed256_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import P_MISC, WORKLOADS, complex_noise, make_inputs, rng  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed256_state0.json")
N_SAMPLES, N_VOXELS = 512, 4096


def selections(M: int, N: int):
    """seeded sample and voxel subsets (shared with the test)"""
    g = rng(5, P_MISC, 7)
    j = np.sort(g.choice(M, N_SAMPLES, replace=False))
    v = np.sort(g.choice(N, N_VOXELS, replace=False))
    return j, v


def adjoint_data(M: int, C: int) -> np.ndarray:
    """the seeded y of the adjoint check, [M][C] complex64"""
    return complex_noise((M, C), rng(5, P_MISC, 8))


def main():
    w = WORKLOADS["mixed_256"]
    t0 = time.time()
    inp = make_inputs(w)
    x = inp["x"].astype(np.complex128)
    d0, k0, S = inp["d"][0], inp["k"][0], inp["S"]
    M, C, shape = k0.shape[0], w.ncoils, w.shape
    js, vs = selections(M, int(np.prod(shape)))
    print(f"inputs {time.time() - t0:.0f}s", flush=True)

    m = oracle.warp.warp(x, d0)
    print(f"warp {time.time() - t0:.0f}s", flush=True)
    yf = oracle.sense.coil_forward(m, S, k0[js])  # [C][512]
    print(f"forward {time.time() - t0:.0f}s", flush=True)
    del m

    y = adjoint_data(M, C)
    v = np.zeros(shape, dtype=np.complex128)
    for c in range(C):
        v += np.conj(S[c].astype(np.complex128)) * oracle.kspace.nufft_adjoint(y[:, c], k0, shape)
        print(f"  adjoint coil {c} {time.time() - t0:.0f}s", flush=True)
    xa = oracle.warp.warp_adjoint(v, d0)
    print(f"adjoint {time.time() - t0:.0f}s", flush=True)

    rec = {
        "workload": w.name,
        "state": 0,
        "note": "FP64 oracle values written by tests/golden/make_mixed256_reference.py",
        "sample_indices": js.tolist(),
        "forward": [[[float(z.real), float(z.imag)] for z in yf[:, i]] for i in range(len(js))],
        "voxels": vs.tolist(),
        "adjoint": [[float(z.real), float(z.imag)] for z in xa.reshape(-1)[vs]],
        "norms": {"forward_sampled": float(np.linalg.norm(yf)), "adjoint_full": float(np.linalg.norm(xa))},
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
