"""The benchmarked workload (160^3 image, 12 coils, 6 respiratory states with
80k..600k radial samples, lambda = 1e-3) against stored FP64 oracle values
(tests/golden/batched160.json, written by
tests/golden/make_batched160_reference.py from oracle/ and synth/ only):

* forward A_p x at 256 seeded samples of every state, all 12 coils (Eq. 10);
* the normal operator sum_p A_p^H A_p x + lambda x at 4096 seeded voxels
  (l2 form of Eq. 11);
* the adjoint sum_p A_p^H y_p at the same voxels for seeded complex noise y
  (Fig. 3b).

Each is checked with the options bench.py times for its headline form (row
blocking 2, k-space tile extent 4, spread chunk 1024, all 6 states per
k-space launch, graph replay) and with the plain options (no blocking, tile
extent 8, chunk 512, one state per launch, no graph): 1e-5 relative L2 for
FP32 grids, 1e-3 for FP16 and BF16 grids (one rounding per direction), the
error printed per result."""
import json
import os
import sys

import numpy as np
import pytest

from synth import WORKLOADS, make_inputs

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_batched160_reference as ref_script  # noqa: E402  (seeded selections and data only)

TUNED = {"kblock": 2, "ktile_t1": 4, "spread_chunk": 1024, "phase_batch": 6, "graph": 1}
PLAIN = {"kblock": 0, "ktile_t1": 8, "spread_chunk": 512, "phase_batch": 1, "graph": 0}
BARS = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 1e-3}


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "batched160.json")) as f:
        rec = json.load(f)
    w = WORKLOADS["batched_160"]
    say("batched_160 inputs")
    inp = make_inputs(w)
    Ms = [k.shape[0] for k in inp["k"]]
    js, vs = ref_script.selections(Ms, int(np.prod(w.shape)))
    assert [j.tolist() for j in js] == rec["sample_indices"] and vs.tolist() == rec["voxels"]
    cplx = np.array([1.0, 1j])
    fwd = [np.array(f) @ cplx for f in rec["forward"]]     # per state [256][C]
    nrm = np.array(rec["normal"]) @ cplx                    # [4096]
    adj = np.array(rec["adjoint"]) @ cplx
    y = ref_script.adjoint_data(int(np.sum(Ms)), w.ncoils)
    return w, inp, js, vs, fwd, nrm, adj, y


def _err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("storage,opts", [("fp32", "tuned"), ("fp32", "plain"), ("fp16", "tuned"),
                                          ("bf16", "tuned")])
def test_batched160_against_fp64(golden, storage, opts):
    import torch
    import paper_2501_16713_amd as isg
    w, inp, js, vs, fwd, nrm, adj, y = golden
    say(f"batched_160 {storage} grids, {opts} options")
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases, storage=storage)
    for k, v in (TUNED if opts == "tuned" else PLAIN).items():
        plan.set_option(k, v)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    x = to_dev(inp["x"])
    # forward, every state, sampled
    yf = plan.sense_forward(x, mots, S, trs)
    off, ef = 0, []
    for p, k in enumerate(inp["k"]):
        idx = torch.from_numpy(js[p] + off).to(yf.device)
        ef.append(_err(yf[idx].cpu().numpy(), fwd[p]))
        off += k.shape[0]
    del yf
    # normal operator (twice: the second call replays the captured graph)
    vi = torch.from_numpy(vs).to(x.device)
    out = torch.empty_like(x)
    plan.normal(x, w.lam, mots, S, trs, out=out)
    en1 = _err(out.reshape(-1)[vi].cpu().numpy(), nrm)
    plan.normal(x, w.lam, mots, S, trs, out=out)
    en2 = _err(out.reshape(-1)[vi].cpu().numpy(), nrm)
    # adjoint of seeded noise
    xa = plan.sense_adjoint(to_dev(y), mots, S, trs)
    ea = _err(xa.reshape(-1)[vi].cpu().numpy(), adj)
    say(f"  A per state {' '.join(f'{e:.1e}' for e in ef)}; N {en1:.2e} / {en2:.2e} (replay); A^H {ea:.2e}")
    for m in mots + trs:
        m.close()
    plan.close()
    del S, x, out, xa
    torch.cuda.empty_cache()
    bar = BARS[storage]
    assert max(ef) < bar and en1 < bar and en2 < bar and ea < bar
