"""Batched execution: the k-space gather and spread of several states in one
launch, graph replay of the normal operator, the spread chunk size and the
autotuner that picks among them.  None of these may change a result beyond
floating-point summation order:

* phase batching runs every state's work exactly as the unbatched launch
  does, so results are compared bit for bit;
* graph replays re-run the captured kernels, so they are compared bit for
  bit with the eager call, replay after replay, with eager work between;
* the row-blocked layout of the internal k-space arrays and the addressing
  form of the FFT passes change addresses only, so results are compared bit
  for bit;
* a different spread chunk or k-space tile extent changes only the order in
  which contributions are summed: 1e-6 relative (a few FP32 roundings), and
  the result is still held to the oracle's 1e-5.
"""
import numpy as np
import pytest

import oracle
from synth import make_inputs, small_workload

from gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    import paper_2501_16713_amd as isg
    # uneven per-state sample counts; 36 x 40 x 48 gives ragged spread tiles
    w = small_workload(shape=(36, 40, 48), ncoils=5, nphases=3, spokes=(30, 90, 55), cfg=140)
    inp = make_inputs(w)
    return isg, w, inp


def _plan(isg, w, inp, stream=None):
    import torch
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    return plan, S, mots, trs


def test_phase_batch_is_bit_exact(setup):
    import torch
    isg, w, inp = setup
    plan, S, mots, trs = _plan(isg, w, inp)
    x = to_dev(inp["x"])
    M = sum(k.shape[0] for k in inp["k"])
    y = to_dev((np.random.default_rng(3).standard_normal((M, w.ncoils, 2)) @ [1, 1j]).astype(np.complex64))
    ref = {}
    for b in (1, 2, 3):
        say(f"phase batch {b}")
        plan.set_option("phase_batch", b)
        assert plan.get_option("phase_batch") == b
        res = (plan.sense_forward(x, mots, S, trs), plan.sense_adjoint(y, mots, S, trs),
               plan.normal(x, 0.3, mots, S, trs))
        torch.cuda.synchronize()
        if b == 1:
            ref = [r.clone() for r in res]
        else:
            for a, r in zip(res, ref):
                assert torch.equal(a, r)


def test_graph_replay_is_bit_exact(setup):
    import torch
    isg, w, inp = setup
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan, S, mots, trs = _plan(isg, w, inp)
        x = to_dev(inp["x"])
        x2 = to_dev(inp["x"][::-1].copy())
        eager = plan.normal(x, 0.1, mots, S, trs).clone()
        eager2 = plan.normal(x2, 0.1, mots, S, trs).clone()
        plan.set_option("graph", 1)
        out = torch.empty_like(x)
        for rep in range(4):
            say(f"graph replay {rep}")
            plan.normal(x, 0.1, mots, S, trs, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, eager)
            # eager work of the program between replays
            z = (x * 2).sum()
            torch.cuda.synchronize()
        # new arguments: a new capture, still exact
        plan.normal(x2, 0.1, mots, S, trs, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, eager2)
        # a destroyed and re-created trajectory must not replay a stale graph
        trs[1].close()
        trs[1] = plan.traj(to_dev(inp["k"][1]))
        plan.normal(x2, 0.1, mots, S, trs, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, eager2)
        del z


def test_spread_chunk_and_oracle(setup):
    import torch
    isg, w, inp = setup
    M = sum(k.shape[0] for k in inp["k"])
    y = (np.random.default_rng(4).standard_normal((M, w.ncoils, 2)) @ [1, 1j]).astype(np.complex64)
    outs = {}
    for chunk in (32, 512):
        say(f"spread chunk {chunk}")
        plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
        plan.set_option("spread_chunk", chunk)
        S = to_dev(inp["S"])
        mots = [plan.motion(to_dev(d)) for d in inp["d"]]
        trs = [plan.traj(to_dev(k)) for k in inp["k"]]
        outs[chunk] = plan.sense_adjoint(to_dev(y), mots, S, trs).cpu().numpy()
    assert rel(outs[32], outs[512]) < 1e-6
    ys, off = [], 0
    for k in inp["k"]:
        ys.append(y[off:off + k.shape[0]].T)
        off += k.shape[0]
    ref = oracle.sense.sense_adjoint(ys, inp["d"], inp["S"], inp["k"], w.shape)
    assert rel(outs[32], ref) < 1e-5


def test_tune_keeps_results(setup):
    import torch
    isg, w, inp = setup
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan, S, mots, trs = _plan(isg, w, inp)
        x = to_dev(inp["x"])
        before = plan.normal(x, 0.2, mots, S, trs).cpu().numpy()
        say("tune")
        rep = plan.tune(x, 0.2, mots, S, trs, reps=2)
        chosen = rep["chosen"]
        assert chosen["chunk"] == plan.get_option("spread_chunk")
        assert chosen["batch"] == plan.get_option("phase_batch")
        assert chosen["graph"] == plan.get_option("graph")
        assert len(rep["candidates"]) >= 5
        after = plan.normal(x, 0.2, mots, S, trs).cpu().numpy()
        after2 = plan.normal(x, 0.2, mots, S, trs).cpu().numpy()
    assert rel(after, before) < 1e-6
    assert np.array_equal(after, after2)


def test_ktile_extent(setup):
    """narrower k-space spread tiles: same operator (summation order only),
    and trajectories binned for another tile shape are refused.  32 x 40 x 48
    takes the register-FFT path whose axis-0 passes skip untouched tiles."""
    import torch
    isg = setup[0]
    w = small_workload(shape=(32, 40, 48), ncoils=6, nphases=2, spokes=(25, 70), cfg=141)
    inp = make_inputs(w)
    x = to_dev(inp["x"])
    res = {}
    for t1 in (8, 4):
        say(f"k-space tile extent {t1}")
        plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
        plan.set_option("ktile_t1", t1)
        assert plan.get_option("ktile_t1") == t1
        S = to_dev(inp["S"])
        mots = [plan.motion(to_dev(d)) for d in inp["d"]]
        trs = [plan.traj(to_dev(k)) for k in inp["k"]]
        res[t1] = plan.normal(x, 0.1, mots, S, trs).cpu().numpy()
        if t1 == 4:
            plan.set_option("ktile_t1", 8)
            with pytest.raises(isg.IsgError):
                plan.normal(x, 0.1, mots, S, trs)
    assert rel(res[4], res[8]) < 1e-6
    want = oracle.sense.normal(inp["x"], 0.1, inp["d"], inp["S"], inp["k"])
    assert rel(res[4], want) < 1e-5


def test_touched_runs_and_columns(setup):
    """the bookkeeping behind the axis-0 passes' tile skipping and their
    algorithmic bytes, bit-exact against the taps the oracle's interpolation
    uses (W = 4 per axis around G k): the grid cells in touched 8-cell runs
    along axis 0 (the k-space tile extent there) and the grid columns (i1, i2)
    holding at least one such run"""
    isg = setup[0]
    w = small_workload(shape=(32, 40, 48), ncoils=2, nphases=2, spokes=(25, 70), cfg=143)
    inp = make_inputs(w)
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases)
    G = tuple(2 * n for n in w.shape)
    for k in inp["k"]:
        say(f"touched runs, {k.shape[0]} samples")
        info = plan.traj(to_dev(k)).info()
        kap = oracle.kspace.grid_coords(k, G)
        idx = [oracle.grid.taps_1d(kap[:, a], G[a])[0] for a in range(3)]
        runs = np.zeros((G[1], G[2], G[0] // 8), dtype=bool)
        for t0 in range(4):
            for t1 in range(4):
                for t2 in range(4):
                    runs[idx[1][t1], idx[2][t2], idx[0][t0] // 8] = True
        assert info["touched_cells"] == 8 * int(runs.sum())
        assert info["active_columns"] == int(runs.any(axis=2).sum())
        assert 0 < info["active_columns"] < G[1] * G[2]


def test_kspace_blocking_is_bit_exact(setup):
    """row-blocked internal k-space arrays (32 x 40 x 48: register-FFT path)"""
    import torch
    isg = setup[0]
    w = small_workload(shape=(32, 40, 48), ncoils=6, nphases=2, spokes=(25, 70), cfg=142)
    inp = make_inputs(w)
    x = to_dev(inp["x"])
    M = sum(k.shape[0] for k in inp["k"])
    y = to_dev((np.random.default_rng(6).standard_normal((M, w.ncoils, 2)) @ [1, 1j]).astype(np.complex64))
    plan, S, mots, trs = _plan(isg, w, inp)
    ref = None
    for kb in (0, 3, 2, 1, 4):
        say(f"k-space blocking {kb}")
        plan.set_option("kblock", kb)
        assert plan.get_option("kblock") == kb
        res = (plan.sense_forward(x, mots, S, trs), plan.sense_adjoint(y, mots, S, trs),
               plan.normal(x, 0.3, mots, S, trs))
        torch.cuda.synchronize()
        if ref is None:
            ref = [r.clone() for r in res]
            want = oracle.sense.normal(inp["x"], 0.3, inp["d"], inp["S"], inp["k"])
            assert rel(res[2].cpu().numpy(), want) < 1e-5
        else:
            for a, r in zip(res, ref):
                assert torch.equal(a, r)


@pytest.mark.parametrize("shape,storage,kblocks", [
    ((16, 32, 48), "fp32", (0, 1, 2)),  # every length has a buffer-addressed form (G = 32, 64, 96)
    ((32, 48, 64), "fp16", (2, 3)),   # half-precision grids; blocks of 8 rows fail 8 | 12 on axis 1
    ((20, 24, 16), "fp32", (2,)),     # G = 40, 48 have none, G = 32 has: mixed passes
    ((48, 40), "bf16", (0,)),         # 2D
])
def test_fft_addressing_is_bit_exact(setup, shape, storage, kblocks):
    """the buffer-addressed FFT passes (a scalar base per tile and element
    index, one 32-bit lane offset, masking by the out-of-range rule) against
    per-lane 64-bit addressing: the same arithmetic, so the same bits"""
    import torch
    isg = setup[0]
    w = small_workload(shape=shape, ncoils=3, nphases=2, spokes=(30, 60), cfg=143)
    inp = make_inputs(w)
    x = to_dev(inp["x"])
    M = sum(k.shape[0] for k in inp["k"])
    y = to_dev((np.random.default_rng(7).standard_normal((M, w.ncoils, 2)) @ [1, 1j]).astype(np.complex64))
    plan = isg.Plan(w.shape, ncoils=w.ncoils, nphases=w.nphases, storage=storage)
    S = to_dev(inp["S"])
    mots = [plan.motion(to_dev(d)) for d in inp["d"]]
    trs = [plan.traj(to_dev(k)) for k in inp["k"]]
    assert plan.get_option("fft_addr") == 1
    for kb in kblocks:
        if len(shape) == 3:
            plan.set_option("kblock", kb)
        res = {}
        for fa in (1, 0):
            say(f"{shape} {storage} kblock {kb} fft_addr {fa}")
            plan.set_option("fft_addr", fa)
            res[fa] = (plan.sense_forward(x, mots, S, trs), plan.sense_adjoint(y, mots, S, trs),
                       plan.normal(x, 0.3, mots, S, trs), plan.warp(x, mots[0]), plan.warp_adjoint(x, mots[1]))
            torch.cuda.synchronize()
        for a, b in zip(res[1], res[0]):
            assert torch.equal(a, b)
    if storage == "fp32":
        want = oracle.sense.normal(inp["x"], 0.3, inp["d"], inp["S"], inp["k"])
        plan.set_option("fft_addr", 1)
        assert rel(plan.normal(x, 0.3, mots, S, trs).cpu().numpy(), want) < 1e-5
