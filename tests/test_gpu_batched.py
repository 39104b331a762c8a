"""Batched transport: many phantoms of uneven size and view count in one
persistent launch, captured in a HIP graph, with autotuned launch options.

Bar: the batched tallies, fates and energies equal the concatenation of the
per-problem runs bit for bit (integer sums, order-independent); per problem
the oracle parity bars of tests/parity.py; graph replays equal the eager
call; every autotune candidate gives identical results.
"""
import sys

import numpy as np
import pytest

import oracle
import phantoms
from parity import batch_parity

pytestmark = pytest.mark.gpu


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch(n=6, hist=200_000):
    rng = np.random.Generator(np.random.PCG64(21))
    out = []
    for p in range(n):
        g = int(rng.integers(20, 41))
        v = int(rng.integers(3, 31))
        pr = phantoms.thorax_problem(f"tb{p}", g, 38.4 / g, 1000 + p, v, 180.0, 32, 1.2, hist + 17 * p,
                                     problem_id=p)
        out.append(pr)
    return out


def outputs(sim):
    return (sim.tally.cpu().numpy().copy(), sim.fates.cpu().numpy().copy(),
            sim.energy.cpu().numpy().copy(), sim.counters.cpu().numpy().copy())


def test_batched_equals_individual_bit_exact():
    mc = _mc()
    probs = small_batch()
    dps = [mc.to_device(p) for p in probs]
    batch = mc.simulate(dps)
    t, f, e, c = outputs(batch)
    off = 0
    for i, dp in enumerate(dps):
        one = mc.simulate(dp)
        t1, f1, e1, c1 = outputs(one)
        np.testing.assert_array_equal(t[off:off + t1.size], t1)
        np.testing.assert_array_equal(f[i], f1[0])
        np.testing.assert_array_equal(e[i], e1[0])
        np.testing.assert_array_equal(c[i], c1[0])
        off += t1.size
    assert off == t.size


def test_batched_matches_oracle_per_problem():
    mc = _mc()
    probs = small_batch()
    dps = [mc.to_device(p) for p in probs]
    sim = mc.simulate(dps, event_capacity=1 << 14)
    batch_parity(probs, dps, sim)


def test_graph_replay_matches_eager():
    mc = _mc()
    import torch
    probs = small_batch(4, 100_000)
    dps = [mc.to_device(p) for p in probs]
    ref = outputs(mc.simulate(dps))
    sim = mc.Simulator(dps)
    runner = mc.GraphRunner(sim)
    for k in range(3):
        sim.tally.fill_(-1)               # stale values must be overwritten by the graph
        runner.replay()
        torch.cuda.synchronize()
        got = outputs(sim)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        # eager work in between replays
        other = mc.simulate(dps[:2])
        assert int(other.fates.sum().item()) == sum(p.n_histories for p in probs[:2])


def test_autotune_candidates_identical():
    mc = _mc()
    probs = small_batch(3, 150_000)
    dps = [mc.to_device(p) for p in probs]
    ref = outputs(mc.simulate(dps))
    for b in (0, 2, 3):
        for h in (1, 4, 64):
            got = outputs(mc.simulate(dps, options={"brick_log2": b, "hist_per_lane": h}))
            for x, y in zip(got, ref):
                np.testing.assert_array_equal(x, y)
    best = mc.autotune(dps, reps=1)
    assert best["brick_log2"] in (0, 2, 3) and best["hist_per_lane"] in (4, 16, 64)


def test_batched_full_size_parity():
    """The batched workload at full size (32 thoraxes, 96^3-160^3, 30-120
    views, 1e7 histories each) in the launch the benchmark times (graph,
    autotuned options), every problem against its own full oracle run:
    tallies explained bin by bin by the histories tallied on one side only
    (the batched kernel's own event list), fates against a replay of all
    3.2e8 histories on both sides; four problems also equal their
    single-problem runs bit for bit."""
    mc = _mc()
    import torch
    probs = phantoms.batched_thoraxes(10 ** 7)
    dps = [mc.to_device(p) for p in probs]
    opts = mc.autotune(dps, reps=1)
    sim = mc.Simulator(dps, options=opts, event_capacity=1 << 17)
    runner = mc.GraphRunner(sim)
    runner.replay()
    torch.cuda.synchronize()
    st = sim.check_status()
    assert st[0] == 0
    f = sim.fates.cpu().numpy()
    t = sim.tally.cpu().numpy()
    off = 0
    for i, (p, dp) in enumerate(zip(probs, dps)):
        size = int(np.prod(p.tally_shape))
        if i in (0, 7, 19, 31):
            one = mc.simulate(dp)
            np.testing.assert_array_equal(t[off:off + size], one.tally.cpu().numpy())
            np.testing.assert_array_equal(f[i], one.fates.cpu().numpy()[0])
        off += size
    say(f"batched full size: {len(probs)} problems, options {opts}")
    errs = batch_parity(probs, dps, sim)
    worst = {k: max(e[k] for e in errs) for k in ("window_total_rel", "primary_rel", "scatter_rel",
                                                    "fates_max_rel", "energy_max_rel")}
    say(f"batched per-result errors (worst problem): {worst}; replay identical "
        f"{min(e['replay_identical_all'] for e in errs):.7f} (worst problem)")
