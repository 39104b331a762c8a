"""Batched transport: many phantoms of uneven size and view count in one
persistent launch, captured in a HIP graph, with autotuned launch options.

Bar: the batched tallies, fates and energies equal the concatenation of the
per-problem runs bit for bit (integer sums, order-independent); per problem
the oracle parity bar of the forward tests; graph replays equal the eager
call; every autotune candidate gives identical results.
"""
import sys

import numpy as np
import pytest

import oracle
import phantoms

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
    sim = mc.simulate([mc.to_device(p) for p in probs])
    f = sim.fates.cpu().numpy()
    for i, p in enumerate(probs):
        o = oracle.simulate(p)
        assert f[i].sum() == p.n_histories
        assert np.all(np.abs(f[i] - o["fates"]) <= 1e-4 * p.n_histories + 1), (i, f[i], o["fates"])


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


def test_batched_full_size_sampled():
    """The batched workload at full size (32 thoraxes, 96^3-160^3, 30-120
    views, 1e7 histories each) in the launch the benchmark times (graph,
    autotuned options), checked on 1000 replayed histories per problem and by
    bit-exact equality with single-problem runs of four of them."""
    mc = _mc()
    import torch
    probs = phantoms.batched_thoraxes(10 ** 7)
    dps = [mc.to_device(p) for p in probs]
    opts = mc.autotune(dps, reps=1)
    sim = mc.Simulator(dps, options=opts)
    runner = mc.GraphRunner(sim)
    runner.replay()
    torch.cuda.synchronize()
    st = sim.check_status()
    assert st[0] == 0
    f = sim.fates.cpu().numpy()
    for i, p in enumerate(probs):
        assert f[i].sum() == p.n_histories
    t = sim.tally.cpu().numpy()
    off = 0
    for i, (p, dp) in enumerate(zip(probs, dps)):
        size = int(np.prod(p.tally_shape))
        if i in (0, 7, 19, 31):
            one = mc.simulate(dp)
            np.testing.assert_array_equal(t[off:off + size], one.tally.cpu().numpy())
            np.testing.assert_array_equal(f[i], one.fates.cpu().numpy()[0])
        off += size
    rng = np.random.Generator(np.random.PCG64(7))
    same_all = []
    for i, (p, dp) in enumerate(zip(probs, dps)):
        g = np.sort(rng.choice(p.n_histories, size=1000, replace=False))
        q, r = divmod(p.n_histories, p.n_views)
        big = q + 1
        view = np.where(g < r * big, g // big, r + (g - r * big) // q).astype(np.int32)
        hist = np.where(g < r * big, g % big, (g - r * big) % q).astype(np.uint64)
        a = mc.replay(dp, view, hist)
        b = oracle.replay(p, view, hist)
        same_all.append((a["fate"] == b["fate"]) & (a["iu"] == b["iu"]) & (a["iv"] == b["iv"])
                        & (a["n_scatter"] == b["n_scatter"]))
    frac = np.concatenate(same_all).mean()
    say(f"batched full size: {len(probs)} problems, replay identical {frac:.6f}, options {opts}")
    assert frac >= 0.999
