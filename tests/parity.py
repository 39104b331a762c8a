"""Shared parity checks of the GPU library against the FP64 oracle.

Per history (identical fate, detector bin and scatter count for at least
99.9 % of replayed histories): FP32 tracking against FP64 can flip a decision
that sits within rounding of a boundary, and the event-keyed random stream
confines such a flip to its own history.

Aggregates: every difference between the GPU's aggregate and the oracle's must
be accounted for by histories that are identified one by one as having a
different outcome on the two sides ("flipped"), and no aggregate may differ by
more than 1e-4 of itself plus its flipped histories:
  * tallies: the transport kernel's own event list (one entry per tallied
    history: work index and bin) against the oracle's list of tallied
    histories; the GPU tally minus the oracle tally must equal, bin by bin, the
    GPU-only entries minus the oracle-only entries;
  * fates: every history of the run is replayed on both sides, and the
    transport kernel's fate counts must equal the replay's exactly.
The relative error of each aggregate is printed (and is what the benchmark
reports per result).
"""
from __future__ import annotations

import sys

import numpy as np

import oracle


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ids_of_work(prob, g):
    """Problem-local work indices -> (view, history id): N_k = floor(N/V) +
    [k < N mod V] histories in view k, view-major."""
    g = np.asarray(g, dtype=np.int64)
    q, r = divmod(prob.n_histories, prob.n_views)
    big = q + 1
    view = np.where(g < r * big, g // big, r + (g - r * big) // max(q, 1))
    hist = np.where(g < r * big, g % big, (g - r * big) % max(q, 1))
    return view.astype(np.int32), hist.astype(np.uint64)


def sample_ids(prob, n, seed=7):
    """n seeded (view, history id) pairs spread over the problem's histories
    (numpy PCG64(seed), without replacement, in work order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.sort(rng.choice(prob.n_histories, size=min(n, prob.n_histories), replace=False))
    return ids_of_work(prob, g)


def same_outcome(g, o):
    return ((g["fate"] == o["fate"]) & (g["iu"] == o["iu"]) & (g["iv"] == o["iv"])
            & (g["n_scatter"] == o["n_scatter"]))


def replay_parity(prob, n=100_000, seed=7, dp=None, options=None):
    """Replay n sampled histories on both sides; >= 99.9 % identical (fate,
    bin, scatter count), emission voxels identical, final energy within 1e-5
    relative where the outcome is identical."""
    mc = _mc()
    views, hists = sample_ids(prob, n, seed)
    dp = dp if dp is not None else mc.to_device(prob)
    g = mc.replay(dp, views, hists, options=options)
    o = oracle.replay(prob, views, hists)
    same = same_outcome(g, o)
    frac = same.mean()
    rel_e = np.abs(g["e_final"][same] - o["e_final"][same]) / o["e_final"][same]
    say(f"{prob.name}: replay identical {frac:.6f} ({(~same).sum()} differ of {len(same)}), "
        f"max rel dE {rel_e.max() if len(rel_e) else 0:.2e}, tallied {np.sum(o['fate'] == 5)}")
    assert np.array_equal(g["emit_voxel"], o["emit_voxel"])      # integer inverse CDF: exact
    assert frac >= 0.999
    assert len(rel_e) == 0 or rel_e.max() < 1e-5
    return g, o


def full_replay(prob, dp, chunk=10_000_000):
    """Replay every history of the run's work range on both sides, in chunks.
    Returns the number compared, the identical fraction, and per fate the
    number of histories that have that fate on exactly one side."""
    mc = _mc()
    begin = prob.history_offset
    end = begin + (prob.history_count or prob.n_histories - begin)
    n_same = 0
    one_side = np.zeros(8, np.int64)
    gpu_fates = np.zeros(8, np.int64)
    max_rel_e = 0.0
    for b in range(begin, end, chunk):
        e = min(end, b + chunk)
        views, hists = ids_of_work(prob, np.arange(b, e))
        g = mc.replay(dp, views, hists)
        o = oracle.replay(prob, views, hists)
        same = same_outcome(g, o)
        n_same += int(same.sum())
        gpu_fates += np.bincount(g["fate"], minlength=8)[:8]
        fd = g["fate"] != o["fate"]
        one_side += np.bincount(g["fate"][fd], minlength=8)[:8] + np.bincount(o["fate"][fd], minlength=8)[:8]
        if same.any():
            max_rel_e = max(max_rel_e, float(np.max(np.abs(g["e_final"][same] - o["e_final"][same])
                                                    / o["e_final"][same])))
        assert np.array_equal(g["emit_voxel"], o["emit_voxel"])
    n = end - begin
    return {"n": n, "identical": n_same / max(n, 1), "fate_flips": one_side, "max_rel_de": max_rel_e,
            "gpu_fates": gpu_fates}


def tallied_flips(prob, events, trip_g, trip_j):
    """The tallied histories whose (work index, bin) appears on one side only:
    the transport kernel's event list against the oracle's tallied list.
    Returns (gpu-only bins, oracle-only bins) as arrays of tally indices."""
    gk = events["work"].astype(np.int64) * (1 << 32) + events["bin"].astype(np.int64)
    ok = np.asarray(trip_g, np.int64) * (1 << 32) + np.asarray(trip_j, np.int64)
    g_only = np.setdiff1d(gk, ok, assume_unique=False)
    o_only = np.setdiff1d(ok, gk, assume_unique=False)
    return g_only & 0xFFFFFFFF, o_only & 0xFFFFFFFF


def oracle_run(prob):
    """The oracle's full run of a problem with its list of tallied histories."""
    return oracle.simulate(prob, want_triplets=True, trip_cap=max(1 << 20, prob.n_histories // 1000))


def compare_aggregates(prob, dp, fates, tally, tsq, energy, cnt, ev, o, replay_all=True):
    """One problem's aggregates from the transport kernel (fates, tally and
    squared tally as float counts, energies in keV, work counters, its event
    list with problem-local work indices) against the oracle run o.  Returns
    the relative error of each aggregate."""
    N = prob.history_count or prob.n_histories - prob.history_offset
    assert cnt[3] == N == fates.sum()
    assert tally.sum() == fates[5] == len(ev)
    np.testing.assert_array_equal(tally, tsq)
    # tallies: the difference is exactly the histories tallied on one side only
    g_only, o_only = tallied_flips(prob, ev, o["trip_g"], o["trip_j"])
    n_bins = int(np.prod(prob.tally_shape))
    explained = (np.bincount(g_only, minlength=n_bins) - np.bincount(o_only, minlength=n_bins)).astype(np.float64)
    np.testing.assert_array_equal((tally - o["tally"]).reshape(-1), explained)
    T = float(o["fates"][5])
    n_flip_tal = len(g_only) + len(o_only)
    err = {"tallied_histories": int(T), "tallied_flipped": n_flip_tal}
    per = int(np.prod(prob.tally_shape[2:]))
    cls_g = (g_only // per) % 2
    cls_o = (o_only // per) % 2
    for c, name in ((0, "primary"), (1, "scatter")):
        a, b = tally[:, c].sum(), o["tally"][:, c].sum()
        flips_c = int(np.sum(cls_g == c) + np.sum(cls_o == c))
        assert abs(a - b) <= 1e-4 * b + flips_c, (name, a, b, flips_c)
        err[f"{name}_rel"] = float(abs(a - b) / max(b, 1.0))
    err["window_total_rel"] = float(abs(tally.sum() - T) / max(T, 1.0))
    assert n_flip_tal <= 1e-3 * T + 1, (n_flip_tal, T)
    # fates: transport counts against a full replay of both sides
    if replay_all:
        fr = full_replay(prob, dp)
        err["replay_identical_all"] = fr["identical"]
        assert fr["identical"] >= 0.999
        # the transport kernel ends every history as its replay does
        np.testing.assert_array_equal(fates[:7], fr["gpu_fates"][:7])
        for i in range(7):
            assert abs(int(fates[i]) - int(o["fates"][i])) <= 1e-4 * o["fates"][i] + fr["fate_flips"][i], \
                (i, fates[i], o["fates"][i], fr["fate_flips"][i])
    err["fates_max_rel"] = float(max(abs(int(fates[i]) - int(o["fates"][i])) / max(int(o["fates"][i]), 1)
                                     for i in range(7)))
    # energies (booked per history on the GPU, per interaction in the oracle)
    for i in range(3):
        assert abs(energy[i] - o["energy"][i]) <= 1e-4 * max(o["energy"][i], 1.0), (i, energy[i], o["energy"][i])
    err["energy_max_rel"] = float(max(abs(energy[i] - o["energy"][i]) / max(o["energy"][i], 1.0)
                                      for i in range(3)))
    # work counters (diagnostics): real collisions and Kahn attempts against
    # the plain walk; tentative collisions only in step_count_parity
    assert abs(cnt[1] - o["n_real"]) <= 1e-4 * o["n_real"]
    assert abs(cnt[2] - o["n_kahn"]) <= 1e-4 * max(o["n_kahn"], 1)
    say(f"{prob.name}: gpu fates {fates.tolist()}\n  oracle fates {o['fates'].tolist()}\n"
        f"  energy gpu {energy[:3]} oracle {o['energy'][:3]}\n  errors {err}")
    return err


def aggregate_parity(prob, options=None, replay_all=True, dp=None):
    """Aggregates of one forward run against the oracle's (see the module
    docstring for the bars).  Returns (Simulator, oracle result, errors)."""
    mc = _mc()
    dp = dp if dp is not None else mc.to_device(prob)
    o = oracle_run(prob)
    sim = mc.simulate(dp, options=options, event_capacity=int(o["fates"][5]) * 2 + 1024)
    sim.check_status()
    assert int(sim.n_events.item()) == int(sim.fates[0, 5].item())
    err = compare_aggregates(
        prob, dp, sim.fates.cpu().numpy()[0], mc.tally_float(sim.tally).reshape(prob.tally_shape),
        mc.tally_float(sim.tally_sq).reshape(prob.tally_shape),
        sim.energy.cpu().numpy()[0].astype(np.float64) / mc.Q23, sim.counters.cpu().numpy()[0],
        sim.events_numpy(), o, replay_all)
    return sim, o, err


def batch_parity(probs, dps, sim, replay_all=True):
    """Every problem of a batched run (a Simulator over probs, with an event
    list) against its own oracle run.  Returns the per-problem errors."""
    mc = _mc()
    fates = sim.fates.cpu().numpy()
    energy = sim.energy.cpu().numpy().astype(np.float64) / mc.Q23
    cnt = sim.counters.cpu().numpy()
    tallies = [mc.tally_float(t) for t in sim.tallies()]
    tsq = [t.cpu().numpy().astype(np.float64) / mc.Q32 for t in
           (sim.tally_sq[off:off + s] for off, s in zip(np.cumsum([0] + sim.sizes[:-1]), sim.sizes))]
    ev = sim.events_numpy()
    assert int(sim.n_events.item()) == len(ev) == int(fates[:, 5].sum())
    work = ev["work"].astype(np.int64)
    prefix = np.cumsum([0] + [p.history_count or p.n_histories - p.history_offset for p in probs])
    errs = []
    for i, (p, dp) in enumerate(zip(probs, dps)):
        mine = ev[(work >= prefix[i]) & (work < prefix[i + 1])].copy()
        mine["work"] -= np.uint64(prefix[i])
        o = oracle_run(p)
        errs.append(compare_aggregates(p, dp, fates[i], tallies[i].reshape(p.tally_shape),
                                       tsq[i].reshape(p.tally_shape), energy[i], cnt[i], mine, o,
                                       replay_all))
    return errs


def step_count_parity(prob, dp=None):
    """Tentative-collision counts of the transport kernel against the oracle
    run with the kernel's escape shortcut (the count is the only thing the
    shortcut changes)."""
    mc = _mc()
    dp = dp if dp is not None else mc.to_device(prob)
    sim = mc.simulate(dp)
    cnt = sim.counters.cpu().numpy()[0]
    o = oracle.simulate(prob, escape_shortcut=True)
    rel = abs(cnt[0] - o["n_tent"]) / o["n_tent"]
    say(f"{prob.name}: tentative collisions gpu {cnt[0]} oracle (escape shortcut) {o['n_tent']} rel {rel:.2e}")
    assert rel <= 1e-4
    return rel
