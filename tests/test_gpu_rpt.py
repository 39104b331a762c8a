"""Reuse of photon tracks (Sec. 5.3) on the GPU against the oracle, through
the C ABI: difference sources (activity - activity_prev).

Bars: the emission voxel of every replayed history is identical (the integer
inverse CDF over |d|), and at least 99.9 % of replayed histories identical;
analog tallies bin by bin as for plain sources (identical up to rare flipped
histories) with the sign of d applied; forced detection and CFD to their
usual bars; a zero previous estimate gives the plain run bit for bit and a
zero new one its exact negation; every listed event carries the sign of d
at its emission voxel; the projector that chains difference projections
agrees with direct projections to the forced-detection noise.
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


def _pair(p, bias=0.1, seed=11):
    new, prev = phantoms.estimate_pair(p.activity, 0.2, seed, bias=bias)
    return p.with_(activity=new, activity_prev=prev), new, prev


def _outputs(sim):
    return [t.cpu().numpy().copy() for t in (sim.tally, sim.tally_sq, sim.fates, sim.energy,
                                             sim.counters)]


def test_rpt_difference_source_matches_oracle():
    mc = _mc()
    base = phantoms.thorax_problem("rpt_thorax64", 64, 0.6, 2, 60, 180.0, 64, 0.6, 2_000_000)
    p, new, prev = _pair(base)
    say(f"rpt parity: {p.name} hist {p.n_histories}")
    d = new.astype(np.int64) - prev.astype(np.int64)
    dp = mc.to_device(p)
    # replay: same emission voxels (from |d|), same histories
    from parity import replay_parity
    replay_parity(p, n=50_000)
    sim = mc.simulate(dp, event_capacity=1 << 16)
    sim.check_status()
    o = oracle.simulate(p)
    t = mc.tally_float(sim.tally).reshape(p.tally_shape)
    tsq = mc.tally_float(sim.tally_sq).reshape(p.tally_shape)
    fates = sim.fates.cpu().numpy()[0]
    n_tal = int(fates[5])
    say(f"  tallied {n_tal}, signed total gpu {t.sum():.0f} oracle {o['tally'].sum():.0f}, "
        f"negative share {(t < 0).sum()} bins")
    assert (t < 0).any() and (t > 0).any()
    assert tsq.sum() == n_tal
    assert np.all(np.abs(t) <= tsq)
    diff = np.abs(t - o["tally"]).sum()
    assert diff <= max(2, 1e-3 * n_tal), diff
    assert np.abs(tsq - o["tally_sq"]).sum() <= max(2, 1e-3 * n_tal)
    for i in range(7):
        assert abs(fates[i] - o["fates"][i]) <= 1e-4 * p.n_histories
    ev = sim.events_numpy()
    assert len(ev) == n_tal
    want = np.where(d.reshape(-1)[ev["emit_voxel"]] < 0, -(1 << 32), 1 << 32)
    np.testing.assert_array_equal(ev["weight"], want)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_rpt_zero_previous_and_negation(mode):
    """activity_prev = 0 is the plain source bit for bit; activity = 0 with
    activity_prev = a negates every contribution exactly (analog, forced
    detection, CFD)."""
    mc = _mc()
    p = phantoms.thorax_problem("rpt_neg", 32, 1.2, 4, 8, 180.0, 32, 1.2, 150_000)
    act = p.activity * np.uint32(5)
    zero = np.zeros_like(act)
    opts = {"forced_detection": mode} if mode else None
    plain = _outputs(mc.simulate(mc.to_device(p.with_(activity=act)), options=opts))
    same = _outputs(mc.simulate(mc.to_device(p.with_(activity=act, activity_prev=zero)), options=opts))
    neg = _outputs(mc.simulate(mc.to_device(p.with_(activity=zero, activity_prev=act)), options=opts))
    for x, y in zip(same, plain):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(neg[0], -plain[0])
    for x, y in zip(neg[1:], plain[1:]):
        np.testing.assert_array_equal(x, y)
    assert np.count_nonzero(plain[0]) > 0


@pytest.mark.parametrize("mode", [1, 2])
def test_rpt_forced_detection_matches_oracle(mode):
    mc = _mc()
    base = phantoms.thorax_problem("rpt_fd", 32, 1.2, 2, 12, 180.0, 32, 1.2, 300_000)
    p, new, prev = _pair(base)
    g = mc.simulate(mc.to_device(p), options={"forced_detection": mode})
    o = (oracle.simulate_fd if mode == 1 else oracle.simulate_cfd)(p)
    gt = mc.tally_float(g.tally).reshape(p.tally_shape)
    ot = o["tally"]
    scale = np.abs(ot).sum()
    l1 = np.abs(gt - ot).sum() / scale
    cls = [abs(gt[:, c].sum() - ot[:, c].sum()) / scale for c in range(2)]
    say(f"rpt mode {mode}: signed total gpu {gt.sum():.6e} oracle {ot.sum():.6e}; bin L1 {l1:.2e}; "
        f"class {cls[0]:.2e} {cls[1]:.2e}")
    assert (ot < 0).any() and (ot > 0).any()
    assert l1 <= 3e-4
    assert max(cls) <= 2e-5


def test_rpt_projector_chains_difference_projections():
    """Three estimates projected in a chain (full, then two differences)
    agree with direct projections of the last estimate (forced detection,
    4e6 histories: ~4e-4 relative noise) to 3e-3 in total and 2 % per view
    and class, and the difference runs use a tenth of the histories or
    less."""
    mc = _mc()
    import torch
    p = phantoms.thorax_problem("rpt_chain", 32, 1.2, 5, 12, 180.0, 32, 1.2, 1)
    est = [p.activity.astype(np.uint32) * np.uint32(1000)]
    for k, bias in enumerate((0.05, -0.03)):
        nxt, _ = phantoms.estimate_pair(est[-1], 0.05, 30 + k, scale=1, bias=bias)
        est.append(nxt)
    dp = mc.to_device(p)
    hpu = 4e6 / float(est[0].sum())
    fd = {"forced_detection": 1}
    rp = mc.RptProjector(dp, hpu, options=fd)
    for a in est:
        proj = rp.project(torch.from_numpy(a.view(np.int32)).to("cuda"))
    say(f"projector histories per call {rp.histories}")
    assert rp.histories[1] <= rp.histories[0] / 10 and rp.histories[2] <= rp.histories[0] / 10
    # direct projections of the last estimate, two independent seeds
    direct = []
    for seed in (901, 902):
        q = mc.RptProjector(dp.with_(seed=seed), hpu, options=fd)
        direct.append(q.project(torch.from_numpy(est[-1].view(np.int32)).to("cuda")).cpu().numpy())
    chain = proj.cpu().numpy()
    ref = 0.5 * (direct[0] + direct[1])
    rel_seeds = abs(direct[0].sum() - direct[1].sum()) / ref.sum()
    rel = abs(chain.sum() - ref.sum()) / ref.sum()
    cells = chain.sum(axis=(2, 3)) / ref.sum(axis=(2, 3)) - 1.0
    say(f"chain vs direct: total rel {rel:.2e} (two direct seeds differ by {rel_seeds:.2e}); "
        f"per view and class max rel {np.abs(cells).max():.2e}")
    # forced detection at 4e6 histories: ~4e-4 relative noise on the total
    assert rel <= 3e-3
    assert np.abs(cells).max() <= 0.02
