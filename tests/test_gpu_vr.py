"""Forced direction and forced interaction (Sec. 5.2, weighted analog
transport) on the GPU against the oracle, through the C ABI.

Bars: replayed histories identical to the oracle's for 99.9 % or more (the
same draws, the cone direction from the emission words, no absorption under
forced interaction); weighted tallies bin by bin within 1e-3 of the total
plus two weights (rare flipped histories; FP32 weights against FP64), per
class within 1e-4; in vacuum the forced-direction total is N (1 - cos a)/2
to FP32 rounding; runs bit-identical from run to run and across launch
options; listed events carry the weights and sum to the tally exactly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import phantoms

pytestmark = pytest.mark.gpu

from parity import sample_ids  # noqa: E402


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _opts(flags, beta):
    return {"variance_reduction": flags, "forced_direction_half_angle": beta}


def vr_parity(prob, flags, beta, n_replay=50_000):
    mc = _mc()
    dp = mc.to_device(prob)
    opts = _opts(flags, beta)
    op = prob.with_(vr_flags=flags, vr_cone_rad=beta)
    views, hists = sample_ids(prob, n_replay)
    g = mc.replay(dp, views, hists, options=opts)
    o = oracle.replay(op, views, hists)
    same = ((g["fate"] == o["fate"]) & (g["iu"] == o["iu"]) & (g["iv"] == o["iv"])
            & (g["n_scatter"] == o["n_scatter"]))
    say(f"{prob.name} vr {flags}: replay identical {same.mean():.6f}; absorbed {np.sum(g['fate'] == 0)}")
    assert same.mean() >= 0.999
    if flags & 2:
        assert np.sum(g["fate"] == 0) == 0
    sim = mc.simulate(dp, options=opts)
    r = oracle.simulate(op)
    gt = mc.tally_float(sim.tally).reshape(prob.tally_shape)
    ot = r["tally"]
    wmax = 0.5 * (1 - math.cos(beta)) if flags & 1 else 1.0
    l1 = np.abs(gt - ot).sum()
    say(f"  weighted total gpu {gt.sum():.6e} oracle {ot.sum():.6e}; bin L1 {l1:.3e} (wmax {wmax:.3e})")
    assert l1 <= 1e-3 * ot.sum() + 2 * wmax
    for c in range(2):
        assert abs(gt[:, c].sum() - ot[:, c].sum()) <= 1e-4 * ot.sum() + 2 * wmax
    return sim


def test_forced_direction_vacuum_total():
    mc = _mc()
    N = 1_000_000
    a = math.radians(3.0)
    p = phantoms.point_cube_64(N).with_(mu=np.zeros((64, 64, 64), np.float32), accept_half_angle_rad=a)
    sim = mc.simulate(mc.to_device(p), options=_opts(1, a))
    tot = mc.tally_float(sim.tally).sum()
    w = 0.5 * (1 - math.cos(a))
    say(f"vacuum forced direction: total {tot:.9e} expected {N * w:.9e}")
    assert tot == pytest.approx(N * w, rel=1e-6)
    assert int(sim.fates[0, 5].item()) == N


@pytest.mark.parametrize("flags", [1, 2, 3])
def test_vr_thorax_matches_oracle(flags):
    p = phantoms.thorax_problem("vr_thorax", 40, 0.96, 2, 12, 180.0, 32, 1.2, 1_000_000).with_(
        pe_fraction=0.05, accept_half_angle_rad=math.radians(5.0), e_lo_kev=110.0, e_cut_kev=60.0)
    vr_parity(p, flags, math.radians(7.0))


def test_vr_point_cube_wide_cone():
    p = phantoms.point_cube_64(1_000_000).with_(accept_half_angle_rad=math.radians(10.0), pe_fraction=0.1)
    vr_parity(p, 3, math.radians(10.0))


def test_vr_run_to_run_options_and_events():
    mc = _mc()
    p = phantoms.thorax_problem("vr_opts", 32, 1.2, 3, 8, 180.0, 32, 1.2, 200_000).with_(
        accept_half_angle_rad=math.radians(6.0), pe_fraction=0.05)
    dp = mc.to_device(p)
    base = _opts(3, math.radians(8.0))
    ref = mc.simulate(dp, options=base)
    outs = [t.cpu().numpy().copy() for t in (ref.tally, ref.tally_sq, ref.fates, ref.counters)]
    for extra in ({"hist_per_lane": 1}, {"block_size": 128, "blocks_per_cu": 1}, {"brick_log2": 2},
                  {"threshold_bytes": 4}):
        g = mc.simulate(dp, options={**base, **extra})
        for x, y in zip((g.tally, g.tally_sq, g.fates, g.counters), outs):
            np.testing.assert_array_equal(x.cpu().numpy(), y)
    ev_sim = mc.simulate(dp, options=base, event_capacity=1 << 16)
    ev = ev_sim.events_numpy()
    assert len(ev) == int(ev_sim.fates[0, 5].item())
    assert int(ev["weight"].sum()) == int(ev_sim.tally.sum().item())
    assert np.all(ev["weight"] < (1 << 32)) and np.all(ev["weight"] > 0)
