"""Convolution-based forced detection (Sec. 5.2) on the GPU against the
oracle, through the C ABI.

Bars: the analog part of a run (fates, energies, counters) equals the plain
run bit for bit; the convolved tally (FP32 scores in Q31.32 layers, FP64
convolution) agrees with the oracle's FP64 one in class totals to 2e-5 and
bin by bin to 3e-4 of the total in L1 (as for forced detection: a copy whose
perpendicular hit lies within FP32 rounding of a pixel edge lands in the
neighbouring pixel, and one within rounding of a layer edge takes the
neighbouring layer's response); on the point source the primary total is the
narrow-beam closed form; runs are bit-identical from run to run, across
launch options and batched or alone; the sum of squares stays zero and the
event counter stays at zero.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import phantoms

pytestmark = pytest.mark.gpu

CFD = {"forced_detection": 2}


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def outputs(sim):
    return (sim.tally.cpu().numpy().copy(), sim.fates.cpu().numpy().copy(),
            sim.energy.cpu().numpy().copy(), sim.counters.cpu().numpy().copy())


def cfd_parity(prob, rel_bin=3e-4, rel_class=2e-5):
    mc = _mc()
    dp = mc.to_device(prob)
    say(f"cfd parity: {prob.name} views {prob.n_views} hist {prob.n_histories}")
    g = mc.simulate(dp, options=CFD)
    a = mc.simulate(dp, want_sq=False)
    o = oracle.simulate_cfd(prob)
    gt = mc.tally_float(g.tally).reshape(prob.tally_shape)
    ot = o["tally"]
    np.testing.assert_array_equal(g.fates.cpu().numpy(), a.fates.cpu().numpy())
    np.testing.assert_array_equal(g.energy.cpu().numpy(), a.energy.cpu().numpy())
    gc, ac = g.counters.cpu().numpy(), a.counters.cpu().numpy()
    np.testing.assert_array_equal(gc[:, :4], ac[:, :4])
    # forced-copy ray walks: at most one per history and one per real
    # collision, each visiting at least one voxel; none in an analog run
    assert not ac[:, 4:].any()
    assert 0 < gc[0, 4] <= gc[0, 3] + gc[0, 1] and gc[0, 5] >= gc[0, 4]
    assert int(g.tally_sq.abs().sum().item()) == 0
    tot = ot.sum()
    l1 = np.abs(gt - ot).sum() / tot
    cls_rel = [abs(gt[:, c].sum() - ot[:, c].sum()) / ot[:, c].sum() for c in range(2)]
    say(f"{prob.name}: CFD total {gt.sum():.6e} oracle {tot:.6e}; bin L1 {l1:.2e}; "
        f"class rel {cls_rel[0]:.2e} {cls_rel[1]:.2e}; "
        f"nonzero bins {np.count_nonzero(gt)} / {np.count_nonzero(ot)}")
    assert l1 <= rel_bin
    assert max(cls_rel) <= rel_class
    return g, gt, o


def test_cfd_point_cube_closed_form_and_oracle():
    """Point source at the cube centre: every primary copy runs 6.4 cm of
    water along the axis, so the class-0 total per history is
    (1 - cos a) / 2 * exp(-6.4 mu) (the responses are normalised and the
    spread stays on the detector)."""
    p = phantoms.point_cube_64(200_000)
    g, gt, o = cfd_parity(p)
    c = math.cos(p.accept_half_angle_rad)
    pexp = 0.5 * (1.0 - c) * math.exp(-float(np.float32(0.151)) * 6.4)
    got = gt[0, 0].sum() / p.n_histories
    say(f"point cube CFD primary per history {got:.8e}, closed form {pexp:.8e}")
    assert got == pytest.approx(pexp, rel=2e-6)


def test_cfd_thorax_small_matches_oracle():
    p = phantoms.thorax_problem("cfd_thorax32", 32, 1.2, 2, 12, 180.0, 32, 1.2, 300_000)
    cfd_parity(p)


def test_cfd_thorax_photoelectric_wide_cone():
    """Photoelectric share 0.3, 10 degree cone (responses up to 19 x 19
    pixels), window down to 100 keV."""
    p = phantoms.thorax_problem("cfd_pe", 32, 1.2, 3, 6, 180.0, 32, 1.2, 200_000).with_(
        pe_fraction=0.3, accept_half_angle_rad=math.radians(10.0), e_lo_kev=100.0, e_cut_kev=100.0)
    cfd_parity(p)


def test_cfd_thorax_128_full_geometry_sampled():
    """The 128^3 thorax geometry (60 views, 64^2 x 6 mm, 94 depth layers) on
    work indices [4e7, 4e7 + 2e5) of its 1e8 histories."""
    p = phantoms.thorax_128(10 ** 8).with_(history_offset=40_000_000, history_count=200_000)
    cfd_parity(p)


def test_cfd_ragged_detector():
    """Detector sizes that are not whole convolution tiles (nu 37, nv 21)."""
    p = phantoms.thorax_problem("cfd_ragged", 24, 1.6, 5, 5, 180.0, 37, 1.1, 120_000).with_(nv=21)
    cfd_parity(p)


def test_cfd_run_to_run_options_and_batch():
    mc = _mc()
    rng = np.random.Generator(np.random.PCG64(29))
    probs = []
    for i in range(3):
        n = int(rng.integers(24, 41))
        probs.append(phantoms.thorax_problem(f"cfdb{i}", n, 38.4 / n, 1300 + i, int(rng.integers(3, 10)),
                                             180.0, 32, 1.2, 50_000 + 7 * i, problem_id=i))
    dps = [mc.to_device(p) for p in probs]
    ref = outputs(mc.simulate(dps[0], options=CFD))
    for opts in ({}, {"hist_per_lane": 1}, {"block_size": 128, "blocks_per_cu": 1},
                 {"hist_per_lane": 7, "brick_log2": 2}, {"threshold_bytes": 4}):
        got = outputs(mc.simulate(dps[0], options={**CFD, **opts}))
        for x, y in zip(got, ref):
            np.testing.assert_array_equal(x, y)
    batch = outputs(mc.simulate(dps, options=CFD))
    off = 0
    for i, dp in enumerate(dps):
        one = outputs(mc.simulate(dp, options=CFD))
        np.testing.assert_array_equal(batch[0][off:off + one[0].size], one[0])
        np.testing.assert_array_equal(batch[1][i], one[1][0])
        off += one[0].size
    sim = mc.simulate(dps[0], options=CFD)
    assert int(sim.n_events.item()) == 0
