"""GPU parity of the forward transport against the FP64 oracle, through the C ABI.

The bars are those of tests/parity.py: identical fate, detector bin and
scatter count for at least 99.9 % of replayed histories; every aggregate
difference accounted for by histories identified as flipped (the transport
kernel's event list against the oracle's tallied list, bin by bin exactly;
fate counts against a replay of every history on both sides), and within
1e-4 of the aggregate plus those flips; energies within 1e-4 relative.  The
oracle walks every history to the grid edge; the kernel's escape shortcut
outside the attenuation box changes only the count of tentative collisions,
which is compared with the oracle run with the same shortcut.
"""
import math

import numpy as np
import pytest

import oracle
import phantoms
from parity import (aggregate_parity, replay_parity, sample_ids, say,  # noqa: F401
                    step_count_parity)

pytestmark = pytest.mark.gpu


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def test_point_cube_64_replay():
    replay_parity(phantoms.point_cube_64(10 ** 6))


def test_point_cube_64_aggregates():
    p = phantoms.point_cube_64(10 ** 6)
    aggregate_parity(p)
    step_count_parity(p)


def test_point_cube_64_photoelectric_heavy():
    p = phantoms.point_cube_64(300_000).with_(pe_fraction=0.3, name="pe_heavy")
    replay_parity(p, 50_000)
    aggregate_parity(p)


def test_thorax_small_replay_and_aggregates():
    p = phantoms.thorax_problem("thorax_64", 64, 0.6, 2, 60, 180.0, 64, 0.6, 2_000_000)
    replay_parity(p)
    aggregate_parity(p)
    step_count_parity(p)


def test_headline_thorax_128_full_parity():
    """The headline workload itself: 128^3 x 3 mm thorax, 60 views, 64^2 x
    6 mm, 126-154 keV, all 1e8 histories.  Aggregates against the oracle's
    full run (tallies explained bin by bin by the flipped tallied histories,
    fates by a replay of all 1e8 histories on both sides), 1e5 replayed ids
    drawn with PCG64(7), and tentative-collision counts against the oracle
    with the kernel's escape shortcut."""
    mc = _mc()
    p = phantoms.thorax_128(10 ** 8)
    dp = mc.to_device(p)
    say("headline parity: 128^3 thorax, 1e8 histories")
    replay_parity(p, n=100_000, seed=7, dp=dp)
    _, _, err = aggregate_parity(p, dp=dp)
    step_count_parity(p, dp=dp)
    say(f"headline per-result errors: {err}")


def _emission_table_kinds(act):
    """How the library's emission tables cover the activity CDF: runs are
    maximal stretches of a grid row with one weight; buckets (a power of two
    >= 2 x runs, width 2^s) hold the run of their first t and how many more
    they meet.  Returns the fraction of the activity mass in buckets meeting
    1, 2 and >= 3 runs, and in runs longer than one voxel with weight > 1
    (where the voxel is a division within the run)."""
    nz, ny, nx = act.shape
    w = act.reshape(-1).astype(np.uint64)
    ix = np.tile(np.arange(nx), ny * nz)
    left = np.concatenate([[0], w[:-1]])
    start = (w > 0) & ((ix == 0) | (left != w))
    idx = np.flatnonzero(start)
    csum = np.concatenate([[0], np.cumsum(w, dtype=np.uint64)])
    c = csum[idx]                                   # weight before each run
    total, R = int(csum[-1]), len(idx)
    run_end = np.concatenate([c[1:], [total]])
    cap = 1 << int(np.ceil(np.log2(2 * R)))
    s = 0
    while ((total - 1) >> s) >= cap:
        s += 1
    starts = np.arange(0, total, 1 << s, dtype=np.uint64)
    ends = np.minimum(starts + np.uint64((1 << s) - 1), np.uint64(total - 1))
    lo = np.searchsorted(c, starts, side="right") - 1
    hi = np.searchsorted(c, ends, side="right") - 1
    span = hi - lo + 1
    mass = (ends - starts + np.uint64(1)).astype(np.float64) / total
    out = {k: float(mass[(span == k) if k < 3 else (span >= 3)].sum()) for k in (1, 2, 3)}
    length = (run_end - c) // w[idx]
    div = (length > 1) & (w[idx] > 1)
    out["division"] = float(((run_end - c)[div]).astype(np.float64).sum() / total)
    out["runs"] = R
    return out


def test_emission_tables_skewed_activity():
    """Activity over nine decades (one hot voxel, a warm block, a faint body)
    gives emission buckets inside one run and buckets meeting many runs (a
    search: the faint body's runs share the few buckets its small mass
    spans), and runs of several voxels with weights above one (a division
    within the run).  The emitted voxel is integer arithmetic
    on both sides and must be identical for every history."""
    p = phantoms.thorax_problem("skewed_act", 40, 0.96, 3, 6, 180.0, 32, 1.2, 300_000)
    act = p.activity.copy()
    act[20, 20, 20] = 3_000_000_000
    act[10:14, 24:30, 15:19] = np.where(act[10:14, 24:30, 15:19] > 0, 2_000_000, 0)
    act[30, 5:9, :] = 7
    p = p.with_(activity=act)
    kinds = _emission_table_kinds(act)
    say(f"emission table mass by runs met per bucket: {kinds}")
    assert kinds[1] > 0.5 and kinds[3] > 1e-4 and kinds["division"] > 1e-3
    g, o = replay_parity(p, n=60_000, seed=11)
    v = g["emit_voxel"]
    assert np.any(v == 20 + 40 * (20 + 40 * 20)) and len(np.unique(v)) >= 90   # hot, warm block, faint body


def test_emission_random_weights_every_voxel_a_run():
    """Random weights 0-5 in every voxel: almost every active voxel is a run
    of its own, so the tables are as large as the grid allows and buckets meet
    one or two runs; every emitted voxel identical to the oracle's."""
    n = 48
    rng = np.random.Generator(np.random.PCG64(19))
    p = phantoms.thorax_problem("rand_act", n, 0.8, 3, 5, 180.0, 32, 1.2, 200_000)
    p = p.with_(activity=rng.integers(0, 6, size=(n, n, n)).astype(np.uint32))
    kinds = _emission_table_kinds(p.activity)
    say(f"random weights: {kinds}")
    assert kinds["runs"] > 0.7 * np.count_nonzero(p.activity) and kinds[2] > 0.1
    replay_parity(p, n=50_000, seed=12)


def test_thorax_odd_non_cubic_grid():
    mu, act = phantoms.thorax(48, 0.8, 9)
    mu = np.ascontiguousarray(mu[3:44, 1:46, :])       # nz=41, ny=45, nx=48
    act = np.ascontiguousarray(act[3:44, 1:46, :])
    p = phantoms.thorax_problem("thorax_odd", 48, 0.8, 9, 7, 180.0, 40, 0.9, 700_001).with_(
        nz=41, ny=45, nx=48, mu=mu, activity=act, e_cut_kev=10.0)
    replay_parity(p, 50_000)
    aggregate_parity(p)


def test_vacuum_geometric_efficiency():
    n = 16
    mu = np.zeros((n, n, n), np.float32)
    act = np.zeros((n, n, n), np.uint32)
    act[n // 2, n // 2, n // 2] = 1
    alpha = math.radians(20.0)
    p = phantoms.point_source_cube("vac", n, 1.0, 400_000).with_(mu=mu, activity=act,
                                                                 accept_half_angle_rad=alpha)
    sim, o, _ = aggregate_parity(p)
    fates = sim.fates.cpu().numpy()[0]
    pexp = 0.5 * (1 - math.cos(alpha))
    z = (fates[5] - p.n_histories * pexp) / math.sqrt(p.n_histories * pexp * (1 - pexp))
    assert abs(z) < 4


@pytest.mark.parametrize("forced_direction", [False, True])
def test_wave_aggregated_tally_equals_per_arrival_sum(forced_direction):
    """Analog arrivals of one wavefront that share a bin are summed before one
    atomic (Sec. 2 tallies); weighted arrivals (forced direction) keep one
    atomic each.  A point source in vacuum with a wide cone on an 8x8 detector
    of 2 cm pixels puts many arrivals of each wavefront into the same few
    bins.  Every bin of the tally (and of the squared tally) must equal the
    sum over that bin's listed arrivals, whose records are written one per
    lane."""
    mc = _mc()
    n = 16
    mu = np.zeros((n, n, n), np.float32)
    act = np.zeros((n, n, n), np.uint32)
    act[n // 2, n // 2, n // 2] = 1
    alpha = math.radians(20.0)
    p = phantoms.point_source_cube("vac_agg", n, 1.0, 300_000, nu=8, pixel_cm=2.0).with_(
        mu=mu, activity=act, accept_half_angle_rad=alpha)
    opts = {"variance_reduction": 1, "forced_direction_half_angle": alpha} if forced_direction else None
    sim = mc.simulate(mc.to_device(p), event_capacity=400_000, options=opts)
    ev = sim.events_numpy()
    n_tallied = int(sim.fates[0, 5].item())
    assert len(ev) == int(sim.n_events.item()) == n_tallied
    assert n_tallied > (p.n_histories // 2 if forced_direction else 5000)
    tally = sim.tally.cpu().numpy().astype(np.int64)
    sq = sim.tally_sq.cpu().numpy().astype(np.int64)
    bins = ev["bin"].astype(np.int64)
    count = np.bincount(bins, minlength=tally.size)
    wsum = np.zeros(tally.size, dtype=np.int64)
    np.add.at(wsum, bins, ev["weight"].astype(np.int64))
    np.testing.assert_array_equal(tally, wsum)
    if forced_direction:
        # one weight for every arrival (no interaction in vacuum): the squared
        # tally is the count times one Q11.52 square
        hit = count > 0
        per = sq[hit] // count[hit]
        assert np.all(per * count[hit] == sq[hit]) and np.all(per == per[0]) and per[0] > 0
        assert np.all(sq[~hit] == 0)
    else:
        np.testing.assert_array_equal(sq, tally)
    say(f"aggregated tally ({'forced direction' if forced_direction else 'analog'}): {n_tallied} "
        f"arrivals in {int((count > 0).sum())} bins, largest bin {int(count.max())}")


def test_run_to_run_and_option_independence():
    mc = _mc()
    p = phantoms.thorax_problem("thorax_64", 64, 0.6, 2, 60, 180.0, 64, 0.6, 1_000_000)
    dp = mc.to_device(p)
    ref = mc.simulate(dp)
    t0 = ref.tally.clone()
    f0 = ref.fates.clone()
    e0 = ref.energy.clone()
    assert int(ref.check_status()[2]) == 1          # segmented map: one-byte palette codes
    for opts in (None, {"hist_per_lane": 1}, {"hist_per_lane": 64, "block_size": 64},
                 {"block_size": 128, "blocks_per_cu": 1}, {"hist_per_lane": 5, "blocks_per_cu": 3},
                 {"threshold_bytes": 4}, {"threshold_bytes": 4, "brick_log2": 3},
                 {"threshold_bytes": 1, "brick_log2": 2}):
        s = mc.simulate(dp, options=opts)
        want_pal = 0 if (opts or {}).get("threshold_bytes") == 4 else 1
        assert int(s.check_status()[2]) == want_pal, opts
        assert bool((s.tally == t0).all()), opts
        assert bool((s.fates == f0).all()), opts
        assert bool((s.energy == e0).all()), opts


@pytest.mark.parametrize("n_distinct", [256, 257])
def test_threshold_palette_capacity(n_distinct):
    """A water cube whose voxels take n_distinct attenuation values (+/-30 %):
    256 distinct thresholds still fit the one-byte palette, 257 fall back to
    the 32-bit table.  Either way the histories match the oracle and the
    forced 32-bit run bit for bit."""
    mc = _mc()
    n = 32
    p = phantoms.point_source_cube(f"pal{n_distinct}", n, 0.6, 400_000, seed=5).with_(
        angles=phantoms.view_angles(8, 180.0), nu=32, nv=32, pixel_cm=1.2)
    rng = np.random.Generator(np.random.PCG64(n_distinct))
    levels = (phantoms.MU_WATER_140 * (0.7 + 0.6 * np.arange(n_distinct) / (n_distinct - 1))).astype(np.float32)
    mu = levels[rng.integers(0, n_distinct, size=(n, n, n))]
    mu.ravel()[:n_distinct] = levels                  # every level present
    act = rng.integers(0, 3, size=(n, n, n)).astype(np.uint32)
    p = p.with_(mu=mu, activity=act, source_mode=phantoms.SOURCE_VOXELS)
    dp = mc.to_device(p)
    a = mc.simulate(dp)
    b = mc.simulate(dp, options={"threshold_bytes": 4})
    assert int(a.check_status()[2]) == (1 if n_distinct <= 256 else 0)
    assert int(b.check_status()[2]) == 0
    for x, y in zip(outputs_of(a), outputs_of(b)):
        np.testing.assert_array_equal(x, y)
    replay_parity(p, n=20_000, seed=n_distinct)


def outputs_of(sim):
    return (sim.tally.cpu().numpy(), sim.fates.cpu().numpy(), sim.energy.cpu().numpy(),
            sim.counters.cpu().numpy())


def test_resume_ranges_sum_exactly():
    mc = _mc()
    p = phantoms.thorax_problem("thorax_64", 64, 0.6, 2, 13, 180.0, 64, 0.6, 500_003)
    full = mc.simulate(mc.to_device(p))
    a = mc.simulate(mc.to_device(p.with_(history_offset=0, history_count=123_457)))
    b = mc.simulate(mc.to_device(p.with_(history_offset=123_457, history_count=0)))
    assert bool((full.tally == a.tally + b.tally).all())
    assert bool((full.fates == a.fates + b.fates).all())
    assert bool((full.energy == a.energy + b.energy).all())


@pytest.mark.parametrize("n", [1, 7, 59, 61])
def test_tiny_history_counts(n):
    # fewer histories than views: some views get none
    p = phantoms.thorax_problem("thorax_32", 32, 1.2, 2, 60, 180.0, 32, 1.2, n)
    mc = _mc()
    sim = mc.simulate(mc.to_device(p))
    o = oracle.simulate(p)
    np.testing.assert_array_equal(sim.fates.cpu().numpy()[0], o["fates"])


def test_event_list_matches_oracle_replay():
    mc = _mc()
    p = phantoms.thorax_problem("thorax_64", 64, 0.6, 2, 60, 180.0, 64, 0.6, 2_000_000)
    sim = mc.simulate(mc.to_device(p), event_capacity=10_000)
    ev = sim.events_numpy()
    assert len(ev) == int(sim.n_events.item()) == int(sim.fates[0, 5].item())
    q, r = divmod(p.n_histories, p.n_views)
    g = ev["work"].astype(np.int64)
    big = q + 1
    view = np.where(g < r * big, g // big, r + (g - r * big) // q).astype(np.int32)
    hist = np.where(g < r * big, g % big, (g - r * big) % q).astype(np.uint64)
    o = oracle.replay(p, view, hist)
    b = ((o["view"] * 2 + o["cls"]) * p.nv + o["iv"]) * p.nu + o["iu"]
    assert np.all(ev["weight"] == 1 << 32)              # an analog arrival counts one
    ok = (o["fate"] == 5) & (b == ev["bin"]) & (o["emit_voxel"] == ev["emit_voxel"])
    say(f"event list: {ok.mean():.6f} of {len(ok)} tallied histories confirmed by the oracle")
    assert ok.mean() >= 0.999


def test_bad_inputs_reported_in_status():
    mc = _mc()
    p = phantoms.point_cube_64(1000)
    mu = p.mu.copy()
    mu[3, 4, 5] = -0.1
    with pytest.raises(mc.McError):
        mc.simulate(mc.to_device(p.with_(mu=mu)))
    with pytest.raises(mc.McError):
        mc.simulate(mc.to_device(p.with_(activity=np.zeros_like(p.activity))))
    mu = p.mu.copy()
    mu[0, 0, 0] = np.nan
    with pytest.raises(mc.McError):
        mc.replay(mc.to_device(p.with_(mu=mu)), np.zeros(4, np.int32), np.arange(4, dtype=np.uint64))


def test_step_cap_reported():
    mc = _mc()
    p = phantoms.point_cube_64(20_000).with_(max_steps=1)
    sim = mc.simulate(mc.to_device(p))
    st = sim.check_status()
    o = oracle.simulate(p)
    assert st[0] & mc.STATUS_CAPPED
    assert st[1] == sim.fates[0, 6].item() == o["fates"][6] > 0


def test_max_axis_grid():
    """The largest grid axis (1024 voxels: packed coordinates use all 10
    bits), with activity in the last voxel along every axis and in the
    first: emission voxels identical to the oracle's, aggregates to 1e-4."""
    nx, ny, nz, vox = 1024, 8, 8, 0.05
    mu = np.full((nz, ny, nx), 0.151, np.float32)
    act = np.zeros((nz, ny, nx), np.uint32)
    act[nz - 1, ny - 1, nx - 1] = 5
    act[0, 0, 0] = 3
    act[nz // 2, ny // 2, 700:710] = 1
    base = phantoms.point_cube_64(400_000)
    p = base.with_(name="max_axis", nx=nx, ny=ny, nz=nz, voxel_cm=vox, mu=mu, activity=act,
                   source_mode=phantoms.SOURCE_VOXELS, accept_half_angle_rad=math.radians(10.0),
                   radius_cm=phantoms.detector_radius(nx, ny, vox), nu=64, nv=16, pixel_cm=0.8)
    g, o = replay_parity(p, n=100_000)
    assert (g["emit_voxel"] == nx * ny * nz - 1).any() and (g["emit_voxel"] == 0).any()
    aggregate_parity(p)
