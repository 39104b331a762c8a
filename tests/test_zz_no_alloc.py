"""The no-allocation forward entry point (mc_simulate_projections_static)
against the workspace entry point, through the C ABI: bit-identical tallies,
squared tallies, fates, energies, counters and event lists on two calls in a
row, the second on a smaller problem (the shared scratch keeps the first
call's contents), and a refusal of a problem whose tables exceed the scratch."""
import numpy as np
import pytest

import phantoms

pytestmark = pytest.mark.gpu


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def _outputs(sim):
    ev = sim.events_numpy()
    order = np.lexsort((ev["bin"], ev["work"]))
    return [t.cpu().numpy().copy() for t in (sim.tally, sim.tally_sq, sim.fates, sim.energy,
                                             sim.counters, sim.n_events)] + [ev[order]]


def _compare(prob, options=None, capacity=1 << 16):
    mc = _mc()
    import torch
    dp = mc.to_device(prob)
    sim = mc.Simulator(dp, event_capacity=capacity, options=options)
    assert mc.workspace_bytes([dp], options) <= mc.STATIC_SCRATCH_BYTES
    sim.run()
    torch.cuda.synchronize()
    assert int(sim.n_events.item()) <= capacity     # a complete list is order-free
    ref = _outputs(sim)
    for t in (sim.tally, sim.tally_sq, sim.fates, sim.energy, sim.counters, sim.n_events):
        t.fill_(-7)                       # stale values must be overwritten
    sim.run_static()
    torch.cuda.synchronize()
    sim.check_status()
    got = _outputs(sim)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    return ref


def test_static_entry_point_matches_workspace_entry_point():
    # first call: the 128^3 thorax (its tables nearly fill the scratch)
    big = _compare(phantoms.thorax_128(2_000_000))
    assert big[2][0, 5] > 0
    # second call, smaller: a 64^3 point cube, with forced detection
    _compare(phantoms.point_cube_64(300_000), options={"forced_detection": 1}, capacity=1 << 21)
    # and a small batch of two thoraxes
    mc = _mc()
    import torch
    probs = [phantoms.thorax_problem(f"s{i}", 32, 1.2, 2 + i, 6, 180.0, 32, 1.2, 100_000 + i,
                                     problem_id=i) for i in range(2)]
    dps = [mc.to_device(p) for p in probs]
    a = mc.Simulator(dps)
    a.run()
    torch.cuda.synchronize()
    ref = [t.cpu().numpy().copy() for t in (a.tally, a.fates)]
    a.run_static()
    torch.cuda.synchronize()
    for x, y in zip([t.cpu().numpy() for t in (a.tally, a.fates)], ref):
        np.testing.assert_array_equal(x, y)


def test_static_entry_point_refuses_oversized_problems():
    mc = _mc()
    p = phantoms.thorax_problem("big", 192, 0.2, 2, 4, 180.0, 32, 1.2, 1000)
    dp = mc.to_device(p)
    assert mc.workspace_bytes([dp]) > mc.STATIC_SCRATCH_BYTES
    sim = mc.Simulator(dp)
    with pytest.raises(mc.McError, match="ENOMEM|capacity|workspace"):
        sim.run_static()
