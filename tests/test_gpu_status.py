"""Outcome codes through the C ABI: mc_check_status maps the status bits a
call left to a return code (bad input, fixed-point overflow, a list too
small, capped histories, in that order of precedence), and the adjoint reruns
with fewer fractional bits when a term overflows."""
import numpy as np
import pytest

import phantoms

pytestmark = pytest.mark.gpu


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def test_check_status_mapping():
    mc = _mc()
    import torch
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    want = [(0, mc.MC_OK), (mc.STATUS_CAPPED, mc.MC_ECAPPED),
            (mc.STATUS_LIST_OVERFLOW | mc.STATUS_CAPPED, mc.MC_ENOMEM),
            (mc.STATUS_TALLY_OVERFLOW | mc.STATUS_LIST_OVERFLOW, mc.MC_EOVERFLOW),
            (mc.STATUS_GRAD_OVERFLOW, mc.MC_EOVERFLOW), (mc.STATUS_ACTIVITY_OVERFLOW, mc.MC_EOVERFLOW),
            (mc.STATUS_BAD_MU | mc.STATUS_TALLY_OVERFLOW, mc.MC_EINVAL),
            (mc.STATUS_BAD_EVENT, mc.MC_EINVAL), (mc.STATUS_NO_ACTIVITY, mc.MC_EINVAL)]
    for bits, code in want:
        st[0] = bits
        assert mc._lib.mc_check_status(st.data_ptr(), mc._stream_ptr()) == code, bits


def test_check_status_of_forward_calls():
    """A clean run checks MC_OK (the tally range check sees no negative
    bin); a step cap of one gives MC_ECAPPED; an event list too small gives
    MC_ENOMEM; a NaN in mu gives MC_EINVAL."""
    mc = _mc()
    p = phantoms.point_cube_64(200_000)
    chk = lambda sim: mc._lib.mc_check_status(sim.status.data_ptr(), mc._stream_ptr())
    sim = mc.simulate(mc.to_device(p), event_capacity=1 << 12)
    assert chk(sim) == mc.MC_OK and int(sim.fates[0, 5].item()) > 2
    assert chk(mc.simulate(mc.to_device(p.with_(max_steps=1)))) == mc.MC_ECAPPED
    small = mc.simulate(mc.to_device(p), event_capacity=1)
    assert int(small.n_events.item()) > 1 and chk(small) == mc.MC_ENOMEM
    mu = p.mu.copy()
    mu[3, 3, 3] = np.nan
    bad = mc.simulate(mc.to_device(p.with_(mu=mu)), sync=False)
    assert chk(bad) == mc.MC_EINVAL
    with pytest.raises(mc.McError, match="invalid argument"):
        bad.check_status()


def test_adjoint_retries_with_fewer_fractional_bits():
    """A loss gradient large enough that its terms overflow at 40 fractional
    bits (G l 2^40 above 4e18 for crossings longer than 0.36 cm) while every
    voxel's sum stays far inside the range at 28 (at most ~1e3 tallied
    crossings of <= 0.7 cm: 1e7 x 700 x 2^28 = 1.9e18): an explicit
    frac_bits=40 raises, the default reruns and returns the frac_bits=28
    result; a gradient too large for 16 bits raises."""
    mc = _mc()
    import torch
    p = phantoms.point_source_cube("adj_retry", 32, 0.4, 300_000).with_(
        accept_half_angle_rad=np.radians(10.0))
    dp = mc.to_device(p)
    sim = mc.simulate(dp, event_capacity=1 << 16)
    G = torch.full(p.tally_shape, 1.0e7, dtype=torch.float64)
    with pytest.raises(mc.GradientOverflow):
        mc.adjoint(dp, G, sim, frac_bits=40)
    g28 = mc.adjoint(dp, G, sim, frac_bits=28)
    g = mc.adjoint(dp, G, sim)
    assert torch.equal(g, g28) and torch.isfinite(g).all() and g.abs().max().item() > 0
    with pytest.raises(mc.GradientOverflow):
        mc.adjoint(dp, torch.full(p.tally_shape, 1.0e30, dtype=torch.float64), sim)
