"""Library calls around the simulator, through the C ABI: the source total and
scaled-tally arithmetic of the reconstruction loops (exact against numpy),
and graph capture of a sequence of calls (every replay equal to the eager
calls, with eager work between replays)."""
import numpy as np
import pytest

import phantoms

pytestmark = pytest.mark.gpu


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def test_source_total_and_scale_tally():
    mc = _mc()
    import torch
    rng = np.random.Generator(np.random.PCG64(61))
    a = rng.integers(0, 4_000_000_000, size=100_003, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 4_000_000_000, size=100_003, dtype=np.uint64).astype(np.uint32)
    ta = torch.from_numpy(a.view(np.int32)).cuda()
    tb = torch.from_numpy(b.view(np.int32)).cuda()
    assert mc.source_total(ta) == int(a.astype(np.uint64).sum())
    assert mc.source_total(ta, tb) == int(np.abs(a.astype(np.int64) - b.astype(np.int64)).sum())
    t = rng.integers(-(1 << 45), 1 << 45, size=70_001)
    tt = torch.from_numpy(t).cuda()
    out = torch.empty(len(t), dtype=torch.float64, device="cuda")
    mc.scale_tally(tt, 3.25, out)
    want = t.astype(np.float64) * (3.25 / 2.0 ** 32)
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    mc.scale_tally(tt, -0.5, out, accumulate=True)
    np.testing.assert_array_equal(out.cpu().numpy(), want + t.astype(np.float64) * (-0.5 / 2.0 ** 32))


def test_graph_of_several_calls_replays_exactly():
    mc = _mc()
    import torch
    pa = phantoms.thorax_problem("ga", 32, 1.2, 2, 6, 180.0, 32, 1.2, 150_000)
    pb = phantoms.point_cube_64(80_000)
    sa = mc.Simulator(mc.to_device(pa), event_capacity=1 << 12)
    sb = mc.Simulator(mc.to_device(pb), options={"forced_detection": 1})
    sa.run(); sb.run()
    torch.cuda.synchronize()
    ref = [t.cpu().numpy().copy() for t in (sa.tally, sa.fates, sa.n_events, sb.tally, sb.fates)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    s = side.cuda_stream
    assert mc._lib.mc_graph_begin(s) == mc.MC_OK
    with torch.cuda.stream(side):
        sa.run()
        sb.run()
    import ctypes as C
    g = C.c_void_p()
    assert mc._lib.mc_graph_end(s, C.byref(g)) == mc.MC_OK
    try:
        for k in range(3):
            for t in (sa.tally, sa.fates, sb.tally, sb.fates):
                t.fill_(-3)
            assert mc._lib.mc_graph_launch(g, mc._stream_ptr()) == mc.MC_OK
            torch.cuda.synchronize()
            got = [t.cpu().numpy() for t in (sa.tally, sa.fates, sa.n_events, sb.tally, sb.fates)]
            for x, y in zip(got, ref):
                np.testing.assert_array_equal(x, y)
            # eager work between replays
            other = mc.simulate(mc.to_device(pb.with_(n_histories=5_000)))
            assert int(other.fates.sum().item()) == 5_000
    finally:
        assert mc._lib.mc_graph_destroy(g) == mc.MC_OK


def test_mlem_mostly_empty_rows_and_graph_replay():
    """A matrix with most bin rows and some voxel rows empty (as an analog
    response matrix is): the iterations sweep only the listed non-empty rows
    and give the oracle's image; 20 iterations captured as one graph replay
    bit-identically to the eager call, with eager work between replays."""
    mc = _mc()
    import oracle
    import torch
    T, truth = phantoms.random_system(200_000, 5000, 1e-5, seed=63)
    rng = np.random.Generator(np.random.PCG64(64))
    P = rng.poisson(T.astype(np.float64) @ truth * 50).astype(np.float32)
    empty_bins = int(np.sum(np.diff(T.tocsr().indptr) == 0))
    empty_vox = int(np.sum(np.diff(T.tocsc().indptr) == 0))
    assert empty_bins > 150_000 and empty_vox > 100
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    ml = mc.Mlem(m)
    S0 = rng.uniform(0.5, 2.0, size=T.shape[1]).astype(np.float32)
    img0 = torch.as_tensor(S0.copy(), device="cuda")
    ml.run(img0, 0)                             # S^0 masked by the sensitivity
    sens = np.asarray(T.sum(axis=0)).ravel()
    np.testing.assert_array_equal(img0.cpu().numpy(), np.where(sens > 0, S0, 0.0).astype(np.float32))
    img = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    ml.run(img, 20)
    eager = img.clone()
    o = oracle.mlem(T.astype(np.float64), P.astype(np.float64), 20)
    g = eager.cpu().numpy().astype(np.float64)
    msk = o > 1e-6 * o.max()
    assert np.max(np.abs(g[msk] - o[msk]) / o[msk]) <= 1e-6
    assert np.all(g[~msk] <= 1e-5 * o.max())

    def recon():
        img.fill_(1.0)
        ml.run(img, 20)
    graph = mc.Graph(recon)
    for k in range(3):
        img.fill_(-7.0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, eager), f"replay {k}"
        other = torch.ones_like(img)
        ml.run(other, 3)                        # eager use of the same workspace between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("n_bins,n_vox,density", [(3000, 800, 0.01), (600_000, 3000, 2e-4),
                                                  (600_000, 3000, 1e-3)])
def test_mlem_entry_count_checked_on_device(n_bins, n_vox, density):
    """mlem_iterate's nnz argument picks the layout (row order, compact, bin
    slices in these three cases); the true count gives the oracle's image,
    bit-reproducibly, and any other value leaves the image NaN."""
    mc = _mc()
    import oracle
    import torch
    T, truth = phantoms.random_system(n_bins, n_vox, density, seed=65)
    rng = np.random.Generator(np.random.PCG64(66))
    P = rng.poisson(T.astype(np.float64) @ truth * 20).astype(np.float32)
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    ws = torch.empty(mc._lib.mlem_workspace_bytes(n_bins, n_vox), dtype=torch.uint8, device="cuda")
    o = oracle.mlem(T.astype(np.float64), P.astype(np.float64), 10)
    msk = o > 1e-6 * o.max()

    def run(nnz):
        img = torch.ones(n_vox, dtype=torch.float32, device="cuda")
        rc = mc._lib.mlem_iterate(n_bins, n_vox, nnz, m.T_rowptr.data_ptr(), m.T_col.data_ptr(),
                                  m.T_val.data_ptr(), m.Tt_rowptr.data_ptr(), m.Tt_col.data_ptr(),
                                  m.Tt_val.data_ptr(), m.proj.data_ptr(), img.data_ptr(), 10,
                                  ws.data_ptr(), ws.numel(), mc._stream_ptr())
        assert rc == mc.MC_OK
        return img
    a = run(T.nnz)
    g = a.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g[msk] - o[msk]) / o[msk]) <= 1e-6
    assert np.all(g[~msk] <= 1e-5 * o.max())
    for wrong in (0, T.nnz - 1, T.nnz + 1, 10 * T.nnz):
        assert torch.isnan(run(wrong)).all(), wrong
    assert torch.equal(run(T.nnz), a)
