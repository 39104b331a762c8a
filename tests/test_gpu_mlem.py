"""Response matrix (Sec. 5.1, Eq. IMC), MLEM (Eq. MLEM) and the ordered-subset
forms (OSEM, Eq. DMOS, the additive-scatter OS-EM of Sec. 5.4) on the GPU
against the oracle, through the C ABI.

Bars: reconstruction on a given matrix (inputs shared, FP32 values, FP64
accumulation on both sides) agrees with the oracle to 1e-6 relative (the
image is returned as FP32); the response matrix built
from the GPU event list has the oracle's sparsity pattern and values to FP32
rounding (1e-6), apart from histories whose fate flipped between FP32 and
FP64; reconstructed images agree to 1e-4 relative L2 (plus the flipped
histories' share).
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


def test_mlem_kernel_matches_oracle():
    mc = _mc()
    import torch
    T, truth = phantoms.random_system(5000, 700, 0.004, seed=31)
    rng = np.random.Generator(np.random.PCG64(32))
    P = rng.poisson(T.astype(np.float64) @ truth).astype(np.float32)
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    img = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    mc.Mlem(m).run(img, 30)
    g = img.cpu().numpy().astype(np.float64)
    o = oracle.mlem(T.astype(np.float64), P.astype(np.float64), 30)
    m_ = o > 1e-6 * o.max()
    rel = np.abs(g[m_] - o[m_]) / o[m_]
    say(f"mlem kernel: max rel {rel.max():.2e}")
    assert rel.max() <= 1e-6     # image stored as float32 at the end
    assert np.all(g[~m_] <= 1e-5 * o.max())


@pytest.mark.parametrize("density", [0.004, 0.1])
def test_mlem_sparse_and_dense_rows(density):
    """Sparse rows (one thread per row) and dense rows (one wavefront per row,
    as forced-detection matrices have) give the oracle's MLEM and OSEM images."""
    mc = _mc()
    import torch
    T, truth = phantoms.random_system(2400, 400, density, seed=34)
    rng = np.random.Generator(np.random.PCG64(35))
    P = rng.poisson(T.astype(np.float64) @ truth * 5).astype(np.float32)
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    img = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    mc.Mlem(m).run(img, 20)
    T64 = T.astype(np.float64)
    o = oracle.mlem(T64, P.astype(np.float64), 20)
    g = img.cpu().numpy().astype(np.float64)
    msk = o > 1e-6 * o.max()
    rel = np.max(np.abs(g[msk] - o[msk]) / o[msk])
    img2 = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    mc.osem(m, img2, 4, 6, 100)
    o2 = oracle.osem(T64, P.astype(np.float64), 4, 6, 100)
    g2 = img2.cpu().numpy().astype(np.float64)
    msk2 = o2 > 1e-6 * o2.max()
    rel2 = np.max(np.abs(g2[msk2] - o2[msk2]) / o2[msk2])
    say(f"density {density}: {T.nnz / T.shape[0]:.1f} per bin row; MLEM max rel {rel:.2e}, OSEM {rel2:.2e}")
    assert rel <= 1e-6 and rel2 <= 1e-6


def _mlem_vs_oracle(T, P, n_iter, m=None):
    mc = _mc()
    import torch
    m = mc.csr_from_scipy(T) if m is None else m
    m.proj = torch.as_tensor(P, device="cuda")
    ml = mc.Mlem(m)
    img = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    ml.run(img, n_iter)
    img2 = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    ml.run(img2, n_iter)
    assert torch.equal(img, img2), "MLEM must be deterministic"
    o = oracle.mlem(T.astype(np.float64), P.astype(np.float64), n_iter)
    g = img.cpu().numpy().astype(np.float64)
    msk = o > 1e-6 * o.max()
    rel = np.max(np.abs(g[msk] - o[msk]) / o[msk])
    assert np.all(g[~msk] <= 1e-5 * o.max())
    return rel


@pytest.mark.parametrize("n_bins,n_vox,density", [
    (1000, 4000, 0.03),        # 120 entries per bin row (64 lanes), 30 per voxel row (16)
    (600_000, 3000, 2e-5),     # large detector, sparse: compact layout, 12 entries per voxel row
    (600_000, 3000, 1e-4),     # compact layout, 60 entries per voxel row (16 lanes)
    (600_000, 20_000, 6e-5),   # bin slices, 4.5 entries per slice (4 lanes)
    (600_000, 3000, 1e-3),     # bin slices, 75 entries per slice (64 lanes)
])
def test_mlem_row_groups_and_bin_slices(n_bins, n_vox, density):
    """Every lane-group size of the sweeps and the per-XCD bin slices of the
    backprojection (2^19 bins or more, 16 entries per voxel row or more) give
    the oracle's image, bit-identically on a second run."""
    T, truth = phantoms.random_system(n_bins, n_vox, density, seed=36)
    rng = np.random.Generator(np.random.PCG64(37))
    P = rng.poisson(T.astype(np.float64) @ truth * 20).astype(np.float32)
    rel = _mlem_vs_oracle(T, P, 20)
    say(f"{n_bins} x {n_vox}, {T.nnz} entries: MLEM max rel {rel:.2e}")
    assert rel <= 1e-6


@pytest.mark.parametrize("n_bins,n_vox,density", [
    (600_000, 3000, 2e-5),     # compact layout
    (1000, 4000, 0.03),        # row order
    (600_000, 3000, 1e-3),     # bin slices
])
def test_mlem_prepared_equals_one_call(n_bins, n_vox, density):
    """mlem_prepare once, then mlem_iterate_prepared per reconstruction (new
    data and a new start image each time) gives mlem_iterate's image bit for
    bit; a call whose entry count differs from the prepared fingerprint
    sweeps nothing and leaves the image NaN, and the workspace serves
    matching calls afterwards."""
    mc = _mc()
    import torch
    T, truth = phantoms.random_system(n_bins, n_vox, density, seed=51)
    rng = np.random.Generator(np.random.PCG64(52))
    m = mc.csr_from_scipy(T)
    ml = mc.Mlem(m)                       # mlem_prepare
    for k in range(2):
        P = torch.as_tensor(rng.poisson(T.astype(np.float64) @ truth * (10 + 10 * k)).astype(np.float32),
                            device="cuda")
        S0 = rng.uniform(0.5, 2.0, size=n_vox).astype(np.float32)
        a = torch.as_tensor(S0.copy(), device="cuda")
        ml.run(a, 7, proj=P)
        b = torch.as_tensor(S0.copy(), device="cuda")
        ml.run_unprepared(b, 7, proj=P)   # set-up repeated inside the call
        assert torch.equal(a, b), k
        assert bool(torch.isfinite(a).all())
    img = torch.ones(n_vox, dtype=torch.float32, device="cuda")
    rc = mc._lib.mlem_iterate_prepared(m.n_bins, m.n_img, m.nnz + 1, *ml._csr(), P.data_ptr(), img.data_ptr(),
                                       3, ml.ws.data_ptr(), ml.ws.numel(), mc._stream_ptr())
    assert rc == 0
    torch.cuda.synchronize()
    assert bool(torch.isnan(img).all())
    c = torch.as_tensor(S0.copy(), device="cuda")
    ml.run(c, 7, proj=P)
    assert torch.equal(c, a)
    say(f"{n_bins} x {n_vox}, {T.nnz} entries: prepared calls identical to one-call MLEM")


def test_mlem_bin_slices_unsorted_rows():
    """Voxel rows whose columns are not ascending: the slice cuts then do not
    follow the slices, but the pieces still cover each row, so the result is
    the oracle's."""
    mc = _mc()
    import torch
    T, truth = phantoms.random_system(600_000, 2000, 6e-4, seed=38)
    rng = np.random.Generator(np.random.PCG64(39))
    P = rng.poisson(T.astype(np.float64) @ truth * 20).astype(np.float32)
    m = mc.csr_from_scipy(T)
    Tt = T.T.tocsr()
    Tt.sort_indices()
    col, val = Tt.indices.copy(), Tt.data.copy()
    for i in range(Tt.shape[0]):      # reverse every voxel row
        a, b = Tt.indptr[i], Tt.indptr[i + 1]
        col[a:b] = col[a:b][::-1]
        val[a:b] = val[a:b][::-1]
    m.Tt_col = torch.as_tensor(col.astype(np.int32), device="cuda")
    m.Tt_val = torch.as_tensor(val.astype(np.float32), device="cuda")
    rel = _mlem_vs_oracle(T, P, 15, m=m)
    say(f"unsorted voxel rows: MLEM max rel {rel:.2e}")
    assert rel <= 1e-6


def test_mlem_fixed_point_on_gpu():
    mc = _mc()
    import torch
    T, n = phantoms.random_system(3000, 400, 0.01, seed=33)
    sens = np.asarray(T.sum(axis=0)).ravel()
    n = np.where(sens > 0, n, 0.0).astype(np.float32)
    P = (T.astype(np.float64) @ n.astype(np.float64)).astype(np.float32)
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    img = torch.as_tensor(n.copy(), device="cuda")
    mc.Mlem(m).run(img, 10)
    np.testing.assert_allclose(img.cpu().numpy(), n, rtol=2e-6, atol=1e-7)


def _flips(sim, oe):
    ev = sim.events_numpy()
    a = set(zip(ev["work"].astype(np.int64).tolist(), ev["bin"].astype(np.int64).tolist()))
    b = set(zip(oe["trip_g"].tolist(), oe["trip_j"].tolist()))
    return len(a ^ b), len(b)


def check_system_and_mlem(prob, n_iter=50, cap=1 << 20):
    mc = _mc()
    import torch
    dp = mc.to_device(prob)
    sim = mc.simulate(dp, event_capacity=cap, want_sq=False)
    assert int(sim.n_events.item()) <= cap
    m = mc.system_matrix(dp, sim)
    oe = oracle.simulate(prob, want_triplets=True, trip_cap=cap)
    To, Po, _ = oracle.system_matrix(prob, oe["trip_i"], oe["trip_j"])
    n_flip, n_tal = _flips(sim, oe)
    Tg = m.to_scipy()
    Tgt = m.to_scipy(transpose=True)
    # the two orientations hold the same matrix
    assert (Tg.T - Tgt).count_nonzero() == 0
    # pattern and values
    diff = (Tg.astype(np.float64) - To)
    rel = np.abs(diff.data) / np.maximum(np.abs(To[diff.nonzero()]).A1, 1e-300) if diff.nnz else np.zeros(0)
    same_pattern = (Tg != 0).astype(np.int8) - (To != 0).astype(np.int8)
    n_pattern = same_pattern.count_nonzero()
    Pg = m.proj.cpu().numpy().astype(np.float64)
    say(f"{prob.name}: nnz gpu {m.nnz} oracle {To.nnz}, pattern diffs {n_pattern}, flipped {n_flip}/{n_tal}, "
        f"max rel value diff on shared entries {np.max(rel[rel < 0.5]) if np.any(rel < 0.5) else 0:.2e}")
    assert n_pattern <= 2 * n_flip
    assert np.sum(np.abs(Pg - Po)) <= 2 * n_flip
    To_f = To.copy()
    shared = To_f.multiply(Tg != 0)
    Tg_s = Tg.multiply(To != 0).astype(np.float64)
    d = np.abs((Tg_s - shared).data)
    assert d.size == 0 or np.max(d / np.abs(shared.data)) <= 1e-6 * (1 + 2 * n_flip)
    # MLEM from S0 = 1 on both sides
    img = torch.ones(m.n_img, dtype=torch.float32, device="cuda")
    mc.Mlem(m).run(img, n_iter)
    g = img.cpu().numpy().astype(np.float64)
    o = oracle.mlem(To, Po, n_iter)
    rl2 = np.linalg.norm(g - o) / np.linalg.norm(o)
    mask = o > 0.01 * o.max()
    mrel = np.max(np.abs(g[mask] - o[mask]) / o[mask]) if mask.any() else 0.0
    say(f"{prob.name}: MLEM {n_iter} it: rel L2 {rl2:.2e}, max rel above 1% {mrel:.2e}")
    assert rl2 <= 1e-4 + 3 * np.sqrt(n_flip / max(n_tal, 1))
    return m


def test_system_matrix_small_thorax():
    p = phantoms.thorax_problem("sm_thorax", 32, 1.2, 2, 12, 180.0, 32, 1.2, 2_000_000,
                                image_factor=4).with_(accept_half_angle_rad=np.radians(6.0))
    check_system_and_mlem(p, n_iter=30)


def test_system_matrix_thorax_256_subset():
    """The large workload's geometry (256^3 x 1.5 mm thorax, 120 views over 360
    degrees, 128^2 x 3 mm, 64^3 image) on the 1e7-history subset: history ids
    [0, ceil(1e7/120)) in every view."""
    V = 120
    n_per_view = -(-10 ** 7 // V)
    p = phantoms.thorax_256(V * n_per_view)
    check_system_and_mlem(p, n_iter=50, cap=1 << 21)


def _views_system(seed, n_views=24, bpv=60, n_vox=300, dens=0.02):
    T, n = phantoms.random_system(n_views * bpv, n_vox, dens, seed)
    sens = np.asarray(T.sum(axis=0)).ravel()
    return T, np.where(sens > 0, n, 0.0), bpv


def test_osem_kernel_matches_oracle():
    mc = _mc()
    import torch
    T, n, bpv = _views_system(51)
    Ts, _, _ = _views_system(52)
    rng = np.random.Generator(np.random.PCG64(53))
    T64, Ts64 = T.astype(np.float64), Ts.astype(np.float64)
    P = rng.poisson((T64 + 0.3 * Ts64) @ n * 4).astype(np.float32)
    s = (0.3 * (Ts64 @ n)).astype(np.float32)
    c = mc.csr_from_scipy(T)
    b = mc.csr_from_scipy((T64 * 0.9).astype(np.float32))
    Pg = torch.as_tensor(P, device="cuda")
    sg = torch.as_tensor(s, device="cuda")
    cases = [("osem", dict(), dict()),
             ("dm-os", dict(b=b), dict(b=(T64 * 0.9).astype(np.float32).astype(np.float64))),
             ("os+scatter", dict(scatter=sg), dict(scatter=s.astype(np.float64)))]
    for name, kg, ko in cases:
        img = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
        mc.osem(c, img, 6, 4, bpv, proj=Pg, **kg)
        g = img.cpu().numpy().astype(np.float64)
        o = oracle.osem(T64, P.astype(np.float64), 6, 4, bpv, **ko)
        m_ = o > 1e-6 * o.max()
        rel = np.max(np.abs(g[m_] - o[m_]) / o[m_])
        say(f"{name}: max rel {rel:.2e}")
        assert rel <= 1e-6


def test_osem_one_subset_equals_mlem_kernel():
    mc = _mc()
    import torch
    T, n, bpv = _views_system(54)
    rng = np.random.Generator(np.random.PCG64(55))
    P = torch.as_tensor(rng.poisson(T.astype(np.float64) @ n * 3).astype(np.float32), device="cuda")
    m = mc.csr_from_scipy(T)
    m.proj = P
    a = torch.ones(T.shape[1], dtype=torch.float32, device="cuda")
    b = a.clone()
    mc.Mlem(m).run(a, 9)
    mc.osem(m, b, 9, 1, bpv)
    np.testing.assert_allclose(b.cpu().numpy(), a.cpu().numpy(), rtol=1e-6)


def test_osem_subset_limit_and_entry_check():
    """At most 64 subsets (one wavefront lane per subset in the split of the
    backprojector); a wrong entry count of b leaves the image NaN."""
    mc = _mc()
    import torch
    T, n, bpv = _views_system(56)
    m = mc.csr_from_scipy(T)
    rng = np.random.Generator(np.random.PCG64(57))
    m.proj = torch.as_tensor(rng.poisson(T.astype(np.float64) @ n * 3).astype(np.float32), device="cuda")
    assert mc._lib.osem_workspace_bytes(m.n_bins, m.n_img, 65, m.nnz) == 0
    with pytest.raises(mc.McError):
        mc.osem(m, torch.ones(m.n_img, dtype=torch.float32, device="cuda"), 1, 65, bpv)
    nb = mc._lib.osem_workspace_bytes(m.n_bins, m.n_img, 4, m.nnz + 1)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    img = torch.ones(m.n_img, dtype=torch.float32, device="cuda")
    rc = mc._lib.osem_iterate(m.n_bins, m.n_img, bpv, 4, m.T_rowptr.data_ptr(), m.T_col.data_ptr(),
                              m.T_val.data_ptr(), m.Tt_rowptr.data_ptr(), m.Tt_col.data_ptr(),
                              m.Tt_val.data_ptr(), m.nnz + 1, m.proj.data_ptr(), None, img.data_ptr(), 2,
                              ws.data_ptr(), nb, mc._stream_ptr())
    assert rc == 0
    torch.cuda.synchronize()
    assert bool(torch.isnan(img).all())
    ok = torch.ones(m.n_img, dtype=torch.float32, device="cuda")
    mc.osem(m, ok, 2, 4, bpv)
    assert bool(torch.isfinite(ok).all())


def test_dual_matrix_and_scatter_forms_thorax():
    """Dual-matrix (backproject with the primary-only matrix) and additive
    scatter (primary matrix + scatter projection) forms on a thorax, GPU
    response matrices against the oracle's."""
    mc = _mc()
    import torch
    p = phantoms.thorax_problem("os_thorax", 32, 1.2, 2, 12, 180.0, 32, 1.2, 3_000_000,
                                image_factor=4).with_(accept_half_angle_rad=np.radians(6.0),
                                                      e_lo_kev=100.0)
    dp = mc.to_device(p)
    sim = mc.simulate(dp, event_capacity=1 << 20, want_sq=False)
    c = mc.system_matrix(dp, sim, "all")
    bp = mc.system_matrix(dp, sim, "primary")
    sc = mc.system_matrix(dp, sim, "scatter")
    oe = oracle.simulate(p, want_triplets=True, trip_cap=1 << 20)
    Co, Po, _ = oracle.system_matrix(p, oe["trip_i"], oe["trip_j"])
    Bo, _, _ = oracle.system_matrix(p, oe["trip_i"], oe["trip_j"], "primary")
    _, So, _ = oracle.system_matrix(p, oe["trip_i"], oe["trip_j"], "scatter")
    n_flip, n_tal = _flips(sim, oe)
    bpv = p.nv * p.nu
    assert sc.proj.sum().item() > 0
    for name, kg, ko in [("dm-os", dict(b=bp), dict(b=Bo)),
                         ("os+scatter", dict(scatter=sc.proj), dict(scatter=So))]:
        img = torch.ones(c.n_img, dtype=torch.float32, device="cuda")
        if name == "os+scatter":
            mc.osem(bp, img, 8, 4, bpv, proj=c.proj, **kg)
            o = oracle.osem(Bo, Po, 8, 4, bpv, **ko)
        else:
            mc.osem(c, img, 8, 4, bpv, **kg)
            o = oracle.osem(Co, Po, 8, 4, bpv, **ko)
        g = img.cpu().numpy().astype(np.float64)
        rl2 = np.linalg.norm(g - o) / np.linalg.norm(o)
        say(f"{name}: rel L2 {rl2:.2e}, flipped {n_flip}/{n_tal}")
        assert rl2 <= 1e-4 + 3 * np.sqrt(n_flip / max(n_tal, 1))


def test_system_matrix_row_length_classes():
    """A hand-made weighted event list whose voxel rows range from 1 to
    20000 events (one with 12000 distinct columns, one with 20000 events over
    3000 columns) and whose bin rows repeat columns: long rows cross many
    radix tiles and runs of equal keys span tile boundaries.  The CSR matches
    the oracle's matrix from the same contributions (sums of Q31.32 weights,
    exact before the FP32 store)."""
    import types
    import torch
    mc = _mc()
    p = phantoms.thorax_problem("rowlen", 32, 1.2, 2, 4, 180.0, 64, 0.6, 4_000_000, image_factor=4)
    p = p.with_(activity=np.ones_like(p.activity))
    rng = np.random.Generator(np.random.PCG64(77))
    per = p.nv * p.nu
    n_bins_cls = p.n_views * 2 * per
    f, nx = p.image_factor, p.nx
    # phantom voxels inside image voxels 0, 1, 2 and a few others
    def phantom_voxel(img):
        mx, my = nx // f, p.ny // f
        ix, iy, iz = img % mx, (img // mx) % my, img // (mx * my)
        return ((iz * f) * p.ny + iy * f) * nx + ix * f
    lengths = {0: 3000, 1: 6000, 2: 20000, 3: 20, 5: 1, 100: 700, 200: 12000}
    emit, bins = [], []
    for img, n in lengths.items():
        emit.append(np.full(n, phantom_voxel(img), dtype=np.uint32))
        if img == 2:      # many repeats: 20000 entries over 3000 bins
            b = rng.choice(n_bins_cls, size=3000, replace=False)[rng.integers(0, 3000, size=n)]
        elif img == 200:  # 12000 distinct bin rows: more than the LDS table holds
            rowsel = rng.choice(n_bins_cls // 2, size=n, replace=False)
            b = (rowsel // per) * 2 * per + rng.integers(0, 2, size=n) * per + rowsel % per
        else:
            b = rng.integers(0, n_bins_cls, size=n)
        bins.append(np.asarray(b).astype(np.uint32))
    emit = np.concatenate(emit)
    bins = np.concatenate(bins)
    w = rng.integers(1, 1 << 34, size=len(bins)).astype(np.int64)
    perm = rng.permutation(len(bins))
    emit, bins, w = emit[perm], bins[perm], w[perm]
    ev = np.zeros(len(bins), dtype=mc.EVENT_DTYPE)
    ev["work"] = np.arange(len(bins))
    ev["bin"], ev["emit_voxel"], ev["weight"] = bins, emit, w
    cap = len(ev)
    raw = torch.from_numpy(ev.view(np.int64).reshape(cap, 3).copy()).cuda()
    sim = types.SimpleNamespace(events=raw, event_capacity=cap,
                                n_events=torch.tensor([cap], dtype=torch.int64, device="cuda"))
    m = mc.system_matrix(mc.to_device(p), sim)
    Tg = m.to_scipy().astype(np.float64)
    mx = nx // f
    img_of = lambda v: ((v % nx) // f) + mx * (((v // nx) % p.ny) // f + (p.ny // f) * ((v // (nx * p.ny)) // f))
    To, Po, _ = oracle.system_matrix(p, img_of(emit.astype(np.int64)), bins.astype(np.int64),
                                     trip_w=w.astype(np.float64) / 2.0 ** 32)
    assert Tg.nnz == To.nnz
    Tt = m.to_scipy(transpose=True).astype(np.float64)
    assert abs(Tt - To.T.tocsr()).max() <= 1e-6 * abs(To).max()
    d = abs(Tg - To)
    assert d.max() <= 1e-6 * abs(To).max()
    np.testing.assert_allclose(m.proj.cpu().numpy(), Po, rtol=1e-6)
    rows = np.diff(m.Tt_rowptr.cpu().numpy())
    say(f"voxel row nnz: {[int(rows[k]) for k in lengths]}")
    for img, n in lengths.items():
        assert rows[img] == len(np.unique(bins[emit == phantom_voxel(img)] // (2 * per) * per
                                          + bins[emit == phantom_voxel(img)] % per))


@pytest.mark.parametrize("case", ["empty", "over_capacity", "garbage_tail", "primary", "scatter",
                                  "one_key", "reverse_sorted"])
def test_system_matrix_list_edges(case):
    """Event-list edge cases of the response-matrix build against the oracle:
    an empty list (every row pointer 0, P = 0); a device-side count above the
    capacity (the binding raises; through the C ABI every value and P_j is
    NaN: a list that lost events gives no matrix); slots past the count
    holding garbage (never read); the primary-only and scatter-only classes;
    every event on one (voxel, bin) key (one run across all radix tiles); a
    list in descending key order."""
    import types
    import torch
    mc = _mc()
    p = phantoms.thorax_problem("edges", 32, 1.2, 4, 4, 360.0, 16, 0.6, 1_000_000, image_factor=2)
    p = p.with_(activity=np.ones_like(p.activity))
    per = p.nv * p.nu
    n_bins_cls = p.n_views * 2 * per
    rng = np.random.Generator(np.random.PCG64(91))
    n_ev = 0 if case == "empty" else 50_000
    emit = rng.integers(0, p.nx * p.ny * p.nz, size=n_ev).astype(np.uint32)
    bins = rng.integers(0, n_bins_cls, size=n_ev).astype(np.uint32)
    w = rng.integers(1, 1 << 34, size=n_ev).astype(np.int64)
    if case == "one_key":
        emit[:], bins[:] = emit[0], bins[0]
    if case == "reverse_sorted":
        order = np.lexsort((emit, bins))[::-1]
        emit, bins, w = emit[order], bins[order], w[order]
    cap = {"empty": 1000, "over_capacity": 30_000, "garbage_tail": 80_000}.get(case, n_ev)
    ev = np.zeros(cap, dtype=mc.EVENT_DTYPE)
    used = min(n_ev, cap)
    ev["bin"][:used], ev["emit_voxel"][:used], ev["weight"][:used] = bins[:used], emit[:used], w[:used]
    if case == "garbage_tail":       # out-of-range bins and voxels past the count
        ev["bin"][n_ev:] = 0xFFFFFFF0
        ev["emit_voxel"][n_ev:] = 0xFFFFFFF0
        ev["weight"][n_ev:] = -1
    raw = torch.from_numpy(ev.view(np.int64).reshape(cap, 3).copy()).cuda()
    sim = types.SimpleNamespace(events=raw, event_capacity=cap,
                                n_events=torch.tensor([n_ev], dtype=torch.int64, device="cuda"))
    classes = case if case in ("primary", "scatter") else "all"
    if case == "over_capacity":
        import ctypes as C
        with pytest.raises(mc.McError, match="lost events"):
            mc.system_matrix(mc.to_device(p), sim)
        dp = mc.to_device(p)
        arr = dp.c_struct()
        nb = mc._lib.mc_system_matrix_workspace_bytes(C.byref(arr), cap)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        n_bins, n_img = p.n_views * p.nv * p.nu, (p.nx // 2) * (p.ny // 2) * (p.nz // 2)
        T_rp = torch.empty(n_bins + 1, dtype=torch.int64, device="cuda")
        Tt_rp = torch.empty(n_img + 1, dtype=torch.int64, device="cuda")
        T_col, Tt_col = (torch.empty(cap, dtype=torch.int32, device="cuda") for _ in range(2))
        T_val, Tt_val = (torch.empty(cap, dtype=torch.float32, device="cuda") for _ in range(2))
        proj = torch.empty(n_bins, dtype=torch.float32, device="cuda")
        rc = mc._lib.mc_system_matrix(C.byref(arr), raw.data_ptr(), sim.n_events.data_ptr(), cap, 3,
                                      T_rp.data_ptr(), T_col.data_ptr(), T_val.data_ptr(),
                                      Tt_rp.data_ptr(), Tt_col.data_ptr(), Tt_val.data_ptr(),
                                      proj.data_ptr(), ws.data_ptr(), nb, mc._stream_ptr())
        assert rc == mc.MC_OK
        nnz = int(T_rp[-1].item())
        assert nnz > 0 and int(Tt_rp[-1].item()) == nnz
        assert torch.isnan(T_val[:nnz]).all() and torch.isnan(Tt_val[:nnz]).all()
        assert torch.isnan(proj).all()
        return
    m = mc.system_matrix(mc.to_device(p), sim, classes=classes)
    mx = p.nx // p.image_factor
    f = p.image_factor
    img_of = lambda v: ((v % p.nx) // f) + mx * (((v // p.nx) % p.ny) // f + (p.ny // f) * ((v // (p.nx * p.ny)) // f))
    To, Po, _ = oracle.system_matrix(p, img_of(emit[:used].astype(np.int64)), bins[:used].astype(np.int64),
                                     classes=classes, trip_w=w[:used].astype(np.float64) / 2.0 ** 32)
    Tg = m.to_scipy().astype(np.float64)
    Tt = m.to_scipy(transpose=True).astype(np.float64)
    say(f"{case}: {used} events, nnz {Tg.nnz} (oracle {To.nnz})")
    assert Tg.nnz == To.nnz and Tt.nnz == To.nnz
    if To.nnz:
        assert abs(Tg - To).max() <= 1e-6 * abs(To).max()
        assert abs(Tt - To.T.tocsr()).max() <= 1e-6 * abs(To).max()
    else:
        assert not m.T_rowptr.any().item() and not m.Tt_rowptr.any().item()
    np.testing.assert_allclose(m.proj.cpu().numpy(), Po, rtol=1e-6, atol=0)


def test_mlem_bin_slices_edges():
    """Bin-slice path (2^19 bins or more, 16+ entries per voxel row, more
    entries than bins and voxels together) with voxels no bin sees: those stay 0; n_iter = 0 returns S^0 masked by the
    sensitivity; a non-uniform S^0 is followed as in the oracle."""
    mc = _mc()
    import torch
    T, truth = phantoms.random_system(600_000, 2000, 6e-4, seed=41)
    T = T.tolil()
    T[:, 1500:1600] = 0.0                 # 100 voxels that no bin sees
    T = T.tocsr()
    T.eliminate_zeros()
    rng = np.random.Generator(np.random.PCG64(42))
    P = rng.poisson(T.astype(np.float64) @ truth * 20).astype(np.float32)
    S0 = rng.uniform(0.5, 2.0, size=T.shape[1]).astype(np.float32)
    m = mc.csr_from_scipy(T)
    m.proj = torch.as_tensor(P, device="cuda")
    ml = mc.Mlem(m)
    sens = np.asarray(T.sum(axis=0)).ravel()
    img0 = torch.as_tensor(S0.copy(), device="cuda")
    ml.run(img0, 0)
    np.testing.assert_array_equal(img0.cpu().numpy(), np.where(sens > 0, S0, 0.0).astype(np.float32))
    img = torch.as_tensor(S0.copy(), device="cuda")
    ml.run(img, 12)
    g = img.cpu().numpy().astype(np.float64)
    o = oracle.mlem(T.astype(np.float64), P.astype(np.float64), 12, S0=S0.astype(np.float64))
    assert np.all(g[1500:1600] == 0.0)
    msk = o > 1e-6 * o.max()
    rel = np.max(np.abs(g[msk] - o[msk]) / o[msk])
    say(f"bin slices with unseen voxels: max rel {rel:.2e}")
    assert rel <= 1e-6
