"""Pins for the FP64 oracle: closed forms, published values, library routines,
invariants.  None of these calls the GPU library.

Each test fixes a part of the oracle against something other than the oracle
itself, so that a dropped term, a wrong sign or index, or a transposed operand
anywhere in it fails at least one of them.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import integrate, optimize, stats

import oracle
import phantoms

HERE = os.path.dirname(os.path.abspath(__file__))
MEC2 = 510.99895
R_E_CM = 2.8179403262e-13  # classical electron radius (CODATA 2018)


def binom_z(k, n, p):
    return (k - n * p) / math.sqrt(n * p * (1 - p))


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(oracle.philox(ctr, key)) == out


_ROCRAND_SRC = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        const unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        const unsigned long long off = ((unsigned long long)c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, sub, off * 4ull);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host_engine():
    """rocRAND's Philox4x32-10 engine, run on the host, as a library reference.
    The engine's counter is (offset/4 in words 0-1, subsequence in words 2-3)."""
    rng = np.random.Generator(np.random.PCG64(11))
    n = 256
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 30) - 1  # keep offset*4 inside 64 bits
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "ref.cpp")
        exe = os.path.join(d, "ref")
        with open(src, "w") as f:
            f.write(_ROCRAND_SRC)
        subprocess.check_call(["hipcc", "-O1", src, "-o", exe])
        inp = "\n".join(" ".join("%x" % int(x) for x in list(ctr[i]) + list(key[i]))
                        for i in range(n)) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == n
    for i in range(n):
        assert list(oracle.philox(ctr[i], key[i])) == ref[i]


# ---------------------------------------------------------------------------
# Uniform conversion: all 2^23 values
# ---------------------------------------------------------------------------

def test_uniform_all_values():
    m = np.arange(1 << 23, dtype=np.uint32)
    u = oracle.uniform_array(m << np.uint32(9))
    assert u.min() > 0.0 and u.max() < 1.0
    assert np.all(np.diff(u) > 0)                              # strictly increasing
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)  # exact in FP32
    np.testing.assert_array_equal(u + u[::-1], 1.0)            # symmetric about 1/2
    assert u.sum() == (1 << 22)                                # mean exactly 1/2
    # the low 9 bits are ignored
    assert oracle.uniform(0x1FF) == oracle.uniform(0)


# ---------------------------------------------------------------------------
# Klein-Nishina
# ---------------------------------------------------------------------------

def kn_pdf_cos(c, k):
    """Klein-Nishina dsigma/dOmega in units of r_e^2 (textbook form)."""
    P = 1.0 / (1.0 + k * (1.0 - c))
    return 0.5 * P * P * (P + 1.0 / P - (1.0 - c * c))


@pytest.mark.parametrize("e", [20.0, 71.0, 126.0, 140.0, 154.0, 167.0, 511.0])
def test_kn_total_matches_integral(e):
    k = e / MEC2
    num, _ = integrate.quad(kn_pdf_cos, -1.0, 1.0, args=(k,), epsabs=0, epsrel=1e-13)
    # kn_total is in units of 2 pi r_e^2; the integral over cos is sigma / (2 pi r_e^2)
    assert oracle.kn_total(e) == pytest.approx(num, rel=1e-10)


def test_kn_total_140_in_barns():
    sigma_b = oracle.kn_total(140.0) * 2 * math.pi * R_E_CM ** 2 / 1e-24
    assert sigma_b == pytest.approx(0.4522955, abs=2e-6)
    # low-energy (Thomson) limit: sigma/sigma_T = 1 - 2k + 26/5 k^2 - 133/10 k^3 + ...
    k = 1.0 / MEC2
    assert oracle.kn_total(1.0) == pytest.approx(4.0 / 3.0 * (1 - 2 * k + 5.2 * k * k),
                                                 rel=20 * k ** 3)


def test_attenuation_shape():
    f = 1e-3
    assert oracle.g_of_e(140.0, f) == pytest.approx(1.0, rel=1e-14)
    assert oracle.p_pe(140.0, f) == pytest.approx(f, rel=1e-14)
    # photoelectric share grows towards low energy, Compton share follows KN
    assert oracle.p_pe(70.0, f) > oracle.p_pe(140.0, f)
    ratio = oracle.g_of_e(126.0, 0.0)
    assert ratio == pytest.approx(0.465338 / 0.452295, rel=2e-6)


def _kahn_acceptance(k):
    a1 = (1 + 2 * k) / (9 + 2 * k)
    e1 = integrate.quad(lambda x: 4 * (1 / x - 1 / x ** 2), 1, 1 + 2 * k)[0] / (2 * k)
    norm2 = 1 - 1 / (1 + 2 * k)

    def f2(x):
        c = 1 - (x - 1) / k
        return 0.5 * (c * c + 1 / x) / x ** 2
    e2 = integrate.quad(f2, 1, 1 + 2 * k)[0] / norm2
    return a1 * e1 + (1 - a1) * e2


def test_kahn_sampler_distribution():
    e = 140.0
    k = e / MEC2
    n = 200_000
    x, attempts = oracle.kahn_samples(e, n, seed=3)
    assert np.all(np.isfinite(x))
    assert np.all((x >= 1.0) & (x <= 1 + 2 * k))
    # Compton relation E' = E / (1 + k (1 - cos)), so cos = 1 - (x - 1)/k
    cos = 1.0 - (x - 1.0) / k
    edges = np.linspace(-1, 1, 41)
    total = integrate.quad(kn_pdf_cos, -1, 1, args=(k,))[0]
    expected = np.array([integrate.quad(kn_pdf_cos, a, b, args=(k,))[0]
                         for a, b in zip(edges[:-1], edges[1:])]) / total
    counts, _ = np.histogram(cos, bins=edges)
    chi2 = np.sum((counts - n * expected) ** 2 / (n * expected))
    assert stats.chi2.sf(chi2, len(counts) - 1) > 1e-4
    mean_c = integrate.quad(lambda c: c * kn_pdf_cos(c, k), -1, 1)[0] / total
    assert mean_c == pytest.approx(0.149397, abs=2e-6)
    sd = math.sqrt(integrate.quad(lambda c: c * c * kn_pdf_cos(c, k), -1, 1)[0] / total
                   - mean_c ** 2)
    assert abs(cos.mean() - mean_c) < 5 * sd / math.sqrt(n)
    # P(E' >= 126 keV): scatter angle below the Compton edge of the window
    c0 = 1 - (140.0 / 126.0 - 1) / k
    p126 = integrate.quad(kn_pdf_cos, c0, 1, args=(k,))[0] / total
    assert p126 == pytest.approx(0.335045, abs=2e-6)
    assert math.degrees(math.acos(c0)) == pytest.approx(53.527, abs=1e-3)
    frac = np.mean(x <= 140.0 / 126.0)
    assert abs(binom_z(frac * n, n, p126)) < 5
    # rejection efficiency of Kahn's method, derived independently
    acc = _kahn_acceptance(k)
    assert acc == pytest.approx(0.587, abs=0.005)
    assert abs(binom_z(n, attempts, acc)) < 5


@pytest.mark.parametrize("w", [0.3, -0.7, 0.999995, -0.9999999, 0.0])
def test_direction_rotation_is_a_rotation(w):
    rng = np.random.Generator(np.random.PCG64(21))
    a = rng.uniform(0, 2 * math.pi)
    s = math.sqrt(1 - w * w)
    d = np.array([s * math.cos(a), s * math.sin(a), w])
    # near the poles the rotation treats d as +-z exactly: error O(sqrt(1 - w^2))
    tol = 20 * math.sqrt(1 - w * w) if abs(w) > 0.99999 else 1e-12
    for cos_t in (0.9, 0.1, -0.6):
        sin_t = math.sqrt(1 - cos_t ** 2)
        phis = np.linspace(0, 2 * math.pi, 24, endpoint=False)
        out = np.array([oracle.rotate(d, cos_t, ph) for ph in phis])
        np.testing.assert_allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-12)
        np.testing.assert_allclose(out @ d, cos_t, atol=tol)
        perp = out - np.outer(out @ d, d)
        np.testing.assert_allclose(np.linalg.norm(perp, axis=1), sin_t, atol=max(tol, 1e-12))
        # equal steps in phi turn the perpendicular part by equal angles
        cosang = np.sum(perp * np.roll(perp, -1, axis=0), axis=1) / sin_t ** 2
        np.testing.assert_allclose(cosang, math.cos(2 * math.pi / 24), atol=max(tol, 1e-10))
        # the perpendicular parts average out: the mean direction is cos_t * d
        np.testing.assert_allclose(out.mean(axis=0), cos_t * d, atol=max(tol, 1e-12))
        # right-handed about d (the near-pole branch turns about +z for either
        # pole, which mirrors the azimuth for d ~ -z: same uniform distribution)
        if abs(w) <= 0.99999 or w > 0:
            assert np.dot(np.cross(perp[0], perp[1]), d) > 0


# ---------------------------------------------------------------------------
# Transport closed forms
# ---------------------------------------------------------------------------

def _cone_primary_prob(alpha, mu_path):
    """P(emitted into the cone about +x and unattenuated) = 1/2 int exp(-mu_path/c) dc."""
    return 0.5 * integrate.quad(lambda c: math.exp(-mu_path / c), math.cos(alpha), 1.0)[0]


def test_geometric_efficiency_vacuum():
    n = 16
    mu = np.zeros((n, n, n), np.float32)
    act = np.zeros((n, n, n), np.uint32)
    act[n // 2, n // 2, n // 2] = 1
    alpha = math.radians(20.0)
    base = phantoms.point_source_cube("vac", n, 1.0, 200_000)
    p = base.with_(mu=mu, activity=act, accept_half_angle_rad=alpha)
    r = oracle.simulate(p)
    N = p.n_histories
    pexp = 0.5 * (1 - math.cos(alpha))
    tal = r["fates"][5]
    assert abs(binom_z(tal, N, pexp)) < 4
    assert r["fates"][2] + tal == N          # nothing else can happen in vacuum
    assert r["tally"][0, 1].sum() == 0       # no scatter
    # primaries land within D tan(alpha) of the detector centre
    iv, iu = np.nonzero(r["tally"][0, 0])
    uc = (iu + 0.5) * p.pixel_cm - 0.5 * p.nu * p.pixel_cm
    vc = (iv + 0.5) * p.pixel_cm - 0.5 * p.nv * p.pixel_cm
    assert np.max(np.hypot(uc, vc)) <= p.radius_cm * math.tan(alpha) + p.pixel_cm


@pytest.mark.parametrize("alpha_deg,N", [(20.0, 1_000_000), (2.0, 1_000_000)])
def test_narrow_beam_primaries_water_cube(alpha_deg, N):
    p = phantoms.point_cube_64(N).with_(accept_half_angle_rad=math.radians(alpha_deg))
    r = oracle.simulate(p)
    pexp = _cone_primary_prob(p.accept_half_angle_rad, 0.151 * 6.4)
    if alpha_deg == 2.0:
        assert pexp == pytest.approx(1.15846e-4, rel=1e-4)
    assert abs(binom_z(r["tally"][0, 0].sum(), N, pexp)) < 4


@pytest.mark.parametrize("extra_majorant", [False, True])
def test_woodcock_two_material_slab(extra_majorant):
    n, d = 64, 0.2
    mu, act = phantoms.slab_phantom(n, d, 0.3, 0.05, 40)   # interface at x = 1.6 cm
    if extra_majorant:
        mu[0, 0, 0] = 0.6   # far corner; doubles the majorant, must not change results
    alpha = math.radians(20.0)
    p = phantoms.point_cube_64(1_000_000).with_(mu=mu, activity=act, accept_half_angle_rad=alpha)
    r = oracle.simulate(p)
    pexp = _cone_primary_prob(alpha, 0.3 * 1.6 + 0.05 * 4.8)
    assert abs(binom_z(r["tally"][0, 0].sum(), p.n_histories, pexp)) < 4
    q, mh = oracle.thresholds(p)
    assert mh == pytest.approx(0.6 if extra_majorant else 0.3, rel=1e-7)
    assert q.max() == 1 << 24


def test_accept_thresholds():
    mu = np.array([0.0, 0.0453, 0.151, 0.27935, 1e-30, 0.151 * (1 + 2**-20)], np.float32)
    mu3 = np.zeros((1, 1, 6), np.float32)
    mu3[0, 0] = mu
    act = np.ones((1, 1, 6), np.uint32)
    p = phantoms.point_cube_64(10).with_(nx=6, ny=1, nz=1, mu=mu3, activity=act)
    q, mh = oracle.thresholds(p)
    assert mh == float(mu.max())
    q = q.reshape(-1)
    assert q[0] == 0 and q[4] == 1 and q[3] == 1 << 24
    # Q/2^24 brackets mu/mu_max from above by less than one step
    ratio = mu.astype(np.float64) / mh
    assert np.all(q / 2.0**24 >= ratio) and np.all(q / 2.0**24 - ratio <= 2.0**-24)


def test_photoelectric_branch_fraction():
    # every Compton scatter lowers E below 140 keV and is cut at once, so the
    # first real collision's branch is observed directly: P(absorbed) = p_pe(140) = f
    p = phantoms.point_source_cube("pe", 32, 0.5, 400_000, e_cut=140.0).with_(pe_fraction=0.3)
    r = oracle.simulate(p)
    a, c = r["fates"][0], r["fates"][1]
    assert abs(binom_z(a, a + c, 0.3)) < 4
    assert r["tally"].sum() == r["tally"][0, 0].sum()   # only primaries survive


def test_conservation_thorax():
    p = phantoms.thorax_problem("t", 32, 1.2, 2, 10, 180.0, 32, 1.2, 200_000).with_(e_cut_kev=10.0)
    r = oracle.simulate(p)
    assert r["fates"].sum() == p.n_histories == r["n_hist"]
    assert r["energy"][:3].sum() == pytest.approx(140.0 * p.n_histories, rel=1e-12)
    assert r["fates"][6] == 0
    assert r["tally"].sum() == r["fates"][5]
    np.testing.assert_array_equal(r["tally"], r["tally_sq"])   # analog weights are 1


def test_emission_multinomial():
    rng = np.random.Generator(np.random.PCG64(5))
    act = rng.integers(0, 6, size=(4, 4, 4)).astype(np.uint32)
    act[0, 0, 0] = 0
    mu = np.full((4, 4, 4), 0.1, np.float32)
    N = 200_000
    p = phantoms.point_cube_64(N).with_(nx=4, ny=4, nz=4, voxel_cm=1.0, mu=mu, activity=act,
                                        source_mode=phantoms.SOURCE_VOXELS)
    rec = oracle.replay(p, np.zeros(N, np.int32), np.arange(N, dtype=np.uint64))
    counts = np.bincount(rec["emit_voxel"], minlength=64)
    a = act.reshape(-1).astype(np.float64)
    assert np.all(counts[a == 0] == 0)
    e = N * a / a.sum()
    m = a > 0
    chi2 = np.sum((counts[m] - e[m]) ** 2 / e[m])
    assert stats.chi2.sf(chi2, m.sum() - 1) > 1e-4


def test_emission_cdf_toy():
    act = np.array([[[1, 0, 3]]], np.uint32)
    mu = np.full((1, 1, 3), 0.1, np.float32)
    N = 100_000
    p = phantoms.point_cube_64(N).with_(nx=3, ny=1, nz=1, voxel_cm=1.0, mu=mu, activity=act,
                                        source_mode=phantoms.SOURCE_VOXELS)
    rec = oracle.replay(p, np.zeros(N, np.int32), np.arange(N, dtype=np.uint64))
    c = np.bincount(rec["emit_voxel"], minlength=3)
    assert c[1] == 0 and c.sum() == N
    assert abs(binom_z(c[0], N, 0.25)) < 4


def test_resume_and_thread_independence():
    p = phantoms.thorax_problem("t", 32, 1.2, 2, 7, 180.0, 32, 1.2, 100_001)
    full = oracle.simulate(p, n_threads=3)
    one = oracle.simulate(p, n_threads=1)
    a = oracle.simulate(p.with_(history_offset=0, history_count=40_000))
    b = oracle.simulate(p.with_(history_offset=40_000, history_count=0))
    np.testing.assert_array_equal(full["tally"], one["tally"])
    np.testing.assert_array_equal(full["fates"], one["fates"])
    np.testing.assert_array_equal(full["tally"], a["tally"] + b["tally"])
    np.testing.assert_array_equal(full["fates"], a["fates"] + b["fates"])
    assert full["n_tent"] == a["n_tent"] + b["n_tent"]


def test_replay_agrees_with_simulate():
    p = phantoms.thorax_problem("t", 32, 1.2, 2, 5, 180.0, 32, 1.2, 50_000)
    r = oracle.simulate(p)
    N, V = p.n_histories, p.n_views
    views = np.concatenate([np.full(N // V + (k < N % V), k, np.int32) for k in range(V)])
    hists = np.concatenate([np.arange(N // V + (k < N % V), dtype=np.uint64) for k in range(V)])
    rec = oracle.replay(p, views, hists)
    np.testing.assert_array_equal(np.bincount(rec["fate"], minlength=8), r["fates"])
    t = rec[rec["fate"] == 5]
    tally = np.zeros(p.tally_shape)
    np.add.at(tally, (t["view"], t["cls"], t["iv"], t["iu"]), 1.0)
    np.testing.assert_array_equal(tally, r["tally"])



# ---------------------------------------------------------------------------
# Projection geometry (Sec. 3: a camera rotating about the axis)
# ---------------------------------------------------------------------------

def _geometry_problem():
    """A small off-centre voxel source in vacuum: 16^3 grid of 1 mm voxels,
    activity in voxel (ix, iy, iz) = (15, 1, 13), 2 degree cone, 16 x 16
    detector of 1 cm pixels, nine views over 180 degrees."""
    n, vox = 16, 0.1
    mu = np.zeros((n, n, n), np.float32)
    act = np.zeros((n, n, n), np.uint32)
    src_idx = (15, 1, 13)                     # (ix, iy, iz)
    act[src_idx[2], src_idx[1], src_idx[0]] = 1
    V = 9
    base = phantoms.point_source_cube("geom", n, vox, 9 * 400_000)
    p = base.with_(mu=mu, activity=act, source_mode=phantoms.SOURCE_VOXELS,
                   angles=phantoms.view_angles(V, 180.0), nu=16, nv=16, pixel_cm=1.0,
                   radius_cm=phantoms.detector_radius(n, n, vox),
                   accept_half_angle_rad=math.radians(2.0))
    centre = np.array([-0.5 * n * vox + (i + 0.5) * vox for i in src_idx])
    return p, centre


def _predicted_pixel(p, centre, theta, mirror_u=False, reverse=False, swap=False):
    """Closed-form landing pixel of a ray along the view normal n = (cos t,
    sin t, 0) from the voxel centre: u = (-sin t, cos t, 0) . x, v = z,
    bin = floor((u + W/2) / pixel); with the alternative conventions a
    plausible mistake would give."""
    t = -theta if reverse else theta
    u = -math.sin(t) * centre[0] + math.cos(t) * centre[1]
    if mirror_u:
        u = -u
    v = centre[2]
    iu = math.floor((u + 0.5 * p.nu * p.pixel_cm) / p.pixel_cm)
    iv = math.floor((v + 0.5 * p.nv * p.pixel_cm) / p.pixel_cm)
    return (iu, iv) if swap else (iv, iu)


def test_projection_geometry_off_centre_source():
    """Primaries of an off-centre source land, view by view, in the pixel the
    camera geometry predicts: the detector axis u_k = (-sin t_k, cos t_k, 0)
    rotating with the view, v along z, half-open bins from the detector edge.
    Views whose predicted landing point has more margin to a pixel edge than
    the largest spread (half the voxel's extent across u or v plus the cone's
    tilt over the flight to the plane) must see every tallied photon in that
    pixel.  A mirrored u axis, a reversed rotation sense or swapped (iu, iv)
    predict a different pixel in at least one checked view, so each would
    fail here."""
    p, c = _geometry_problem()
    r = oracle.simulate(p)
    tally = r["tally"]
    assert tally[:, 1].sum() == 0                      # vacuum: no scatter
    half = 0.5 * p.nx * p.voxel_cm
    t_max = p.radius_cm + half * math.sqrt(2)          # longest flight from the grid to the plane
    tilt = t_max * math.tan(p.accept_half_angle_rad)
    checked = 0
    alternatives = {"mirror_u": False, "reverse": False, "swap": False}
    for k, th in enumerate(p.angles):
        u = -math.sin(th) * c[0] + math.cos(th) * c[1]
        spread_u = 0.5 * p.voxel_cm * (abs(math.sin(th)) + abs(math.cos(th))) + tilt
        spread_v = 0.5 * p.voxel_cm + tilt
        fu = (u + 0.5 * p.nu * p.pixel_cm) / p.pixel_cm
        fv = (c[2] + 0.5 * p.nv * p.pixel_cm) / p.pixel_cm
        mu_ = min(fu - math.floor(fu), math.ceil(fu) - fu) * p.pixel_cm
        mv_ = min(fv - math.floor(fv), math.ceil(fv) - fv) * p.pixel_cm
        view = tally[k, 0]
        assert view.sum() > 50, k
        if mu_ <= spread_u or mv_ <= spread_v:
            continue
        checked += 1
        iv, iu = _predicted_pixel(p, c, th)
        nz = np.argwhere(view > 0)
        assert nz.tolist() == [[iv, iu]], (k, nz.tolist(), (iv, iu))
        for name in alternatives:
            if _predicted_pixel(p, c, th, **{name: True}) != (iv, iu):
                alternatives[name] = True
    assert checked >= 4, checked
    assert all(alternatives.values()), alternatives
    # about (1 - cos a)/2 of each view's photons pass the collimator
    per_view = tally[:, 0].sum(axis=(1, 2))
    pexp = 0.5 * (1 - math.cos(p.accept_half_angle_rad))
    n_view = p.n_histories // p.n_views
    assert np.all(np.abs((per_view - n_view * pexp) / math.sqrt(n_view * pexp)) < 5)

# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------

def test_adjoint_primary_scaling_closed_form():
    """Only primaries in the window (E exactly 140).  Scaling mu -> s mu:
    d lambda/ds = -N/2 int (mu h/c) exp(-mu h/c) dc; the estimator is
    sum_v mu_v dlambda/dmu_v."""
    N = 400_000
    alpha = math.radians(20.0)
    p = phantoms.point_source_cube("adj", 32, 0.4, N).with_(
        accept_half_angle_rad=alpha, e_lo_kev=140.0, e_hi_kev=140.0)
    G = np.ones(p.tally_shape)
    r = oracle.adjoint(p, G)
    est = float(np.sum(r["grad"] * p.mu.astype(np.float64)))
    mh = 0.151 * 6.4
    exp_ = -N * 0.5 * integrate.quad(lambda c: (mh / c) * math.exp(-mh / c), math.cos(alpha), 1)[0]
    k = r["fates"][5]
    assert k > 1000
    # per-history value is mu*h/c in [0.966, 1.03]: sd ~ sqrt(k)
    assert abs(est - exp_) < 4 * math.sqrt(k) * 1.0


def test_adjoint_matches_analog_crn_fd_on_scaling():
    """Independent of the likelihood-ratio machinery: re-simulate at mu*(1+-h)
    with the same random numbers and difference the primary counts."""
    N = 400_000
    alpha = math.radians(20.0)
    base = phantoms.point_source_cube("adj", 32, 0.4, N).with_(
        accept_half_angle_rad=alpha, e_lo_kev=140.0, e_hi_kev=140.0)
    h = 0.02
    lp = oracle.simulate(base.with_(mu=(base.mu * (1 + h)).astype(np.float32)))["tally"].sum()
    lm = oracle.simulate(base.with_(mu=(base.mu * (1 - h)).astype(np.float32)))["tally"].sum()
    fd = (lp - lm) / (2 * h)
    G = np.ones(base.tally_shape)
    est = float(np.sum(oracle.adjoint(base, G)["grad"] * base.mu.astype(np.float64)))
    # CRN difference counts histories whose fate flips: Poisson with mean ~ |fd|*2h
    sd = math.sqrt(abs(fd) * 2 * h) / (2 * h)
    assert abs(fd - est) < 4 * sd + 0.02 * abs(est)


def test_adjoint_gradient_matches_path_frozen_fd():
    N = 300_000
    p = phantoms.point_source_cube("adj", 32, 0.4, N).with_(accept_half_angle_rad=math.radians(10))
    ref = oracle.simulate(p.with_(seed=1))
    lam_ref = ref["tally"].sum(axis=1)
    y = phantoms.poisson_target(lam_ref, seed=4)
    fwd = oracle.simulate(p)
    lam = fwd["tally"].sum(axis=1)
    eps = 1e-6 * lam.max()
    _, dl = oracle.poisson_loss_grad(lam, y, eps)
    G = np.repeat(dl[:, None], 2, axis=1)
    r0 = oracle.adjoint(p, G)
    cand = np.flatnonzero(r0["n_contrib"].reshape(-1) >= 50)
    assert len(cand) >= 16
    vox = phantoms.pick(4, cand, 16)
    r = oracle.adjoint(p, G, pert_voxels=vox, delta=1e-3, lam=lam, y=y, eps=eps)
    g = r["grad"].reshape(-1)[vox]
    fd = r["fd"]
    scale = np.maximum(np.abs(fd), 1e-2 * np.abs(fd).max())
    assert np.all(np.abs(g - fd) <= 1e-5 * scale), (g, fd)
    np.testing.assert_array_equal(r["grad"], r0["grad"])


def _replay_all(prob):
    N, V = prob.n_histories, prob.n_views
    views = np.concatenate([np.full(N // V + (k < N % V), k, np.int32) for k in range(V)])
    hists = np.concatenate([np.arange(N // V + (k < N % V), dtype=np.uint64) for k in range(V)])
    return oracle.replay(prob, views, hists), views, hists


def _tally_key(rec):
    """Per history: its bin if tallied, else -1."""
    b = ((rec["view"].astype(np.int64) * 2 + rec["cls"]) * 10_000 + rec["iv"]) * 10_000 + rec["iu"]
    return np.where(rec["fate"] == 5, b, -1)


def test_adjoint_with_scatter_matches_analog_crn_fd_on_scaling():
    """Scattered photons in the window (100-154 keV): under mu -> s mu the
    likelihood-ratio estimate sum_v mu_v dlambda/dmu_v, which now includes
    the Compton-vertex term c_v/mu_v, must match the central difference of
    analog runs at s = 1 +- h on the same random numbers.  The FD's error is
    set by the histories whose tally outcome differs between the two runs
    (counted exactly by replaying both); dropping the vertex term moves the
    estimate by the number of Compton vertices on tallied paths, many times
    that error."""
    N = 2_000_000
    alpha = math.radians(20.0)
    base = phantoms.point_source_cube("adjs", 32, 0.4, N).with_(
        accept_half_angle_rad=alpha, e_lo_kev=100.0, e_hi_kev=154.0, e_cut_kev=100.0)
    h = 0.1
    rp, _, _ = _replay_all(base.with_(mu=(base.mu * (1 + h)).astype(np.float32)))
    rm, _, _ = _replay_all(base.with_(mu=(base.mu * (1 - h)).astype(np.float32)))
    lp, lm = np.sum(rp["fate"] == 5), np.sum(rm["fate"] == 5)
    fd = (lp - lm) / (2 * h)
    n_diff = int(np.sum(_tally_key(rp) != _tally_key(rm)))
    G = np.ones(base.tally_shape)
    r = oracle.adjoint(base, G)
    est = float(np.sum(r["grad"] * base.mu.astype(np.float64)))
    T = r["fates"][5]
    # the vertex term alone: +1 per Compton vertex of every tallied path
    rec0, _, _ = _replay_all(base)
    vertices = float(np.sum(rec0["n_scatter"][rec0["fate"] == 5]))
    sd_fd = math.sqrt(n_diff) / (2 * h)
    # per tallied history |c - mu lt| <= max(n_scatter, mu * longest path (g <= 1.2)) ~ 3
    sd_est = 3.0 * math.sqrt(T)
    bias = 0.01 * abs(fd)             # O(h^2) curvature of exp(-s mu L): (mu L)^2 h^2 / 6 < 1 %
    tol = 4 * (sd_fd + sd_est) + bias
    assert np.sum(rec0["n_scatter"][rec0["fate"] == 5] > 0) > 0.15 * T     # scatter is in the window
    assert abs(fd - est) < tol, (fd, est, tol)
    assert vertices > 1.5 * tol, (vertices, tol)


def test_adjoint_list_matches_full_adjoint():
    """The gradient over an explicit list of histories: over every history it
    is the full gradient; over two halves it adds up; the returned bins agree
    with the replay records."""
    N = 60_000
    p = phantoms.thorax_problem("adjl", 32, 1.2, 2, 6, 180.0, 32, 1.2, N)
    rng = np.random.Generator(np.random.PCG64(8))
    G = rng.uniform(-1, 1, p.tally_shape)
    full = oracle.adjoint(p, G)["grad"]
    rec, views, hists = _replay_all(p)
    g_all, bins = oracle.adjoint_list(p, G, views, hists)
    np.testing.assert_allclose(g_all, full, rtol=1e-9, atol=1e-12 * np.abs(full).max())
    want = np.where(rec["fate"] == 5,
                    ((rec["view"].astype(np.int64) * 2 + rec["cls"]) * p.nv + rec["iv"]) * p.nu + rec["iu"],
                    -1)
    np.testing.assert_array_equal(bins, want)
    half = len(views) // 2
    a, _ = oracle.adjoint_list(p, G, views[:half], hists[:half])
    b, _ = oracle.adjoint_list(p, G, views[half:], hists[half:])
    np.testing.assert_allclose(a + b, full, rtol=1e-9, atol=1e-12 * np.abs(full).max())


# ---------------------------------------------------------------------------
# MLEM (Sec. 5.1, Eq. MLEM)
# ---------------------------------------------------------------------------

def _rand_T(rng, nb, nv, dens):
    import scipy.sparse as sp
    T = sp.random(nb, nv, density=dens, random_state=np.random.RandomState(1), format="csr")
    T.data = rng.uniform(0.1, 1.0, size=T.nnz)
    return T


def test_mlem_fixed_point_and_conservation():
    rng = np.random.Generator(np.random.PCG64(8))
    T = _rand_T(rng, 300, 120, 0.05)
    n = rng.uniform(0.5, 3.0, size=120)
    sens = np.asarray(T.sum(axis=0)).ravel()
    n[sens == 0] = 0
    P = T @ n
    S = oracle.mlem(T, P, 5, S0=n)
    np.testing.assert_allclose(S, n, rtol=1e-12)
    Pn = rng.poisson(P * 10) / 10.0
    S = None
    for k in range(1, 6):
        S = oracle.mlem(T, Pn, k)
        y = T @ S
        # sum_i sens_i S_i = sum of P over bins with positive reprojection
        assert np.dot(sens, S) == pytest.approx(Pn[(T @ oracle.mlem(T, Pn, k - 1)) > 0].sum(), rel=1e-12)


def test_mlem_monotone_likelihood():
    rng = np.random.Generator(np.random.PCG64(9))
    T = _rand_T(rng, 200, 80, 0.08)
    truth = rng.uniform(0, 5, size=80)
    P = rng.poisson(T @ truth).astype(np.float64)
    ll = [oracle.poisson_loglik(T, P, oracle.mlem(T, P, k)) for k in range(0, 30)]
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[-1]))


def test_mlem_one_voxel():
    import scipy.sparse as sp
    T = sp.csr_matrix(np.array([[0.2], [0.5], [0.0], [0.3]]))
    P = np.array([3.0, 7.0, 2.0, 4.0])
    S = oracle.mlem(T, P, 1, S0=np.array([17.0]))
    assert S[0] == pytest.approx((3 + 7 + 4) / 1.0, rel=1e-14)   # sum P over seen bins / sum T


def test_mlem_small_toy_vs_constrained_maximiser():
    import scipy.sparse as sp
    A = np.array([[0.6, 0.1], [0.3, 0.5], [0.1, 0.4]])   # 3 bins x 2 voxels
    P = np.array([5.0, 9.0, 4.0])
    T = sp.csr_matrix(A)
    S = oracle.mlem(T, P, 3000)

    def negll(s):
        y = A @ s
        return -(np.sum(P * np.log(y)) - np.sum(y))
    res = optimize.minimize(negll, x0=np.ones(2), bounds=[(1e-9, None)] * 2, method="L-BFGS-B",
                            options={"ftol": 1e-15, "gtol": 1e-12})
    np.testing.assert_allclose(S, res.x, rtol=1e-5)


def test_system_matrix_normalisation_and_fixed_point():
    """T n = P bin by bin with n_i the expected emissions per view (the
    self-consistent reading), and hence n is an MLEM fixed point."""
    V = 4
    p = phantoms.thorax_problem("sm", 16, 2.4, 2, V, 180.0, 16, 2.4, 400_000, image_factor=2).with_(
        accept_half_angle_rad=np.radians(15.0))
    r = oracle.simulate(p, want_triplets=True)
    T, P, frac = oracle.system_matrix(p, r["trip_i"], r["trip_j"])
    assert P.sum() == r["fates"][5]
    n = (p.n_histories / V) * frac            # N divisible by V: same count for every view
    np.testing.assert_allclose(T @ n, P, rtol=1e-12, atol=1e-12)
    S = oracle.mlem(T, P, 5, S0=n)
    seen = np.asarray(T.sum(axis=0)).ravel() > 0
    np.testing.assert_allclose(S[seen], n[seen], rtol=1e-10)
    # a row is a bin: its entries are counts over expected emissions
    i, j = r["trip_i"][0], r["trip_j"][0]
    row = (j // (2 * p.nv * p.nu)) * p.nv * p.nu + j % (p.nv * p.nu)
    c = np.sum((r["trip_i"] == i) & ((r["trip_j"] // (2 * p.nv * p.nu)) * p.nv * p.nu
                                     + r["trip_j"] % (p.nv * p.nu) == row))
    assert T[row, i] == pytest.approx(c / n[i], rel=1e-12)


def _views_system(seed, n_views=12, bpv=40, n_vox=90, dens=0.05):
    T, n = phantoms.random_system(n_views * bpv, n_vox, dens, seed)
    sens = np.asarray(T.sum(axis=0)).ravel()
    return T.astype(np.float64), np.where(sens > 0, n, 0.0), bpv


def test_osem_one_subset_is_mlem():
    T, n, bpv = _views_system(41)
    rng = np.random.Generator(np.random.PCG64(42))
    P = rng.poisson(T @ n * 5).astype(np.float64)
    np.testing.assert_allclose(oracle.osem(T, P, 7, 1, bpv), oracle.mlem(T, P, 7), rtol=1e-12)


def test_osem_fixed_point_and_subset_conservation():
    T, n, bpv = _views_system(43)
    P = T @ n
    S = oracle.osem(T, P, 3, 4, bpv, S0=n)
    np.testing.assert_allclose(S, n, rtol=1e-10)
    # one subset update: sum_i sens_k,i S_i' = sum_{j in k, y_j > 0} P_j
    rng = np.random.Generator(np.random.PCG64(44))
    Pn = rng.poisson(P * 3).astype(np.float64) / 3
    S1 = oracle.osem(T, Pn, 1, 1, bpv)               # any positive start
    rows = np.flatnonzero((np.arange(T.shape[0]) // bpv) % 4 == 0)
    sens0 = np.asarray(T[rows].sum(axis=0)).ravel()
    y = T[rows] @ S1
    S2 = oracle.osem(T, Pn, 1, 4, bpv, S0=S1)         # first update of the pass is subset 0
    # isolate subset 0's update by running a one-pass, one-subset-only variant
    mask = np.zeros(T.shape[0])
    mask[rows] = 1
    Tk = T.multiply(mask[:, None]).tocsr()
    S_k = oracle.osem(Tk, Pn, 1, 4, bpv, S0=S1)
    upd = sens0 > 0
    assert np.dot(sens0[upd], S_k[upd]) == pytest.approx(Pn[rows][y > 0].sum(), rel=1e-12)
    assert np.all(np.isfinite(S2))


def test_osem_additive_scatter_and_dual_matrix_reduce():
    T, n, bpv = _views_system(45)
    Ts, _, _ = _views_system(46)
    rng = np.random.Generator(np.random.PCG64(47))
    P = rng.poisson((T + 0.3 * Ts) @ n * 4).astype(np.float64)
    base = oracle.osem(T, P, 4, 3, bpv)
    np.testing.assert_allclose(oracle.osem(T, P, 4, 3, bpv, scatter=np.zeros(T.shape[0])), base, rtol=1e-12)
    np.testing.assert_allclose(oracle.osem(T, P, 4, 3, bpv, b=T), base, rtol=1e-12)
    # consistent data with an additive scatter term: n is a fixed point
    s = 0.3 * (Ts @ n)
    Pc = T @ n + s
    np.testing.assert_allclose(oracle.osem(T, Pc, 3, 3, bpv, scatter=s, S0=n), n, rtol=1e-10)


# ---------------------------------------------------------------------------
# Forced detection (Sec. 5.2)
# ---------------------------------------------------------------------------

def test_fd_angular_density_normalised_and_matches_kahn_sampler():
    """The angular density forced detection weights with integrates to one over
    the sphere and is the distribution Kahn's sampler draws from (chi-square of
    the sampler's cos(theta) against bin integrals of the density)."""
    for e in (20.0, 126.0, 140.0):
        norm = 2 * math.pi * integrate.quad(lambda c: oracle.kn_pdf(e, c), -1, 1,
                                            epsabs=0, epsrel=1e-12)[0]
        assert norm == pytest.approx(1.0, rel=1e-10)
    e, n = 140.0, 200_000
    k = e / MEC2
    x, _ = oracle.kahn_samples(e, n, seed=11)
    cos = 1.0 - (x - 1.0) / k
    edges = np.linspace(-1, 1, 51)
    expected = np.array([2 * math.pi * integrate.quad(lambda c: oracle.kn_pdf(e, c), a, b)[0]
                         for a, b in zip(edges[:-1], edges[1:])])
    counts, _ = np.histogram(cos, bins=edges)
    chi2 = np.sum((counts - n * expected) ** 2 / (n * expected))
    assert stats.chi2.sf(chi2, len(counts) - 1) > 1e-4


def test_fd_ray_integral_closed_forms():
    """Exact line integrals: mu times the distance to the exit face in the water
    cube, and the two lengths in a two-material slab."""
    rng = np.random.Generator(np.random.PCG64(12))
    p = phantoms.point_cube_64(10)
    H = 6.4
    mu_w = float(np.float32(0.151))
    for _ in range(20):
        x = rng.uniform(-H * 0.99, H * 0.99, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t_exit = min((math.copysign(H, d[a]) - x[a]) / d[a] for a in range(3))
        assert oracle.ray_integral(p, x, d) == pytest.approx(mu_w * t_exit, rel=1e-12)
    mu, act = phantoms.slab_phantom(64, 0.2, 0.3, 0.05, 40)     # interface at x = 1.6 cm
    ps = p.with_(mu=mu, activity=act)
    ma, mb = float(np.float32(0.3)), float(np.float32(0.05))
    for _ in range(20):
        x = np.array([rng.uniform(-6.3, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1)])
        d = np.array([1.0, rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)])
        d /= np.linalg.norm(d)
        t_exit = min((math.copysign(H, d[a]) - x[a]) / d[a] for a in range(3))
        t_if = (1.6 - x[0]) / d[0]
        want = ma * t_if + mb * (t_exit - t_if) if t_if < t_exit else ma * t_exit
        assert oracle.ray_integral(ps, x, d) == pytest.approx(want, rel=1e-12)


def test_fd_point_source_primaries_closed_form():
    """Point source in the water cube: each history's emission score is
    (1 - cos a)/2 exp(-mu h / cos b) with b uniform in the cone, whose mean is
    the narrow-beam closed form 1/2 int exp(-mu h / c) dc; the analog part of
    the run (fates, energies) is unchanged."""
    N = 200_000
    p = phantoms.point_cube_64(N)
    r = oracle.simulate_fd(p)
    a = oracle.simulate(p)
    alpha = p.accept_half_angle_rad
    pexp = _cone_primary_prob(alpha, 0.151 * 6.4)
    got = r["tally"][0, 0].sum() / N
    lo = 0.5 * (1 - math.cos(alpha)) * math.exp(-0.151 * 6.4 / math.cos(alpha))
    hi = 0.5 * (1 - math.cos(alpha)) * math.exp(-0.151 * 6.4)
    sd = (hi - lo) / math.sqrt(12 * N)          # spread of one history's score is below (hi-lo)/sqrt(12)
    assert abs(got - pexp) < 5 * sd + 1e-9 * pexp
    np.testing.assert_array_equal(r["fates"], a["fates"])
    np.testing.assert_allclose(r["energy"], a["energy"], rtol=1e-12)
    # primaries land within D tan(alpha) of the detector centre
    iv, iu = np.nonzero(r["tally"][0, 0])
    uc = (iu + 0.5) * p.pixel_cm - 0.5 * p.nu * p.pixel_cm
    vc = (iv + 0.5) * p.pixel_cm - 0.5 * p.nv * p.pixel_cm
    assert np.max(np.hypot(uc, vc)) <= p.radius_cm * math.tan(alpha) + p.pixel_cm


def _batch_totals(prob, n_batch, fd):
    """Per-class window totals of n_batch independent runs (Philox seeds
    100 + b), each covering every view."""
    out = []
    for b in range(n_batch):
        r = (oracle.simulate_fd if fd else oracle.simulate)(prob.with_(seed=100 + b))
        out.append([r["tally"][:, 0].sum(), r["tally"][:, 1].sum()])
    return np.array(out)


def test_fd_unbiased_against_analog():
    """Forced detection and analog transport estimate the same expected counts:
    a 32^3 thorax, 4 views, 15 degree cone, photoelectric share 0.3 at 140 keV
    (so the not-absorbed factor matters).  Per class, the two totals agree
    within 4 combined standard errors (batch means)."""
    base = phantoms.thorax_problem("fd_thorax", 32, 1.2, 2, 4, 180.0, 32, 1.2, 1)
    base = base.with_(accept_half_angle_rad=math.radians(15.0), pe_fraction=0.3,
                      e_lo_kev=100.0, e_cut_kev=100.0)
    na, nf = 500_000, 25_000           # histories per batch
    A = _batch_totals(base.with_(n_histories=na), 8, fd=False) / na
    F = _batch_totals(base.with_(n_histories=nf), 8, fd=True) / nf
    ma, mf = A.mean(0), F.mean(0)
    se = np.sqrt(A.var(0, ddof=1) / 8 + F.var(0, ddof=1) / 8)
    assert np.all(mf > 0) and np.all(ma > 0)
    assert np.all(np.abs(ma - mf) < 4 * se), (ma, mf, se)
    # forced detection's estimate is far tighter per history
    assert np.all(F.std(0) * math.sqrt(nf) < A.std(0) * math.sqrt(na))


def test_box_escape_shortcut_changes_only_step_counts():
    """The optional escape shortcut (a photon in a voxel outside the
    attenuation box, moving away from it, escapes at once) is exact: against
    the default plain walk every replayed history ends with the same fate,
    bin, scatter count and energy, tallies and fates are identical, and only
    the number of tentative collisions drops (here by a quarter)."""
    p = phantoms.thorax_problem("box", 48, 0.8, 2, 12, 180.0, 32, 1.2, 200_000)
    rng = np.random.Generator(np.random.PCG64(13))
    views = rng.integers(0, p.n_views, 20_000).astype(np.int32)
    hists = rng.integers(0, p.n_histories // p.n_views, 20_000).astype(np.uint64)
    a = oracle.replay(p, views, hists)
    ra = oracle.simulate(p)
    b = oracle.replay(p, views, hists, escape_shortcut=True)
    rb = oracle.simulate(p, escape_shortcut=True)
    for f in ("fate", "iu", "iv", "n_scatter", "emit_voxel", "cls", "e_final"):
        np.testing.assert_array_equal(a[f], b[f])
    assert np.all(b["n_tent"] <= a["n_tent"])
    np.testing.assert_array_equal(ra["tally"], rb["tally"])
    np.testing.assert_array_equal(ra["fates"], rb["fates"])
    assert rb["n_tent"] < 0.85 * ra["n_tent"]


def test_fd_response_matrix_consistency():
    """The forced-detection response matrix (weights = scores) reproduces its
    run's forced-detection projection (P = T n with n the expected emissions
    per image voxel), its projection equals the run's tally with the classes
    merged, and its sensitivity per image voxel agrees with the analog
    matrix's within the analog counting error."""
    p = phantoms.thorax_problem("fd_sys", 32, 1.2, 2, 6, 180.0, 32, 1.2, 40_000,
                                image_factor=4).with_(accept_half_angle_rad=math.radians(8.0))
    r = oracle.simulate_fd(p, want_triplets=True)
    T, P, frac = oracle.system_matrix(p, r["trip_i"], r["trip_j"], trip_w=r["trip_w"])
    np.testing.assert_allclose(P, r["tally"].sum(axis=1).reshape(-1), rtol=1e-12, atol=1e-18)
    per = p.nv * p.nu
    q, rem = divmod(p.n_histories, p.n_views)
    n_view = np.array([q + (k < rem) for k in range(p.n_views)], dtype=np.float64)
    TP = (T @ frac) * np.repeat(n_view, per)           # sum_i T_ij N_view(j) A_i / A
    np.testing.assert_allclose(TP, P, rtol=1e-9, atol=1e-15)
    assert T.nnz > 20 * len(np.unique(r["trip_i"]))      # dense compared with analog lists
    a = oracle.simulate(p.with_(n_histories=4_000_000), want_triplets=True)
    Ta, Pa, _ = oracle.system_matrix(p.with_(n_histories=4_000_000), a["trip_i"], a["trip_j"])
    sf = np.asarray(T.sum(axis=0)).ravel()
    sa = np.asarray(Ta.sum(axis=0)).ravel()
    # compare the total sensitivity (analog: ~1e4 counts, 1 % error)
    assert abs(sf.sum() - sa.sum()) < 4 * sa.sum() / math.sqrt(Pa.sum())


# ---------------------------------------------------------------------------
# Convolution-based forced detection (Sec. 5.2)
# ---------------------------------------------------------------------------

def test_cfd_collimator_response():
    """The depth-dependent response of the ideal cone collimator: normalised,
    symmetric, confined to the disk of radius d tan(alpha), and its encircled
    fraction follows the closed form (1 - cos atan(r/d)) / (1 - cos alpha)
    (uniform directions in the cone) to within the pixel discretisation."""
    a = math.radians(2.0)
    for d, pix in ((5.0, 0.6), (28.0, 0.6), (40.0, 0.3)):
        k = oracle.cfd_kernel(d, a, pix)
        assert k.sum() == pytest.approx(1.0, abs=1e-12)
        np.testing.assert_allclose(k, k[::-1, :], atol=1e-15)
        np.testing.assert_allclose(k, k.T, atol=1e-15)
        h = (k.shape[0] - 1) // 2
        yy, xx = np.mgrid[-h:h + 1, -h:h + 1] * pix
        r_near = np.hypot(np.maximum(np.abs(xx) - pix / 2, 0), np.maximum(np.abs(yy) - pix / 2, 0))
        assert np.all(k[r_near > d * math.tan(a) + 1e-12] == 0.0)
    d = 20.0
    rho = d * math.tan(a)
    for n_pix, tol in ((40, 0.05), (80, 0.025)):
        pix = rho / n_pix
        k = oracle.cfd_kernel(d, a, pix)
        h = (k.shape[0] - 1) // 2
        yy, xx = np.mgrid[-h:h + 1, -h:h + 1] * pix
        r = np.hypot(xx, yy)
        for f in (0.3, 0.6, 0.9):
            want = (1 - math.cos(math.atan(f * rho / d))) / (1 - math.cos(a))
            assert abs(k[r <= f * rho].sum() - want) <= tol * want


def test_cfd_point_source_closed_form():
    """Point source in the water cube: every history deposits the same
    primary weight (1 - cos a)/2 exp(-mu h) in one layer and pixel, so the
    primary projection is exactly N times that weight spread by the response
    at that layer's depth."""
    N = 20_000
    p = phantoms.point_cube_64(N)
    r = oracle.simulate_cfd(p, want_layers=True)
    w = 0.5 * (1 - math.cos(p.accept_half_angle_rad)) * math.exp(-float(np.float32(0.151)) * 6.4)
    lay = r["layers"][0, :, 0]
    nz = np.argwhere(lay != 0)
    assert len(nz) == 1
    l, iv, iu = nz[0]
    assert lay[l, iv, iu] == pytest.approx(N * w, rel=1e-12)
    assert l == int(math.floor(p.radius_cm / p.pixel_cm))
    k = oracle.cfd_kernel((l + 0.5) * p.pixel_cm, p.accept_half_angle_rad, p.pixel_cm)
    h = (k.shape[0] - 1) // 2
    proj = r["tally"][0, 0]
    np.testing.assert_allclose(proj[iv - h:iv + h + 1, iu - h:iu + h + 1], N * w * k, rtol=1e-12)
    assert proj.sum() == pytest.approx(N * w, rel=1e-12)


def test_cfd_agrees_with_forced_detection():
    """On the same histories CFD differs from forced detection only by taking
    the attenuation and angular density at the cone axis and the spread from
    the response: per class the totals agree to O(alpha^2) (here 3e-3), and
    the analog part of the run is unchanged."""
    p = phantoms.thorax_problem("cfd_thorax", 32, 1.2, 2, 12, 180.0, 32, 1.2, 100_000)
    c = oracle.simulate_cfd(p)
    f = oracle.simulate_fd(p)
    for k in range(2):
        assert c["tally"][:, k].sum() == pytest.approx(f["tally"][:, k].sum(), rel=3e-3)
    np.testing.assert_array_equal(c["fates"], f["fates"])


# --- reuse of photon tracks (Sec. 5.3): difference sources ------------------

def _rpt_problem(n_hist, seed=0, bias=0.0):
    p = phantoms.thorax_problem("rpt", 24, 1.6, 7, 6, 180.0, 24, 1.6, n_hist, seed=seed,
                                image_factor=1)
    new, prev = phantoms.estimate_pair(p.activity, 0.2, 11, bias=bias)
    return p, new, prev


def test_rpt_difference_source_structure():
    """A difference source draws its histories from |d| and signs each
    contribution by d at the emitting voxel: with a zero previous estimate it
    is the plain run; with a zero new one every contribution is negated
    (forced detection and CFD too); in general its tally equals the plain run
    on |d| (the same histories) with each tallied history's sign read from d."""
    p, new, prev = _rpt_problem(60_000)
    zero = np.zeros_like(new)
    plain = oracle.simulate(p.with_(activity=new))
    same = oracle.simulate(p.with_(activity=new, activity_prev=zero))
    neg = oracle.simulate(p.with_(activity=zero, activity_prev=new))
    for k in ("tally", "tally_sq", "fates", "energy"):
        np.testing.assert_array_equal(same[k], plain[k])
    np.testing.assert_array_equal(neg["tally"], -plain["tally"])
    np.testing.assert_array_equal(neg["tally_sq"], plain["tally_sq"])
    np.testing.assert_array_equal(neg["fates"], plain["fates"])
    for fn in (oracle.simulate_fd, oracle.simulate_cfd):
        a = fn(p.with_(activity=new))
        b = fn(p.with_(activity=zero, activity_prev=new))
        np.testing.assert_array_equal(b["tally"], -a["tally"])

    d = new.astype(np.int64) - prev.astype(np.int64)
    ref = oracle.simulate(p.with_(activity=np.abs(d).astype(np.uint32)), want_triplets=True)
    got = oracle.simulate(p.with_(activity=new, activity_prev=prev))
    sign = np.where(d.reshape(-1)[ref["trip_i"]] < 0, -1.0, 1.0)
    assert (sign < 0).any() and (sign > 0).any()
    expect = np.zeros(int(np.prod(p.tally_shape)))
    np.add.at(expect, ref["trip_j"], sign)
    np.testing.assert_array_equal(got["tally"].reshape(-1), expect)
    np.testing.assert_array_equal(got["tally_sq"], ref["tally_sq"])
    np.testing.assert_array_equal(got["fates"], ref["fates"])


def test_rpt_projection_identity():
    """The identity reuse of photon tracks rests on: the projection of the new
    estimate equals the projection of the previous one plus that of the
    difference.  With the projection of a source of total |activity| A from
    N histories over V views P = A V / N x tally, three independent forced-
    detection runs agree per class and per view within 5 standard errors
    (estimated from the sums of squared scores); the difference here is 10 %
    of the estimate on average with both signs present."""
    n = 240_000
    p, new, prev = _rpt_problem(n, bias=0.1)
    d = new.astype(np.int64) - prev.astype(np.int64)
    assert (d < 0).any() and (d > 0).any()
    runs = []
    for seed, kw, total in ((21, dict(activity=prev), prev.sum(dtype=np.int64)),
                            (22, dict(activity=new, activity_prev=prev), np.abs(d).sum()),
                            (23, dict(activity=new), new.sum(dtype=np.int64))):
        o = oracle.simulate_fd(p.with_(seed=seed, **kw))
        s = float(total) * p.n_views / n
        runs.append((s * o["tally"], s * s * o["tally_sq"]))
    (pp, vp), (pd, vd), (pn, vn) = runs
    for axis in ((0, 2, 3), (1, 2, 3)):      # per class, per view
        diff = pn.sum(axis=axis) - pp.sum(axis=axis) - pd.sum(axis=axis)
        se = np.sqrt(vn.sum(axis=axis) + vp.sum(axis=axis) + vd.sum(axis=axis))
        assert np.all(np.abs(diff) <= 5 * se), (diff / se)
    # the difference's projection is the ~10 % change, well resolved
    assert pd.sum() == pytest.approx(pn.sum() - pp.sum(), rel=0.2)
    assert pd.sum() > 10 * math.sqrt(vd.sum())


# --- coarse-grid scatter modelling (Sec. 5.4) --------------------------------

def test_cgsm_block_activity():
    """Block-summed source: equal to the reshape-and-sum of each block,
    repeated over the block; total f^3 times the original; f = 1 changes
    nothing; indivisible grids are refused."""
    rng = np.random.Generator(np.random.PCG64(3))
    act = rng.integers(0, 1000, size=(6, 4, 8)).astype(np.uint32)
    for f in (1, 2):
        b = oracle.block_activity(act, f)
        s = act.astype(np.uint64).reshape(6 // f, f, 4 // f, f, 8 // f, f).sum(axis=(1, 3, 5))
        np.testing.assert_array_equal(b[::f, ::f, ::f], s)
        np.testing.assert_array_equal(b, np.kron(s, np.ones((f, f, f), dtype=np.uint64)))
        assert int(b.sum()) == f ** 3 * int(act.sum(dtype=np.uint64))
    np.testing.assert_array_equal(oracle.block_activity(act, 1), act)
    with pytest.raises(ValueError):
        oracle.block_activity(act, 3)


def test_cgsm_expand_projection():
    """The expansion is scipy's linear interpolation on the coarse pixel
    centres (coordinates clamped to the outermost centres) divided by f^2;
    a constant stays constant (/f^2); a ramp along u is reproduced exactly
    between the outermost centres; f = 1 is the identity."""
    from scipy.interpolate import RegularGridInterpolator
    rng = np.random.Generator(np.random.PCG64(5))
    c = rng.uniform(0.0, 10.0, size=(3, 2, 5, 7))
    for f in (1, 2, 3):
        e = oracle.expand_projection(c, f)
        assert e.shape == (3, 2, 5 * f, 7 * f)
        yc, xc = np.arange(5.0), np.arange(7.0)
        yf = np.clip((np.arange(5 * f) + 0.5) / f - 0.5, 0, 4)
        xf = np.clip((np.arange(7 * f) + 0.5) / f - 0.5, 0, 6)
        Y, X = np.meshgrid(yf, xf, indexing="ij")
        for v in range(3):
            for k in range(2):
                ref = RegularGridInterpolator((yc, xc), c[v, k])(np.stack([Y, X], -1)) / f ** 2
                np.testing.assert_allclose(e[v, k], ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(oracle.expand_projection(c, 1), c)
    const = np.full((1, 1, 4, 4), 8.0)
    np.testing.assert_allclose(oracle.expand_projection(const, 2), 2.0, rtol=0, atol=1e-15)
    ramp = np.tile(np.arange(6.0), (1, 1, 3, 1))
    e = oracle.expand_projection(ramp, 2)
    u = (np.arange(12) + 0.5) / 2 - 0.5
    inner = (u >= 0) & (u <= 5)
    np.testing.assert_allclose(e[0, 0, :, inner].T, np.tile(u[inner] / 4, (6, 1)), rtol=1e-14)


def test_cgsm_scatter_estimate():
    """Coarse-grid scatter: with f = 1 the coarse problem is the problem
    (identical tallies); with f = 2 the expanded forced-detection scatter
    projection from 1e6 histories lies closer (relative L2) to an 8e6-history
    fine reference than the fine estimate from the same 1e6 histories, with
    its total within 2 % (the smoothing the method relies on)."""
    p = phantoms.thorax_problem("cgsm", 32, 1.2, 2, 12, 180.0, 32, 1.2, 1_000_000, seed=9)
    a = oracle.simulate_fd(p.with_(n_histories=60_000))
    b = oracle.simulate_fd(oracle.coarse_problem(p.with_(n_histories=60_000), 1))
    np.testing.assert_array_equal(a["tally"], b["tally"])
    ref = oracle.simulate_fd(p.with_(n_histories=8_000_000, seed=5))["tally"][:, 1] / 8e6
    fine = oracle.simulate_fd(p)["tally"][:, 1] / 1e6
    cg = oracle.expand_projection(oracle.simulate_fd(oracle.coarse_problem(p, 2))["tally"], 2)[:, 1] / 1e6
    rl2 = lambda x: np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert rl2(cg) < 0.7 * rl2(fine), (rl2(cg), rl2(fine))
    assert cg.sum() == pytest.approx(ref.sum(), rel=0.02)


# --- emission lines (Sec. 3: Tl-201 at 71 and 167 keV) ----------------------

def _g_numeric(e, f_pe):
    """Attenuation at e relative to 140 keV from the numerically integrated
    Klein-Nishina cross-section and the E^-3 photoelectric term."""
    kn = lambda x: integrate.quad(kn_pdf_cos, -1.0, 1.0, args=(x / MEC2,), epsrel=1e-12)[0]
    return (1.0 - f_pe) * kn(e) / kn(140.0) + f_pe * (140.0 / e) ** 3


@pytest.mark.parametrize("e0", [71.0, 167.0])
def test_emission_line_narrow_beam(e0):
    """A point source emitting at e0 in the water cube: primaries counted in a
    window about e0 follow 1/2 int exp(-mu140 g(e0) h / c) dc with g from
    the integrated cross-section (20 degree cone)."""
    N = 400_000
    p = phantoms.point_cube_64(N).with_(e0_kev=e0, e_lo_kev=e0 - 10.0, e_hi_kev=e0 + 10.0,
                                        e_cut_kev=min(e0 - 10.0, 100.0),
                                        accept_half_angle_rad=math.radians(20.0), pe_fraction=0.02)
    r = oracle.simulate(p)
    g = _g_numeric(e0, 0.02)
    pexp = _cone_primary_prob(p.accept_half_angle_rad, float(np.float32(0.151)) * g * 6.4)
    assert abs(binom_z(r["tally"][0, 0].sum(), N, pexp)) < 4
    assert g == pytest.approx(oracle.g_of_e(e0, 0.02), rel=1e-9)


@pytest.mark.parametrize("e0", [71.0, 167.0])
def test_emission_line_branch_and_conservation(e0):
    """With the cut at the line energy every Compton scatter ends its history,
    so the first real collision's branch is observed: P(absorbed) =
    f (140/e0)^3 / g(e0); energies add up to e0 per history."""
    N = 300_000
    f = 0.05
    p = phantoms.point_source_cube("pe_line", 32, 0.5, N, e_cut=e0).with_(pe_fraction=f, e0_kev=e0,
                                                                          e_lo_kev=e0 - 5, e_hi_kev=e0 + 5)
    r = oracle.simulate(p)
    a, c = r["fates"][0], r["fates"][1]
    assert abs(binom_z(a, a + c, f * (140.0 / e0) ** 3 / _g_numeric(e0, f))) < 4
    q = phantoms.thorax_problem("t_line", 24, 1.6, 2, 6, 180.0, 24, 1.6, 100_000).with_(
        e0_kev=e0, e_cut_kev=20.0, e_lo_kev=0.9 * e0, e_hi_kev=1.1 * e0)
    s = oracle.simulate(q)
    assert s["energy"][:3].sum() == pytest.approx(e0 * q.n_histories, rel=1e-12)
    assert s["fates"].sum() == q.n_histories


def test_emission_line_limits():
    p = phantoms.point_cube_64(100)
    for bad in (dict(e0_kev=600.0), dict(e0_kev=80.0, e_cut_kev=90.0)):
        with pytest.raises(RuntimeError):
            oracle.simulate(p.with_(**bad))


# --- forced direction and forced interaction (Sec. 5.2) ---------------------

def test_forced_direction_vacuum_exact():
    """Forced direction into the acceptance cone in vacuum: every photon is
    detected as a primary with weight (1 - cos a)/2, so the tally total is
    N (1 - cos a) / 2 exactly (the analog geometric efficiency, without
    noise), and the sum of squared weights N ((1 - cos a)/2)^2."""
    N = 50_000
    a = math.radians(3.0)
    p = phantoms.point_cube_64(N).with_(mu=np.zeros((64, 64, 64), np.float32), accept_half_angle_rad=a,
                                        vr_flags=1, vr_cone_rad=a)
    r = oracle.simulate(p)
    w = 0.5 * (1.0 - math.cos(a))
    assert r["tally"][0, 0].sum() == pytest.approx(N * w, rel=1e-12)
    assert r["tally_sq"].sum() == pytest.approx(N * w * w, rel=1e-12)
    assert r["fates"][5] == N


def test_forced_direction_narrow_beam():
    """In the water cube the weighted primaries estimate 1/2 int exp(-mu h/c)
    dc over the cone, the analog closed form, to well within its small
    variance; a wider forcing cone (2 alpha) gives the same expectation."""
    N = 100_000
    a = math.radians(2.0)
    pexp = _cone_primary_prob(a, float(np.float32(0.151)) * 6.4)
    for beta in (a, 2 * a):
        p = phantoms.point_cube_64(N).with_(vr_flags=1, vr_cone_rad=beta)
        r = oracle.simulate(p)
        est = r["tally"][0, 0].sum() / N
        w = 0.5 * (1.0 - math.cos(beta))
        sd = math.sqrt(pexp * w / N)          # binomial in units of the weight
        assert abs(est - pexp) < 5 * sd + 1e-12, (beta, est, pexp)


def test_forced_interaction_unbiased():
    """Forced interaction replaces photoelectric absorption by the weight
    factor 1 - p_pe(E): no history is absorbed, and with a large
    photoelectric share (0.3) the weighted tally per class agrees with
    analog transport of independent histories within 5 standard errors."""
    base = phantoms.thorax_problem("fi", 24, 1.6, 2, 8, 180.0, 24, 1.6, 400_000).with_(
        pe_fraction=0.3, accept_half_angle_rad=math.radians(10.0), e_lo_kev=100.0, e_cut_kev=100.0)
    fi = oracle.simulate(base.with_(vr_flags=2, seed=31))
    an = oracle.simulate(base.with_(seed=32))
    assert fi["fates"][0] == 0
    for c in range(2):
        a, b = fi["tally"][:, c].sum(), an["tally"][:, c].sum()
        se = math.sqrt(fi["tally_sq"][:, c].sum() + an["tally_sq"][:, c].sum())
        assert abs(a - b) < 5 * se, (c, a, b, se)
    # the weights are products of (1 - p_pe) factors: below 1, above 0.7^k
    assert np.all(fi["tally_sq"] <= fi["tally"] + 1e-12)


def test_variance_reduction_refused_where_undefined():
    p = phantoms.point_cube_64(100)
    for bad in (dict(vr_flags=4), dict(vr_flags=1, vr_cone_rad=0.0)):
        with pytest.raises(RuntimeError):
            oracle.simulate(p.with_(**bad))
    with pytest.raises(RuntimeError):
        oracle.simulate_fd(p.with_(vr_flags=2))
