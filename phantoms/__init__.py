"""Seeded synthetic inputs: attenuation maps, activity maps, detector geometry.

This module is the one place where inputs are made.  Both the CPU oracle and the
GPU path read what it returns; it holds none of the transport arithmetic (no
cross sections, sampling, tracking or tallying) -- only the description of the
objects being imaged and of the camera, as plain arrays and numbers.

The paper images Tc-99m (140 keV, Sec. 3) in anthropomorphic thorax phantoms
(MCAT, XCAT, physical phantoms; Sec. 5.2-5.5).  None of those phantoms is
available here, so a project-defined thorax made of seeded ellipsoids stands in
for them (see ``thorax``).  Camera geometry follows the rotating
parallel-hole SPECT description of Sec. 3 (views over 180 or 360 degrees).

Conventions
-----------
* Arrays are ``[nz][ny][nx]`` with x fastest; lengths in cm; energies in keV.
* The voxel grid is centred on the origin; voxel (i, j, k) spans
  ``[-H + i*d, -H + (i+1)*d)`` on each axis with ``H = n*d/2``.
* mu is the linear attenuation coefficient at 140 keV in 1/cm (water 0.151).
* activity is a non-negative integer weight per voxel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MU_WATER_140 = 0.151  # 1/cm, water at 140 keV

# Source modes understood by both implementations.
SOURCE_VOXELS = 0  # emit from voxels in proportion to activity, uniform inside the voxel
SOURCE_POINT = 1   # emit from the grid centre exactly (activity still picks, and is ignored)


@dataclass
class Problem:
    """One emission problem: phantom + camera + history budget."""
    name: str
    nx: int
    ny: int
    nz: int
    voxel_cm: float
    mu: np.ndarray            # float32 [nz, ny, nx]
    activity: np.ndarray      # uint32  [nz, ny, nx]
    angles: np.ndarray        # float64 [n_views], radians
    nu: int
    nv: int
    pixel_cm: float
    radius_cm: float
    accept_half_angle_rad: float
    e_lo_kev: float
    e_hi_kev: float
    e_cut_kev: float
    n_histories: int
    seed: int = 0
    problem_id: int = 0
    source_mode: int = SOURCE_VOXELS
    image_factor: int = 0
    pe_fraction: float = 1.0e-3
    max_steps: int = 1000
    history_offset: int = 0
    history_count: int = 0    # 0 = all remaining histories
    # optional previous activity [nz, ny, nx] uint32: the source is then the
    # difference activity - activity_prev (signed)
    activity_prev: Optional[np.ndarray] = None
    e0_kev: float = 140.0     # emission line energy
    # variance reduction by weighting, for the oracle (the GPU library takes
    # these as call options): 1 forced direction, 2 forced interaction
    vr_flags: int = 0
    vr_cone_rad: float = 0.0

    @property
    def n_views(self) -> int:
        return int(self.angles.shape[0])

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def tally_shape(self):
        return (self.n_views, 2, self.nv, self.nu)

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


def detector_radius(nx: int, ny: int, voxel_cm: float) -> float:
    """Detector plane distance: circumscribed radius of the grid's xy square + 1 cm."""
    lx, ly = nx * voxel_cm, ny * voxel_cm
    return 0.5 * math.sqrt(lx * lx + ly * ly) + 1.0


def view_angles(n_views: int, arc_deg: float) -> np.ndarray:
    """theta_k = k * arc / V, k = 0..V-1 (camera rotation about z)."""
    return np.arange(n_views, dtype=np.float64) * (math.radians(arc_deg) / n_views)


def voxel_centres(n: int, voxel_cm: float) -> np.ndarray:
    return -0.5 * n * voxel_cm + (np.arange(n, dtype=np.float64) + 0.5) * voxel_cm


def water_cube(n: int, voxel_cm: float, mu: float = MU_WATER_140):
    """Uniform cube with one active voxel at the grid centre (n even)."""
    mu_map = np.full((n, n, n), mu, dtype=np.float32)
    act = np.zeros((n, n, n), dtype=np.uint32)
    act[n // 2, n // 2, n // 2] = 1
    return mu_map, act


# Reference thorax on a 38.4 cm grid (half-width 19.2 cm): centre, semi-axes,
# density, activity.  x lateral, +y posterior, z axial.  Painted in order; a
# later region overrides an earlier one.  Project-defined, not a published
# phantom.
_THORAX_REF_HALF = 19.2
_THORAX = [
    # name,      centre,            semi-axes,          rho,  activity
    ("body",     (0.0, 0.0, 0.0),   (16.0, 11.0, 24.0), 1.0,  1),
    ("lung_l",   (8.0, 1.0, 3.0),   (5.5, 7.5, 11.0),   0.3,  1),
    ("lung_r",   (-8.0, 1.0, 3.0),  (5.5, 7.5, 11.0),   0.3,  1),
    ("liver",    (-5.0, -1.0, -11.0), (8.0, 6.0, 5.0),  1.0,  4),
    ("lv_outer", (3.0, -3.5, 0.0),  (4.0, 3.5, 5.0),    1.0,  8),
    ("spine",    (0.0, 8.0, 0.0),   (1.8, 1.8, 24.0),   1.85, 1),
]
_LV_WALL_CM = 1.0


def thorax(n: int, voxel_cm: float, seed: int, jitter: float = 0.15):
    """Seeded ellipsoid thorax on an n^3 grid.

    Every semi-axis is multiplied by U(1-jitter, 1+jitter) from numpy PCG64(seed),
    drawn region by region in table order (3 draws each).  The LV cavity is the
    jittered outer shell shrunk by the 1 cm wall and has activity 1 (blood pool,
    same as background), so the myocardial wall is 8:1 against background and
    the liver 4:1.  Geometry is scaled by s = H / 19.2 cm.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    half = 0.5 * n * voxel_cm
    s = half / _THORAX_REF_HALF
    c = voxel_centres(n, voxel_cm)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    rho = np.zeros((n, n, n), dtype=np.float64)
    act = np.zeros((n, n, n), dtype=np.uint32)
    for name, ctr, axes, dens, a in _THORAX:
        f = rng.uniform(1.0 - jitter, 1.0 + jitter, size=3)
        ax = np.array(axes) * f * s
        cc = np.array(ctr) * s
        inside = (((x - cc[0]) / ax[0]) ** 2 + ((y - cc[1]) / ax[1]) ** 2
                  + ((z - cc[2]) / ax[2]) ** 2) < 1.0
        rho[inside] = dens
        act[inside] = a
        if name == "lv_outer":
            inner = ax - _LV_WALL_CM * s
            inside = (((x - cc[0]) / inner[0]) ** 2 + ((y - cc[1]) / inner[1]) ** 2
                      + ((z - cc[2]) / inner[2]) ** 2) < 1.0
            rho[inside] = 1.0
            act[inside] = 1
    mu = (MU_WATER_140 * rho).astype(np.float32)
    return mu, act


def slab_phantom(n: int, voxel_cm: float, mu_a: float, mu_b: float, split: int):
    """Two-material slab along x (planes of constant x); active voxel at grid centre."""
    mu = np.zeros((n, n, n), dtype=np.float32)
    mu[:, :, :split] = mu_a
    mu[:, :, split:] = mu_b
    act = np.zeros((n, n, n), dtype=np.uint32)
    act[n // 2, n // 2, n // 2] = 1
    return mu, act


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

WINDOW = (126.0, 154.0)
ALPHA_2DEG = math.radians(2.0)


def point_source_cube(name: str, n: int, voxel_cm: float, n_hist: int, seed: int = 0,
                      nu: int = 128, pixel_cm: float = 0.4, e_cut: float = 10.0) -> Problem:
    mu, act = water_cube(n, voxel_cm)
    return Problem(name=name, nx=n, ny=n, nz=n, voxel_cm=voxel_cm, mu=mu, activity=act,
                   angles=view_angles(1, 360.0), nu=nu, nv=nu, pixel_cm=pixel_cm,
                   radius_cm=detector_radius(n, n, voxel_cm),
                   accept_half_angle_rad=ALPHA_2DEG, e_lo_kev=WINDOW[0], e_hi_kev=WINDOW[1],
                   e_cut_kev=e_cut, n_histories=n_hist, seed=seed, source_mode=SOURCE_POINT)


def thorax_problem(name: str, n: int, voxel_cm: float, phantom_seed: int, n_views: int,
                   arc_deg: float, nu: int, pixel_cm: float, n_hist: int, seed: int = 0,
                   problem_id: int = 0, image_factor: int = 0) -> Problem:
    mu, act = thorax(n, voxel_cm, phantom_seed)
    return Problem(name=name, nx=n, ny=n, nz=n, voxel_cm=voxel_cm, mu=mu, activity=act,
                   angles=view_angles(n_views, arc_deg), nu=nu, nv=nu, pixel_cm=pixel_cm,
                   radius_cm=detector_radius(n, n, voxel_cm),
                   accept_half_angle_rad=ALPHA_2DEG, e_lo_kev=WINDOW[0], e_hi_kev=WINDOW[1],
                   e_cut_kev=WINDOW[0], n_histories=n_hist, seed=seed, problem_id=problem_id,
                   image_factor=image_factor)


def point_cube_64(n_hist: int = 10**6) -> Problem:
    """Point source at the centre of a 64^3 water cube, 2 mm voxels, one view."""
    return point_source_cube("point_cube_64", 64, 0.2, n_hist)


def thorax_128(n_hist: int = 10**8) -> Problem:
    """128^3 thorax at 3 mm, 60 views over 180 degrees, 64x64 pixels at 6 mm."""
    return thorax_problem("thorax_128", 128, 0.3, 2, 60, 180.0, 64, 0.6, n_hist)


def batched_thoraxes(n_hist_each: int = 10**7, n_problems: int = 32) -> List[Problem]:
    """32 thoraxes with grids U{96..160} at 3 mm and U{30..120} views over 180 degrees."""
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = rng.integers(96, 161, size=n_problems)
    views = rng.integers(30, 121, size=n_problems)
    out = []
    for p in range(n_problems):
        n = int(sizes[p])
        out.append(thorax_problem(f"thorax_batch_{p}", n, 0.3, 1000 + p, int(views[p]), 180.0,
                                  64, 0.6, n_hist_each, problem_id=p))
    return out


def point_cube_128_adjoint(n_hist: int = 10**7) -> Problem:
    """Adjoint workload: 128^3 x 1 mm water cube, centred point source, one view."""
    return point_source_cube("point_cube_128", 128, 0.1, n_hist)


def thorax_256(n_hist: int = 10**9) -> Problem:
    """256^3 thorax at 1.5 mm, 120 views over 360 degrees, 128x128 pixels at 3 mm."""
    return thorax_problem("thorax_256", 256, 0.15, 5, 120, 360.0, 128, 0.3, n_hist,
                          image_factor=4)


# Tl-201 (Sec. 3): photons at 71 and 167 keV.  Their relative yields
# (0.9 : 0.1) and the 20 % photopeak windows about each line are input choices.
TL201_LINES = ((71.0, 0.9), (167.0, 0.1))
TL201_WINDOWS = ((64.0, 78.0), (150.0, 184.0))


def line_window_problems(base: Problem, n_hist: int, lines=TL201_LINES,
                         windows=TL201_WINDOWS) -> List[Problem]:
    """A multi-line source acquired in several windows: one problem per (line,
    window), line-major.  Line k gets round(n_hist p_k / V) V histories and
    problem_id k, so all windows of a line see the same photons; the cut is
    the lowest window edge."""
    V = base.n_views
    e_cut = min(lo for lo, _ in windows)
    out = []
    for k, (e0, frac) in enumerate(lines):
        n_k = max(1, int(round(n_hist * frac / V))) * V
        for w, (lo, hi) in enumerate(windows):
            out.append(base.with_(name=f"{base.name}_l{k}_w{w}", e0_kev=e0, e_lo_kev=lo, e_hi_kev=hi,
                                  e_cut_kev=e_cut, n_histories=n_k, problem_id=k))
    return out


def estimate_pair(act: np.ndarray, rel: float, seed: int, scale: int = 1000, bias: float = 0.0):
    """Two successive image estimates for reuse of photon tracks: the previous
    one is act * scale, the new one that times (1 + bias + rel * U(-1, 1))
    voxel by voxel (numpy PCG64(seed)), rounded.  Returns (new, previous),
    uint32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prev = act.astype(np.float64) * scale
    new = np.rint(prev * (1.0 + bias + rel * rng.uniform(-1.0, 1.0, size=act.shape)))
    return new.astype(np.uint32), prev.astype(np.uint32)


def poisson_target(lam: np.ndarray, seed: int = 4) -> np.ndarray:
    """Seeded Poisson noise on an expected projection (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.poisson(lam).astype(np.float64)


def pick(rng_seed: int, candidates: np.ndarray, k: int) -> np.ndarray:
    """Seeded choice of k distinct entries from candidates (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    return np.sort(rng.choice(candidates, size=k, replace=False))


def random_system(n_bins: int, n_vox: int, density: float, seed: int):
    """Seeded sparse non-negative matrix (bins x voxels, float32 values) and a
    positive image, as scipy CSR and numpy arrays: a stand-in response matrix
    for reconstruction tests."""
    import scipy.sparse as sp
    rng = np.random.Generator(np.random.PCG64(seed))
    nnz = max(1, int(n_bins * n_vox * density))
    rows = rng.integers(0, n_bins, size=nnz)
    cols = rng.integers(0, n_vox, size=nnz)
    vals = rng.uniform(0.05, 1.0, size=nnz).astype(np.float32)
    T = sp.coo_matrix((vals, (rows, cols)), shape=(n_bins, n_vox)).tocsr()
    T.sum_duplicates()
    T.data = T.data.astype(np.float32)
    image = rng.uniform(0.5, 4.0, size=n_vox)
    return T, image
