"""FP64 CPU oracle (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does,
and it shares no code with the GPU library.

* ``simulate`` / ``replay`` / ``adjoint`` wrap the C++ transport oracle in
  ``mc_oracle.cpp`` (history-by-history photon transport, Sec. 2; rotating
  parallel-hole camera with photopeak window, Sec. 3).
* ``system_matrix`` turns the oracle's tallied (source voxel, bin) pairs into
  the Monte Carlo response matrix T_ij of Sec. 5.1, Eq. IMC.
* ``mlem`` is the update of Sec. 5.1, Eq. MLEM, written out in FP64.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FATES = ["ABSORBED", "CUT", "ESCAPED", "ESCAPED_FOV", "OUT_OF_WINDOW", "TALLIED", "CAPPED", "SPARE"]


def build(force: bool = True) -> str:
    """Compile the oracle with the system C++ compiler (no GPU code involved)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("source_mode", C.c_int32),
        ("voxel_cm", C.c_double),
        ("mu140", C.POINTER(C.c_float)), ("activity", C.POINTER(C.c_uint32)),
        ("n_views", C.c_int32), ("nu", C.c_int32), ("nv", C.c_int32), ("image_factor", C.c_int32),
        ("angle_rad", C.POINTER(C.c_double)),
        ("pixel_cm", C.c_double), ("radius_cm", C.c_double), ("accept_half_angle_rad", C.c_double),
        ("e_lo_kev", C.c_double), ("e_hi_kev", C.c_double), ("e_cut_kev", C.c_double),
        ("pe_fraction", C.c_double),
        ("n_histories", C.c_uint64), ("history_offset", C.c_uint64), ("history_count", C.c_uint64),
        ("seed", C.c_uint32), ("problem_id", C.c_uint32), ("max_steps", C.c_uint32),
        ("n_threads", C.c_uint32),
        ("activity_prev", C.POINTER(C.c_uint32)),
        ("e0_kev", C.c_double),
        ("vr_flags", C.c_int32), ("escape_shortcut", C.c_int32), ("vr_cone_rad", C.c_double),
    ]


class _Result(C.Structure):
    _fields_ = [("fates", C.c_int64 * 8), ("energy", C.c_double * 4),
                ("n_tent", C.c_int64), ("n_real", C.c_int64), ("n_kahn", C.c_int64),
                ("n_hist", C.c_int64)]


RECORD_DTYPE = np.dtype([("fate", np.int32), ("view", np.int32), ("iu", np.int32),
                         ("iv", np.int32), ("n_scatter", np.int32), ("n_tent", np.int32),
                         ("emit_voxel", np.int32), ("cls", np.int32), ("e_final", np.float64)])

_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)          # (re)builds a missing or stale library
        lib = C.CDLL(_LIB_PATH)
        P = C.POINTER
        lib.orc_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        lib.orc_uniform.argtypes = [C.c_uint32]
        lib.orc_uniform.restype = C.c_double
        lib.orc_uniform_array.argtypes = [P(C.c_uint32), C.c_uint64, P(C.c_double)]
        for f in ("orc_kn_total",):
            getattr(lib, f).argtypes = [C.c_double]
            getattr(lib, f).restype = C.c_double
        for f in ("orc_g", "orc_p_pe"):
            getattr(lib, f).argtypes = [C.c_double, C.c_double]
            getattr(lib, f).restype = C.c_double
        lib.orc_kahn_samples.argtypes = [C.c_double, C.c_uint32, C.c_uint64, P(C.c_double),
                                         P(C.c_int64)]
        lib.orc_rotate.argtypes = [P(C.c_double), C.c_double, C.c_double]
        lib.orc_thresholds.argtypes = [P(_Problem), P(C.c_uint32), P(C.c_double)]
        lib.orc_simulate.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(_Result),
                                     P(C.c_int64), P(C.c_int64), P(C.c_int64), C.c_uint64,
                                     P(C.c_uint64)]
        lib.orc_simulate_fd.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(_Result),
                                        P(C.c_int64), P(C.c_int64), P(C.c_double), P(C.c_int64),
                                        C.c_uint64, P(C.c_uint64)]
        lib.orc_simulate_cfd.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(_Result)]
        lib.orc_cfd_kernel.argtypes = [C.c_double, C.c_double, C.c_double, P(C.c_double), P(C.c_int32)]
        lib.orc_cfd_layers.argtypes = [P(_Problem)]
        lib.orc_cfd_layers.restype = C.c_int32
        lib.orc_kn_pdf.argtypes = [C.c_double, C.c_double]
        lib.orc_kn_pdf.restype = C.c_double
        lib.orc_ray_integral.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.orc_replay.argtypes = [P(_Problem), P(C.c_int32), P(C.c_uint64), C.c_int64, C.c_void_p]
        lib.orc_adjoint_list.argtypes = [P(_Problem), P(C.c_double), P(C.c_int32), P(C.c_uint64),
                                         C.c_int64, P(C.c_double), P(C.c_int64)]
        lib.orc_adjoint.argtypes = [P(_Problem), P(C.c_double), P(C.c_double), P(C.c_int64),
                                    C.c_int32, P(C.c_int32), C.c_double, P(C.c_double),
                                    P(C.c_double), C.c_double, P(C.c_double), P(_Result)]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return C.cast(None, C.POINTER(ct))
    return a.ctypes.data_as(C.POINTER(ct))


def _make_problem(prob, n_threads: int = 0, escape_shortcut: bool = False):
    """Marshal a phantoms.Problem into the C structure (keeps arrays alive).

    escape_shortcut: end a history at once when its tentative collision point
    lies outside the attenuation box and it moves away from it (exact in real
    arithmetic, fewer virtual steps).  Off by default: the oracle walks every
    history to the grid edge; only the step-count comparison with a kernel
    that takes the shortcut, and timing, switch it on."""
    mu = np.ascontiguousarray(prob.mu, dtype=np.float32)
    act = np.ascontiguousarray(prob.activity, dtype=np.uint32)
    ang = np.ascontiguousarray(prob.angles, dtype=np.float64)
    prev = (np.ascontiguousarray(prob.activity_prev, dtype=np.uint32)
            if getattr(prob, "activity_prev", None) is not None else None)
    p = _Problem(nx=prob.nx, ny=prob.ny, nz=prob.nz, source_mode=prob.source_mode,
                 voxel_cm=prob.voxel_cm, mu140=_ptr(mu, C.c_float), activity=_ptr(act, C.c_uint32),
                 n_views=prob.n_views, nu=prob.nu, nv=prob.nv, image_factor=prob.image_factor,
                 angle_rad=_ptr(ang, C.c_double), pixel_cm=prob.pixel_cm,
                 radius_cm=prob.radius_cm, accept_half_angle_rad=prob.accept_half_angle_rad,
                 e_lo_kev=prob.e_lo_kev, e_hi_kev=prob.e_hi_kev, e_cut_kev=prob.e_cut_kev,
                 pe_fraction=prob.pe_fraction, n_histories=prob.n_histories,
                 history_offset=prob.history_offset, history_count=prob.history_count,
                 seed=prob.seed, problem_id=prob.problem_id, max_steps=prob.max_steps,
                 n_threads=n_threads, activity_prev=_ptr(prev, C.c_uint32),
                 e0_kev=float(getattr(prob, "e0_kev", 140.0)),
                 vr_flags=int(getattr(prob, "vr_flags", 0)),
                 vr_cone_rad=float(getattr(prob, "vr_cone_rad", 0.0)),
                 escape_shortcut=1 if escape_shortcut else 0)
    return p, (mu, act, ang, prev)


def _result_dict(r: _Result):
    return {"fates": np.array(list(r.fates), dtype=np.int64),
            "energy": np.array(list(r.energy), dtype=np.float64),
            "n_tent": r.n_tent, "n_real": r.n_real, "n_kahn": r.n_kahn, "n_hist": r.n_hist}


# ---------------------------------------------------------------------------
# Small pieces
# ---------------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    lib = _load()
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib.orc_philox(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform(r: int) -> float:
    return _load().orc_uniform(int(r) & 0xFFFFFFFF)


def uniform_array(r: np.ndarray) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.uint32)
    out = np.empty(len(r), dtype=np.float64)
    _load().orc_uniform_array(_ptr(r, C.c_uint32), len(r), _ptr(out, C.c_double))
    return out


def kn_total(e_kev: float) -> float:
    """Klein-Nishina total cross-section per electron in units of 2 pi r_e^2."""
    return _load().orc_kn_total(float(e_kev))


def g_of_e(e_kev: float, f_pe: float) -> float:
    return _load().orc_g(float(e_kev), float(f_pe))


def p_pe(e_kev: float, f_pe: float) -> float:
    return _load().orc_p_pe(float(e_kev), float(f_pe))


def kahn_samples(e_kev: float, n: int, seed: int = 0):
    x = np.empty(n, dtype=np.float64)
    att = C.c_int64()
    _load().orc_kahn_samples(float(e_kev), seed, n, _ptr(x, C.c_double), C.byref(att))
    return x, att.value


def rotate(d, cos_t: float, phi: float) -> np.ndarray:
    v = (C.c_double * 3)(*[float(x) for x in d])
    _load().orc_rotate(v, float(cos_t), float(phi))
    return np.array(list(v))


def thresholds(prob):
    p, keep = _make_problem(prob)
    q = np.empty(prob.n_vox, dtype=np.uint32)
    mh = C.c_double()
    rc = _load().orc_thresholds(C.byref(p), _ptr(q, C.c_uint32), C.byref(mh))
    if rc != 0:
        raise ValueError("invalid problem")
    return q.reshape(prob.mu.shape), mh.value


# ---------------------------------------------------------------------------
# Transport
# ---------------------------------------------------------------------------

def simulate(prob, n_threads: int = 0, want_triplets: bool = False, trip_cap: int = 1 << 22,
             escape_shortcut: bool = False):
    """Forward simulation.  Returns dict with tally, tally_sq ([V,2,nv,nu], FP64),
    fates, energy (deposited, escaped, capped), counters and, if asked, per
    tallied history its image voxel of emission (trip_i), bin (trip_j) and work
    index relative to history_offset (trip_g)."""
    lib = _load()
    p, keep = _make_problem(prob, n_threads, escape_shortcut)
    tally = np.zeros(prob.tally_shape, dtype=np.float64)
    tsq = np.zeros(prob.tally_shape, dtype=np.float64)
    res = _Result()
    ti = tj = tg = None
    ntrip = C.c_uint64(0)
    if want_triplets:
        ti = np.empty(trip_cap, dtype=np.int64)
        tj = np.empty(trip_cap, dtype=np.int64)
        tg = np.empty(trip_cap, dtype=np.int64)
    rc = lib.orc_simulate(C.byref(p), _ptr(tally, C.c_double), _ptr(tsq, C.c_double),
                          C.byref(res), _ptr(ti, C.c_int64), _ptr(tj, C.c_int64),
                          _ptr(tg, C.c_int64), trip_cap if want_triplets else 0, C.byref(ntrip))
    if rc != 0:
        raise RuntimeError(f"orc_simulate failed ({rc})")
    out = _result_dict(res)
    out["tally"] = tally
    out["tally_sq"] = tsq
    if want_triplets:
        n = ntrip.value
        out["trip_i"] = ti[:n].copy()
        out["trip_j"] = tj[:n].copy()
        out["trip_g"] = tg[:n].copy()
    return out


def simulate_fd(prob, n_threads: int = 0, want_triplets: bool = False, trip_cap: int = 1 << 24):
    """Forced-detection forward simulation (Sec. 5.2): the analog histories'
    fates, energies and counters, and the forced-detection tally and the sum
    of squared scores ([V,2,nv,nu], FP64); with want_triplets, per nonzero
    score its image voxel of emission (trip_i), bin (trip_j), score (trip_w)
    and work index relative to history_offset (trip_g)."""
    lib = _load()
    p, keep = _make_problem(prob, n_threads)
    tally = np.zeros(prob.tally_shape, dtype=np.float64)
    tsq = np.zeros(prob.tally_shape, dtype=np.float64)
    res = _Result()
    ti = tj = tg = tw = None
    ntrip = C.c_uint64(0)
    if want_triplets:
        ti = np.empty(trip_cap, dtype=np.int64)
        tj = np.empty(trip_cap, dtype=np.int64)
        tg = np.empty(trip_cap, dtype=np.int64)
        tw = np.empty(trip_cap, dtype=np.float64)
    rc = lib.orc_simulate_fd(C.byref(p), _ptr(tally, C.c_double), _ptr(tsq, C.c_double),
                             C.byref(res), _ptr(ti, C.c_int64), _ptr(tj, C.c_int64),
                             _ptr(tw, C.c_double), _ptr(tg, C.c_int64),
                             trip_cap if want_triplets else 0, C.byref(ntrip))
    if rc != 0:
        raise RuntimeError(f"orc_simulate_fd failed ({rc})")
    out = _result_dict(res)
    out["tally"] = tally
    out["tally_sq"] = tsq
    if want_triplets:
        n = ntrip.value
        for k, a in (("trip_i", ti), ("trip_j", tj), ("trip_w", tw), ("trip_g", tg)):
            out[k] = a[:n].copy()
    return out


def simulate_cfd(prob, n_threads: int = 0, want_layers: bool = False):
    """Convolution-based forced detection (Sec. 5.2): the analog histories'
    fates, energies and counters; tally [V,2,nv,nu] from the depth layers
    convolved with the collimator response; with want_layers the deposits
    [V, L, 2, nv, nu]."""
    lib = _load()
    p, keep = _make_problem(prob, n_threads)
    L = lib.orc_cfd_layers(C.byref(p))
    tally = np.zeros(prob.tally_shape, dtype=np.float64)
    lay = np.zeros((prob.n_views, L, 2, prob.nv, prob.nu), dtype=np.float64) if want_layers else None
    res = _Result()
    if lib.orc_simulate_cfd(C.byref(p), _ptr(tally, C.c_double), _ptr(lay, C.c_double), C.byref(res)) != 0:
        raise RuntimeError("orc_simulate_cfd failed")
    out = _result_dict(res)
    out["tally"] = tally
    if want_layers:
        out["layers"] = lay
    return out


def cfd_kernel(depth_cm: float, alpha: float, pixel_cm: float) -> np.ndarray:
    """Collimator response at a depth, on the pixel grid ((2h+1) x (2h+1))."""
    lib = _load()
    h = C.c_int32(0)
    lib.orc_cfd_kernel(float(depth_cm), float(alpha), float(pixel_cm), None, C.byref(h))
    n = 2 * h.value + 1
    out = np.zeros((n, n), dtype=np.float64)
    lib.orc_cfd_kernel(float(depth_cm), float(alpha), float(pixel_cm), _ptr(out, C.c_double), C.byref(h))
    return out


def kn_pdf(e_kev: float, cos_t: float) -> float:
    """Klein-Nishina angular density per steradian at e_kev."""
    return _load().orc_kn_pdf(float(e_kev), float(cos_t))


def ray_integral(prob, x, d) -> float:
    """Integral of the 140 keV attenuation map from point x along unit d to
    the grid edge."""
    lib = _load()
    p, keep = _make_problem(prob)
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = C.c_double(0.0)
    if lib.orc_ray_integral(C.byref(p), _ptr(x, C.c_double), _ptr(d, C.c_double), C.byref(out)) != 0:
        raise RuntimeError("orc_ray_integral failed")
    return out.value


def replay(prob, views: np.ndarray, hists: np.ndarray, n_threads: int = 0,
           escape_shortcut: bool = False) -> np.ndarray:
    lib = _load()
    p, keep = _make_problem(prob, n_threads, escape_shortcut)
    views = np.ascontiguousarray(views, dtype=np.int32)
    hists = np.ascontiguousarray(hists, dtype=np.uint64)
    out = np.zeros(len(views), dtype=RECORD_DTYPE)
    rc = lib.orc_replay(C.byref(p), _ptr(views, C.c_int32), _ptr(hists, C.c_uint64),
                        len(views), out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise RuntimeError("orc_replay failed")
    return out


def adjoint(prob, G: np.ndarray, pert_voxels=None, delta: float = 1e-3, lam=None, y=None,
            eps: float = 0.0, n_threads: int = 0):
    """Path-frozen likelihood-ratio gradient and finite differences (FP64)."""
    lib = _load()
    p, keep = _make_problem(prob, n_threads)
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1)
    grad = np.zeros(prob.n_vox, dtype=np.float64)
    ncon = np.zeros(prob.n_vox, dtype=np.int64)
    res = _Result()
    npert = 0 if pert_voxels is None else len(pert_voxels)
    pv = None if pert_voxels is None else np.ascontiguousarray(pert_voxels, dtype=np.int32)
    fd = np.zeros(max(npert, 1), dtype=np.float64)
    lam_ = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    y_ = None if y is None else np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    rc = lib.orc_adjoint(C.byref(p), _ptr(G, C.c_double), _ptr(grad, C.c_double),
                         _ptr(ncon, C.c_int64), npert, _ptr(pv, C.c_int32), float(delta),
                         _ptr(lam_, C.c_double), _ptr(y_, C.c_double), float(eps),
                         _ptr(fd, C.c_double), C.byref(res))
    if rc != 0:
        raise RuntimeError("orc_adjoint failed")
    out = _result_dict(res)
    out["grad"] = grad.reshape(prob.mu.shape)
    out["n_contrib"] = ncon.reshape(prob.mu.shape)
    out["fd"] = fd[:npert]
    return out


def adjoint_list(prob, G: np.ndarray, views: np.ndarray, hists: np.ndarray, n_threads: int = 0):
    """The path-frozen gradient of sum_b G_b tally_b restricted to the listed
    (view, history id) pairs: each is replayed and, if tallied, adds
    G_b (c_{h,v}/mu0_v - lt_{h,v}).  Returns (grad [nz,ny,nx], bin of each
    listed history in the tally layout or -1 when it is not tallied)."""
    lib = _load()
    p, keep = _make_problem(prob, n_threads)
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1)
    views = np.ascontiguousarray(views, dtype=np.int32)
    hists = np.ascontiguousarray(hists, dtype=np.uint64)
    grad = np.zeros(prob.n_vox, dtype=np.float64)
    bins = np.empty(len(views), dtype=np.int64)
    rc = lib.orc_adjoint_list(C.byref(p), _ptr(G, C.c_double), _ptr(views, C.c_int32),
                              _ptr(hists, C.c_uint64), len(views), _ptr(grad, C.c_double),
                              _ptr(bins, C.c_int64))
    if rc != 0:
        raise RuntimeError("orc_adjoint_list failed")
    return grad.reshape(prob.mu.shape), bins


# ---------------------------------------------------------------------------
# Poisson loss of the adjoint workload, written out.
# ---------------------------------------------------------------------------

def poisson_loss_grad(lam: np.ndarray, y: np.ndarray, eps: float):
    """L = sum_b [lam_b - y_b ln(lam_b + eps)];  dL/dlam_b = 1 - y_b/(lam_b + eps)."""
    L = float(np.sum(lam - y * np.log(lam + eps)))
    return L, 1.0 - y / (lam + eps)


# ---------------------------------------------------------------------------
# Response matrix and MLEM (Sec. 5.1)
# ---------------------------------------------------------------------------

def system_matrix(prob, trip_i: np.ndarray, trip_j: np.ndarray, classes: str = "all",
                  trip_w: Optional[np.ndarray] = None):
    """Response matrix of Sec. 5.1 (Eq. IMC) from the tallied histories.

    T_ij = c_ij / n_i(j): c_ij tallied photons emitted in image voxel i and
    counted in projection bin j (primary and scattered alike: j = (view, iv,
    iu)) -- or, with trip_w, the summed forced-detection scores of those
    contributions -- n_i(j) = N_view(j) * A_i / A the expected number emitted in i towards
    bin j's view (A_i: activity summed over image voxel i, A: total).
    classes = "primary" / "scatter" keeps only unscattered / scattered
    photons (the dual-matrix backprojector, the scatter projection).  Returns
    (T as scipy CSR, rows = bins, FP64; P_j = sum_i c_ij; expected emissions
    n_i per view-averaged history count)."""
    import scipy.sparse as sp
    f = prob.image_factor
    mx, my, mz = prob.nx // f, prob.ny // f, prob.nz // f
    n_img = mx * my * mz
    act = prob.activity.astype(np.float64)
    a_img = act.reshape(mz, f, my, f, mx, f).sum(axis=(1, 3, 5)).reshape(-1)
    total = act.sum()
    V, per = prob.n_views, prob.nv * prob.nu
    n_bins = V * per
    cls = (trip_j // per) % 2
    keep = {"all": np.ones(len(trip_j), bool), "primary": cls == 0, "scatter": cls == 1}[classes]
    w = np.ones(len(trip_i)) if trip_w is None else np.asarray(trip_w, dtype=np.float64)
    trip_i, trip_j, w = trip_i[keep], trip_j[keep], w[keep]
    view = trip_j // (2 * per)
    row = view * per + trip_j % per
    n_view = np.array([prob.n_histories // V + (1 if k < prob.n_histories % V else 0)
                       for k in range(V)], dtype=np.float64)
    c = sp.coo_matrix((w, (row, trip_i)), shape=(n_bins, n_img)).tocsr()
    c.sum_duplicates()
    P = np.asarray(c.sum(axis=1)).ravel()
    c = c.tocoo()
    n_i = n_view[c.row // per] * a_img[c.col] / total
    T = sp.csr_matrix((c.data / n_i, (c.row, c.col)), shape=(n_bins, n_img))
    return T, P, a_img / total


def mlem(T, P: np.ndarray, n_iter: int, S0: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. MLEM: S_i <- S_i / sum_j T_ij * sum_m P_m T_im / (sum_l S_l T_lm).

    T is bins x voxels (scipy sparse, FP64).  Conventions: voxels no bin sees
    (sum_j T_ij = 0) stay 0; a bin whose reprojection is 0 contributes 0;
    S0 defaults to 1 on voxels with positive sensitivity."""
    T = T.tocsr().astype(np.float64)
    P = np.asarray(P, dtype=np.float64)
    sens = np.asarray(T.sum(axis=0)).ravel()
    seen = sens > 0
    S = np.where(seen, 1.0, 0.0) if S0 is None else np.where(seen, np.asarray(S0, np.float64), 0.0)
    for _ in range(n_iter):
        y = T @ S
        ratio = np.zeros_like(y)
        nz = y > 0
        ratio[nz] = P[nz] / y[nz]
        back = T.T @ ratio
        S = np.where(seen, S * back / np.where(seen, sens, 1.0), 0.0)
    return S


def osem(c, P: np.ndarray, n_iter: int, n_subsets: int, bins_per_view: int, b=None,
         scatter: Optional[np.ndarray] = None, S0: Optional[np.ndarray] = None) -> np.ndarray:
    """Ordered subsets, written out from Sec. 5.3 (Eq. DMOS) and Sec. 5.4
    (the Sohlberg OS-EM equation).  Subset k = views v with v mod n_subsets
    == k.  For each subset in order:
        y_j = sum_i c_ij S_i + s_j  (j in k)
        S_i <- S_i / sum_{j in k} b_ij * sum_{j in k} b_ij P_j / y_j
    b defaults to c (plain OSEM), s to 0; voxels with no weight in a subset
    keep their value; voxels no bin sees are 0."""
    c = c.tocsr().astype(np.float64)
    b = c if b is None else b.tocsr().astype(np.float64)
    P = np.asarray(P, dtype=np.float64)
    s = np.zeros(c.shape[0]) if scatter is None else np.asarray(scatter, dtype=np.float64)
    view = np.arange(c.shape[0]) // bins_per_view
    subset = view % n_subsets
    seen = np.asarray(b.sum(axis=0)).ravel() > 0
    S = np.where(seen, 1.0, 0.0) if S0 is None else np.where(seen, np.asarray(S0, np.float64), 0.0)
    for _ in range(n_iter):
        for k in range(n_subsets):
            rows = np.flatnonzero(subset == k)
            ck, bk = c[rows], b[rows]
            y = ck @ S + s[rows]
            ratio = np.zeros_like(y)
            nz = y > 0
            ratio[nz] = P[rows][nz] / y[nz]
            sens = np.asarray(bk.sum(axis=0)).ravel()
            back = bk.T @ ratio
            upd = sens > 0
            S = np.where(upd, S * back / np.where(upd, sens, 1.0), S)
    return S


def poisson_loglik(T, P: np.ndarray, S: np.ndarray) -> float:
    y = T @ S
    m = y > 0
    return float(np.sum(P[m] * np.log(y[m]) - y[m]))


# ---------------------------------------------------------------------------
# Coarse-grid scatter modelling (Sec. 5.4): the scatter projection is
# simulated with larger source voxels and larger detector pixels, then
# expanded and interpolated back to the normal pixel size.
# ---------------------------------------------------------------------------

def block_activity(act: np.ndarray, f: int) -> np.ndarray:
    """Source with f^3-voxel source voxels: every voxel takes the summed
    activity of its f x f x f block (so an emission is uniform over the
    block).  act [nz, ny, nx] with every axis a multiple of f; returns uint64."""
    nz, ny, nx = act.shape
    if nz % f or ny % f or nx % f:
        raise ValueError("grid not divisible by the coarsening factor")
    out = np.zeros(act.shape, dtype=np.uint64)
    a = act.astype(np.uint64)
    for bz in range(nz // f):
        for by in range(ny // f):
            zs, ys = slice(bz * f, (bz + 1) * f), slice(by * f, (by + 1) * f)
            for bx in range(nx // f):
                xs = slice(bx * f, (bx + 1) * f)
                out[zs, ys, xs] = a[zs, ys, xs].sum()
    return out


def expand_projection(coarse: np.ndarray, f: int) -> np.ndarray:
    """Coarse projection [..., nv_c, nu_c] -> [..., nv_c f, nu_c f]: each
    normal pixel takes the bilinear interpolation, at its centre, of the
    coarse values read as samples at the coarse pixel centres (held constant
    beyond the outermost centres), divided by f^2 (counts per normal pixel)."""
    c = np.asarray(coarse, dtype=np.float64)
    nvc, nuc = c.shape[-2:]
    out = np.zeros(c.shape[:-2] + (nvc * f, nuc * f))

    def weights(i, n_c):
        x = min(max((i + 0.5) / f - 0.5, 0.0), n_c - 1.0)
        i0 = int(math.floor(x))
        i1 = min(i0 + 1, n_c - 1)
        return i0, i1, x - i0

    for j in range(nvc * f):
        j0, j1, ty = weights(j, nvc)
        for i in range(nuc * f):
            i0, i1, tx = weights(i, nuc)
            out[..., j, i] = ((1 - ty) * ((1 - tx) * c[..., j0, i0] + tx * c[..., j0, i1])
                              + ty * ((1 - tx) * c[..., j1, i0] + tx * c[..., j1, i1])) / (f * f)
    return out


def coarse_problem(prob, f: int):
    """The problem CGSM simulates: block-summed source (block_activity, which
    must fit uint32), detector pixels f times larger (nu, nv multiples of f);
    attenuation, geometry and history budget unchanged."""
    act = block_activity(prob.activity, f)
    if act.max() > np.iinfo(np.uint32).max:
        raise ValueError("block activity exceeds 32 bits")
    if prob.nu % f or prob.nv % f:
        raise ValueError("detector not divisible by the coarsening factor")
    return prob.with_(activity=act.astype(np.uint32), nu=prob.nu // f, nv=prob.nv // f,
                      pixel_cm=prob.pixel_cm * f)
