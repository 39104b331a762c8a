"""Python binding of libmcspect (MI355X Monte Carlo SPECT transport).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libmcspect.so`` behind the C ABI declared in ``include/mcspect.h``.
PyTorch provides device memory and the current HIP stream.  If the library is
missing this module raises at import: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Union

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MCSPECT_LIB names another build of the same sources (the region-profile
# build of region_profile.py); by default the product library.
LIB_PATH = os.environ.get("MCSPECT_LIB") or os.path.join(_HERE, "libmcspect.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{os.path.basename(LIB_PATH)} not built at {LIB_PATH}; run paper_2105_13324_amd.build.build()")

# torch first: it loads its HIP runtime (soname libamdhip64.so.7), and the
# library's own dependency then binds to that same copy.  Two HIP runtimes in
# one process do not share devices.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

MC_OK, MC_EINVAL, MC_ENOMEM, MC_EDEVICE, MC_EOVERFLOW, MC_ECAPPED = 0, -1, -2, -3, -4, -5
STATUS_BAD_MU, STATUS_NO_ACTIVITY, STATUS_BAD_ANGLE, STATUS_LIST_OVERFLOW, STATUS_CAPPED = 1, 2, 4, 8, 16
STATUS_GRAD_OVERFLOW, STATUS_BAD_EVENT, STATUS_ACTIVITY_OVERFLOW, STATUS_TALLY_OVERFLOW = 32, 64, 128, 256
FATES = ["ABSORBED", "CUT", "ESCAPED", "ESCAPED_FOV", "OUT_OF_WINDOW", "TALLIED", "CAPPED", "SPARE"]
Q32 = float(2 ** 32)   # tally fixed point: Q31.32
Q23 = float(2 ** 23)   # energy fixed point: Q40.23 keV
Q52 = float(2 ** 52)   # forced-detection sum of squared scores: Q11.52

# Exported symbols, as declared in include/mcspect.h.
EXPORTS = ["mc_workspace_bytes", "mc_simulate_projections", "mc_simulate_projections_static",
           "mc_replay_histories",
           "mc_adjoint_mu", "mc_system_matrix_workspace_bytes", "mc_system_matrix",
           "mlem_workspace_bytes", "mlem_iterate", "mlem_prepare", "mlem_iterate_prepared",
           "osem_workspace_bytes", "osem_iterate",
           "mc_block_activity", "mc_expand_projection", "mc_source_total", "mc_scale_tally",
           "mc_graph_begin", "mc_graph_end", "mc_graph_launch", "mc_graph_destroy", "mc_autotune",
           "mc_check_status", "mc_error_string", "mc_last_hip_error"]


class McProblem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("source_mode", C.c_int32),
        ("voxel_cm", C.c_double),
        ("mu140", C.c_void_p), ("activity", C.c_void_p),
        ("n_views", C.c_int32), ("nu", C.c_int32), ("nv", C.c_int32),
        ("angle_rad", C.c_void_p),
        ("pixel_cm", C.c_double), ("radius_cm", C.c_double), ("accept_half_angle_rad", C.c_double),
        ("e_lo_kev", C.c_double), ("e_hi_kev", C.c_double), ("e_cut_kev", C.c_double),
        ("pe_fraction", C.c_double),
        ("n_histories", C.c_uint64), ("history_offset", C.c_uint64), ("history_count", C.c_uint64),
        ("seed", C.c_uint32), ("problem_id", C.c_uint32),
        ("image_factor", C.c_int32), ("max_steps", C.c_uint32),
        ("activity_prev", C.c_void_p),
        ("e0_kev", C.c_double),
    ]


class McOptions(C.Structure):
    _fields_ = [("hist_per_lane", C.c_int32), ("block_size", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("brick_log2", C.c_int32),
                ("threshold_bytes", C.c_int32), ("forced_detection", C.c_int32),
                ("kernel_events", C.c_void_p * 2),
                ("variance_reduction", C.c_int32), ("pad_vr", C.c_int32),
                ("forced_direction_half_angle_rad", C.c_double),
                ("reuse_staging", C.c_int32), ("pad_rs", C.c_int32)]


EVENT_DTYPE = np.dtype([("work", np.uint64), ("bin", np.uint32), ("emit_voxel", np.uint32),
                        ("weight", np.int64)])
RECORD_DTYPE = np.dtype([("fate", np.int32), ("view", np.int32), ("iu", np.int32), ("iv", np.int32),
                         ("n_scatter", np.int32), ("n_tent", np.int32), ("emit_voxel", np.int32),
                         ("cls", np.int32), ("e_final", np.float64)])
assert C.sizeof(McProblem) == 176

_vp, _i32, _i64, _u64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
_lib.mc_workspace_bytes.argtypes = [C.POINTER(McProblem), _i32, C.POINTER(McOptions)]
_lib.mc_workspace_bytes.restype = _sz
_lib.mc_simulate_projections.argtypes = [C.POINTER(McProblem), _i32, C.POINTER(McOptions),
                                         _vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp, _sz, _vp]
_lib.mc_simulate_projections.restype = C.c_int
_lib.mc_simulate_projections_static.argtypes = [C.POINTER(McProblem), _i32, C.POINTER(McOptions),
                                                _vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp]
_lib.mc_simulate_projections_static.restype = C.c_int
STATIC_SCRATCH_BYTES = 64 * 1024 * 1024   # MC_STATIC_SCRATCH_BYTES
_lib.mc_replay_histories.argtypes = [C.POINTER(McProblem), C.POINTER(McOptions), _vp, _vp, _i64,
                                     _vp, _vp, _vp, _sz, _vp]
_lib.mc_replay_histories.restype = C.c_int
_lib.mc_adjoint_mu.argtypes = [C.POINTER(McProblem), C.POINTER(McOptions), _vp, _vp, _vp, _u64,
                               _vp, C.c_int32, _vp, _vp, _sz, _vp]
_lib.mc_adjoint_mu.restype = C.c_int
_lib.mc_system_matrix_workspace_bytes.argtypes = [C.POINTER(McProblem), _u64]
_lib.mc_system_matrix_workspace_bytes.restype = _sz
_lib.mc_system_matrix.argtypes = [C.POINTER(McProblem), _vp, _vp, _u64, C.c_int32, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.osem_workspace_bytes.argtypes = [_i64, _i64, C.c_int32, _i64]
_lib.osem_workspace_bytes.restype = _sz
_lib.osem_iterate.argtypes = [_i64, _i64, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                              _vp, _vp, C.c_int32, _vp, _sz, _vp]
_lib.osem_iterate.restype = C.c_int
_lib.mc_system_matrix.restype = C.c_int
_lib.mlem_workspace_bytes.argtypes = [_i64, _i64]
_lib.mlem_workspace_bytes.restype = _sz
_lib.mlem_iterate.argtypes = [_i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp,
                              _sz, _vp]
_lib.mlem_iterate.restype = C.c_int
_lib.mlem_iterate_prepared.argtypes = _lib.mlem_iterate.argtypes
_lib.mlem_iterate_prepared.restype = C.c_int
_lib.mlem_prepare.argtypes = [_i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.mlem_prepare.restype = C.c_int
_lib.mc_block_activity.argtypes = [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp]
_lib.mc_block_activity.restype = C.c_int
_lib.mc_expand_projection.argtypes = [_vp, _i64, _i32, _i32, _i32, C.c_double, _vp, _vp]
_lib.mc_expand_projection.restype = C.c_int
_lib.mc_source_total.argtypes = [_vp, _vp, _i64, _vp, _vp]
_lib.mc_source_total.restype = C.c_int
_lib.mc_scale_tally.argtypes = [_vp, _i64, C.c_double, _vp, _i32, _vp]
_lib.mc_scale_tally.restype = C.c_int
_lib.mc_graph_begin.argtypes = [_vp]
_lib.mc_graph_begin.restype = C.c_int
_lib.mc_graph_end.argtypes = [_vp, C.POINTER(_vp)]
_lib.mc_graph_end.restype = C.c_int
_lib.mc_graph_launch.argtypes = [_vp, _vp]
_lib.mc_graph_launch.restype = C.c_int
_lib.mc_graph_destroy.argtypes = [_vp]
_lib.mc_graph_destroy.restype = C.c_int
_lib.mc_autotune.argtypes = [C.POINTER(McProblem), _i32, C.POINTER(McOptions), _i32, _i32, _vp, _vp, _vp,
                             _vp, _sz, _vp, C.POINTER(_i32), C.POINTER(C.c_float)]
_lib.mc_autotune.restype = C.c_int
_lib.mc_check_status.argtypes = [_vp, _vp]
_lib.mc_check_status.restype = C.c_int
_lib.mc_error_string.argtypes = [C.c_int]
_lib.mc_error_string.restype = C.c_char_p
_lib.mc_last_hip_error.argtypes = []
_lib.mc_last_hip_error.restype = C.c_int


class McError(RuntimeError):
    pass


class GradientOverflow(McError):
    """A term of the adjoint's fixed-point sums exceeded its range."""


def _check(rc: int, what: str):
    if rc != MC_OK:
        msg = _lib.mc_error_string(rc).decode()
        if rc == MC_EDEVICE:
            msg += f" (hip error {_lib.mc_last_hip_error()})"
        raise McError(f"{what}: {msg} ({rc})")


def _torch():
    import torch
    return torch


@dataclass
class DeviceProblem:
    """A problem whose arrays live on the GPU (torch tensors) plus its scalars."""
    nx: int
    ny: int
    nz: int
    voxel_cm: float
    mu: "object"          # torch.float32 [nz, ny, nx]
    activity: "object"    # torch.int32 view of uint32 [nz, ny, nx]
    angles: "object"      # torch.float64 [V]
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
    source_mode: int = 0
    image_factor: int = 0
    pe_fraction: float = 1e-3
    max_steps: int = 1000
    history_offset: int = 0
    history_count: int = 0
    activity_prev: Optional[object] = None   # device uint32 map: difference source
    e0_kev: float = 140.0                    # emission line energy

    @property
    def n_views(self) -> int:
        return int(self.angles.shape[0])

    @property
    def tally_shape(self):
        return (self.n_views, 2, self.nv, self.nu)

    def with_(self, **kw) -> "DeviceProblem":
        d = dict(self.__dict__)
        d.update(kw)
        return DeviceProblem(**d)

    def c_struct(self) -> McProblem:
        return McProblem(
            nx=self.nx, ny=self.ny, nz=self.nz, source_mode=self.source_mode,
            voxel_cm=self.voxel_cm, mu140=self.mu.data_ptr(), activity=self.activity.data_ptr(),
            n_views=self.n_views, nu=self.nu, nv=self.nv, angle_rad=self.angles.data_ptr(),
            pixel_cm=self.pixel_cm, radius_cm=self.radius_cm,
            accept_half_angle_rad=self.accept_half_angle_rad, e_lo_kev=self.e_lo_kev,
            e_hi_kev=self.e_hi_kev, e_cut_kev=self.e_cut_kev, pe_fraction=self.pe_fraction,
            n_histories=self.n_histories, history_offset=self.history_offset,
            history_count=self.history_count, seed=self.seed, problem_id=self.problem_id,
            image_factor=self.image_factor, max_steps=self.max_steps,
            activity_prev=self.activity_prev.data_ptr() if self.activity_prev is not None else None,
            e0_kev=self.e0_kev)


_SCALARS = ["nx", "ny", "nz", "voxel_cm", "nu", "nv", "pixel_cm", "radius_cm",
            "accept_half_angle_rad", "e_lo_kev", "e_hi_kev", "e_cut_kev", "n_histories", "seed",
            "problem_id", "source_mode", "image_factor", "pe_fraction", "max_steps",
            "history_offset", "history_count", "e0_kev"]


def to_device(prob, device="cuda") -> DeviceProblem:
    """Copy a host problem description (numpy arrays + scalars) to the GPU."""
    torch = _torch()
    mu = torch.from_numpy(np.ascontiguousarray(prob.mu, dtype=np.float32)).to(device)
    act = torch.from_numpy(np.ascontiguousarray(prob.activity, dtype=np.uint32).view(np.int32)).to(device)
    ang = torch.from_numpy(np.ascontiguousarray(prob.angles, dtype=np.float64)).to(device)
    kw = {k: getattr(prob, k) for k in _SCALARS}
    prev = getattr(prob, "activity_prev", None)
    if prev is not None:
        prev = torch.from_numpy(np.ascontiguousarray(prev, dtype=np.uint32).view(np.int32)).to(device)
    return DeviceProblem(mu=mu, activity=act, angles=ang, activity_prev=prev, **kw)


def _opts(options: Optional[dict]) -> Optional[McOptions]:
    if not options:
        return None
    o = McOptions(hist_per_lane=int(options.get("hist_per_lane", 0)),
                  block_size=int(options.get("block_size", 0)),
                  blocks_per_cu=int(options.get("blocks_per_cu", 0)),
                  brick_log2=int(options.get("brick_log2", 0)),
                  threshold_bytes=int(options.get("threshold_bytes", 0)),
                  forced_detection=int(options.get("forced_detection", 0)),
                  variance_reduction=int(options.get("variance_reduction", 0)),
                  forced_direction_half_angle_rad=float(options.get("forced_direction_half_angle", 0.0)))
    ev = options.get("kernel_events")
    if ev is not None:
        o.kernel_events[0] = ev[0]
        o.kernel_events[1] = ev[1]
    return o


class KernelTimer:
    """A hipEvent_t pair the library records around its transport kernel."""

    def __init__(self):
        self._hip = C.CDLL("libamdhip64.so")
        self._hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self._hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self._hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = [C.c_void_p(), C.c_void_p()]
        for e in self.ev:
            if self._hip.hipEventCreate(C.byref(e)) != 0:
                raise McError("hipEventCreate failed")

    @property
    def handles(self):
        return (self.ev[0].value, self.ev[1].value)

    def elapsed_ms(self) -> float:
        ms = C.c_float()
        if self._hip.hipEventElapsedTime(C.byref(ms), self.ev[0], self.ev[1]) != 0:
            raise McError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        try:
            for e in self.ev:
                if e.value:
                    self._hip.hipEventDestroy(e)
        except Exception:
            pass


def _stream_ptr():
    return _torch().cuda.current_stream().cuda_stream


def workspace_bytes(problems: Sequence[DeviceProblem], options=None) -> int:
    arr = (McProblem * len(problems))(*[p.c_struct() for p in problems])
    o = _opts(options)
    n = _lib.mc_workspace_bytes(arr, len(problems), C.byref(o) if o else None)
    if n == 0:
        raise McError("mc_workspace_bytes: invalid problem description")
    return int(n)


class Simulator:
    """Holds the outputs and workspace of repeated mc_simulate_projections calls
    on a fixed set of problems (no allocation per call)."""

    def __init__(self, problems: Union[DeviceProblem, Sequence[DeviceProblem]], *,
                 event_capacity: int = 0, want_sq: bool = True, options: Optional[dict] = None):
        torch = _torch()
        if isinstance(problems, DeviceProblem):
            problems = [problems]
        self.problems: List[DeviceProblem] = list(problems)
        self.options = _opts(options)
        n = len(self.problems)
        self._arr = (McProblem * n)(*[p.c_struct() for p in self.problems])
        dev = self.problems[0].mu.device
        self.sizes = [int(np.prod(p.tally_shape)) for p in self.problems]
        total = sum(self.sizes)
        self.tally = torch.zeros(total, dtype=torch.int64, device=dev)
        self.tally_sq = torch.zeros(total, dtype=torch.int64, device=dev) if want_sq else None
        self.fates = torch.zeros((n, 8), dtype=torch.int64, device=dev)
        self.energy = torch.zeros((n, 4), dtype=torch.int64, device=dev)
        self.counters = torch.zeros((n, 8), dtype=torch.int64, device=dev)
        self.status = torch.zeros(4, dtype=torch.int64, device=dev)
        self.event_capacity = int(event_capacity)
        self.events = (torch.zeros((max(self.event_capacity, 1), 3), dtype=torch.int64, device=dev)
                       if self.event_capacity else None)
        self.n_events = torch.zeros(1, dtype=torch.int64, device=dev)
        nb = _lib.mc_workspace_bytes(self._arr, n, C.byref(self.options) if self.options else None)
        if nb == 0:
            raise McError("mc_workspace_bytes: invalid problem description")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=dev)

    def run(self, kernel_events=None):
        """Enqueue one mc_simulate_projections on the current stream.  kernel_events:
        optional (hipEvent_t, hipEvent_t) handles recorded around the transport kernel."""
        opts = self.options
        if kernel_events is not None:
            opts = McOptions()
            if self.options is not None:
                C.memmove(C.byref(opts), C.byref(self.options), C.sizeof(McOptions))
            opts.kernel_events[0] = kernel_events[0]
            opts.kernel_events[1] = kernel_events[1]
        rc = _lib.mc_simulate_projections(
            self._arr, len(self.problems), C.byref(opts) if opts else None,
            self.tally.data_ptr(), self.tally_sq.data_ptr() if self.tally_sq is not None else None,
            self.fates.data_ptr(), self.energy.data_ptr(), self.counters.data_ptr(),
            self.events.data_ptr() if self.events is not None else None, self.event_capacity,
            self.n_events.data_ptr(), self.status.data_ptr(), self.workspace.data_ptr(),
            self.workspace.numel(), _stream_ptr())
        _check(rc, "mc_simulate_projections")

    def run_static(self):
        """The same call through mc_simulate_projections_static: the library's
        per-device scratch array instead of this Simulator's workspace (for
        callers that cannot allocate; calls overlapping on one device race)."""
        opts = self.options
        rc = _lib.mc_simulate_projections_static(
            self._arr, len(self.problems), C.byref(opts) if opts else None,
            self.tally.data_ptr(), self.tally_sq.data_ptr() if self.tally_sq is not None else None,
            self.fates.data_ptr(), self.energy.data_ptr(), self.counters.data_ptr(),
            self.events.data_ptr() if self.events is not None else None, self.event_capacity,
            self.n_events.data_ptr(), self.status.data_ptr(), _stream_ptr())
        _check(rc, "mc_simulate_projections_static")

    def check_status(self):
        """mc_check_status on the call's status: raises McError for bad
        device input or a tally that left its fixed-point range; returns the
        status array (list overflow and capped histories are reported there)."""
        rc = _lib.mc_check_status(self.status.data_ptr(), _stream_ptr())
        st = self.status.cpu().numpy()
        if rc in (MC_EINVAL, MC_EOVERFLOW, MC_EDEVICE):
            raise McError(f"{_lib.mc_error_string(rc).decode()} (status bits {int(st[0])})")
        return st

    def tallies(self):
        """Per-problem tally tensors (int64 Q31.32) shaped [V, 2, nv, nu]."""
        out, off = [], 0
        for p, s in zip(self.problems, self.sizes):
            out.append(self.tally[off:off + s].view(p.tally_shape))
            off += s
        return out

    def events_numpy(self) -> np.ndarray:
        n = min(int(self.n_events.item()), self.event_capacity)
        if self.events is None or n == 0:
            return np.zeros(0, dtype=EVENT_DTYPE)
        raw = self.events[:n].cpu().numpy()
        return raw.view(EVENT_DTYPE).reshape(-1)


def simulate(problems, *, event_capacity: int = 0, want_sq: bool = True, options=None,
             sync: bool = True) -> Simulator:
    """One forward run (allocates outputs and workspace)."""
    sim = Simulator(problems, event_capacity=event_capacity, want_sq=want_sq, options=options)
    sim.run()
    if sync:
        _torch().cuda.synchronize()
        sim.check_status()
    return sim


def replay(problem: DeviceProblem, views, hists, options=None) -> np.ndarray:
    """Per-history records for listed (view, history id) pairs of one problem."""
    torch = _torch()
    dev = problem.mu.device
    v = torch.as_tensor(np.ascontiguousarray(views, dtype=np.int32), device=dev)
    h = torch.as_tensor(np.ascontiguousarray(hists, dtype=np.uint64).view(np.int64), device=dev)
    n = int(v.numel())
    rec = torch.zeros((max(n, 1), 5), dtype=torch.int64, device=dev)   # 40-byte records
    status = torch.zeros(4, dtype=torch.int64, device=dev)
    arr = problem.c_struct()
    o = _opts(options)
    nb = _lib.mc_workspace_bytes(C.byref(arr), 1, C.byref(o) if o else None)
    if nb == 0:
        raise McError("mc_workspace_bytes: invalid problem description")
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    rc = _lib.mc_replay_histories(C.byref(arr), C.byref(o) if o else None, v.data_ptr(), h.data_ptr(),
                                  n, rec.data_ptr(), status.data_ptr(), ws.data_ptr(), nb,
                                  _stream_ptr())
    _check(rc, "mc_replay_histories")
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    if st[0] & (STATUS_BAD_MU | STATUS_NO_ACTIVITY | STATUS_BAD_ANGLE):
        raise McError(f"invalid device input (status bits {int(st[0])})")
    return rec[:n].cpu().numpy().view(RECORD_DTYPE).reshape(-1)


def tally_float(t) -> np.ndarray:
    """Fixed-point tally -> float64 counts."""
    return t.cpu().numpy().astype(np.float64) / Q32


class RptProjector:
    """Reuse of photon tracks (Sec. 5.3) for the reprojections of an iterative
    reconstruction: the first call simulates the whole estimate; each later
    call simulates only the difference to the previous estimate (a signed
    source, activity_prev) and adds its projection to the previous one.

    problem: the geometry and camera (its activity is replaced per call).
    histories_per_unit: histories per unit of source activity (|d| for a
    difference), rounded to a whole number per view, at least one per view.
    Projections are float64 tensors [V, 2, nv, nu] in activity units: the
    expected projection of a source of total activity A from N histories over
    V views is tally x A V / N."""

    def __init__(self, problem: DeviceProblem, histories_per_unit: float, options=None):
        self.problem = problem
        self.hpu = float(histories_per_unit)
        self.options = options
        self.prev = None
        self.projection = None
        self.histories = []        # histories simulated per call
        self.seed = int(problem.seed)

    def _run(self, activity, prev, out, accumulate):
        V = self.problem.n_views
        total = source_total(activity, prev)
        per_view = max(1, int(round(self.hpu * total / V)))
        n = per_view * V
        self.seed += 1
        dp = self.problem.with_(activity=activity, activity_prev=prev, n_histories=n,
                                history_offset=0, history_count=0, seed=self.seed)
        self.histories.append(n)
        if total == 0:
            if not accumulate:
                out.zero_()
            return
        sim = simulate(dp, want_sq=False, options=self.options)
        scale_tally(sim.tally, total * V / n, out, accumulate)

    def project(self, activity):
        """Projection of the estimate `activity` (device uint32 map stored as
        int32, as to_device makes it)."""
        torch = _torch()
        activity = activity.contiguous()
        if self.prev is None:
            self.projection = torch.empty(self.problem.tally_shape, dtype=torch.float64,
                                          device=activity.device)
            self._run(activity, None, self.projection, False)
        else:
            self._run(activity, self.prev, self.projection, True)
        self.prev = activity.clone()
        return self.projection


def source_total(activity, activity_prev=None) -> int:
    """Total weight of a source, sum |activity - activity_prev| (of activity
    without a previous map), computed on the device (mc_source_total) and
    read back (the history count of a projection is set from it)."""
    torch = _torch()
    total = torch.zeros(1, dtype=torch.int64, device=activity.device)
    _check(_lib.mc_source_total(activity.data_ptr(),
                                activity_prev.data_ptr() if activity_prev is not None else None,
                                activity.numel(), total.data_ptr(), _stream_ptr()), "mc_source_total")
    return int(total.item()) & 0xFFFFFFFFFFFFFFFF


def scale_tally(tally, scale: float, out, accumulate: bool = False):
    """out = tally x 2^-32 x scale, or out + that (mc_scale_tally); out: device
    float64 tensor with as many elements as the tally."""
    if out.numel() != tally.numel() or out.dtype != _torch().float64 or not out.is_contiguous():
        raise McError("scale_tally: out must be a contiguous float64 tensor of the tally's size")
    _check(_lib.mc_scale_tally(tally.data_ptr(), tally.numel(), float(scale), out.data_ptr(),
                               1 if accumulate else 0, _stream_ptr()), "mc_scale_tally")
    return out


def coarse_problem(problem: DeviceProblem, factor: int) -> DeviceProblem:
    """Coarse-grid scatter modelling (Sec. 5.4): the same problem with the
    block-summed source (mc_block_activity) and a detector of factor times
    larger pixels (nu, nv multiples of factor).  Raises if a block sum
    overflows 32 bits."""
    torch = _torch()
    f = int(factor)
    if problem.activity_prev is not None:
        raise McError("coarse_problem takes a plain source")
    if problem.nu % f or problem.nv % f:
        raise McError("detector size not a multiple of the coarsening factor")
    out = torch.empty_like(problem.activity)
    status = torch.zeros(1, dtype=torch.int64, device=out.device)
    _check(_lib.mc_block_activity(problem.activity.data_ptr(), problem.nx, problem.ny, problem.nz, f,
                                  out.data_ptr(), status.data_ptr(), _stream_ptr()), "mc_block_activity")
    if int(status.item()) & STATUS_ACTIVITY_OVERFLOW:
        raise McError("block activity exceeds 32 bits")
    return problem.with_(activity=out, nu=problem.nu // f, nv=problem.nv // f,
                         pixel_cm=problem.pixel_cm * f)


def expand_projection(tally, shape, factor: int, scale: float = 1.0):
    """A coarse Q31.32 tally [V, 2, nv_c, nu_c] expanded to the normal pixels,
    float64 [V, 2, nv_c f, nu_c f]: counts per normal pixel times scale
    (mc_expand_projection)."""
    torch = _torch()
    V, K, nv_c, nu_c = shape
    f = int(factor)
    src = tally.contiguous()
    out = torch.empty((V, K, nv_c * f, nu_c * f), dtype=torch.float64, device=tally.device)
    _check(_lib.mc_expand_projection(src.data_ptr(), V * K, nu_c, nv_c, f, float(scale),
                                     out.data_ptr(), _stream_ptr()), "mc_expand_projection")
    return out


class ScatterModel:
    """Monte Carlo scatter projection for OS-EM with an additive scatter term
    (Sec. 5.4), with the two accelerations the paper reviews: coarse-grid
    scatter modelling (the scatter is simulated on coarse_problem(problem,
    factor) and expanded) and intermittent scatter modelling (only the first
    n_updates calls simulate; later calls return the last estimate).

    estimate(activity): the class-1 (scattered) projection [V, nv, nu],
    float64, in activity units (tally x A V / N for a source of total
    activity A from N histories over V views).  activity: device uint32 map
    (stored as int32, as to_device makes it) on the problem's grid."""

    def __init__(self, problem: DeviceProblem, histories: int, factor: int = 2, n_updates: int = 2,
                 forced_detection: int = 1):
        self.problem = problem
        V = problem.n_views
        self.histories = max(1, int(histories) // V) * V
        self.factor = int(factor)
        self.n_updates = int(n_updates)
        self.options = {"forced_detection": int(forced_detection)} if forced_detection else None
        self.calls = 0
        self.simulations = 0
        self.last = None

    def estimate(self, activity):
        self.calls += 1
        if self.last is not None and self.simulations >= self.n_updates:
            return self.last
        dp = self.problem.with_(activity=activity.contiguous(), n_histories=self.histories,
                                history_offset=0, history_count=0,
                                seed=int(self.problem.seed) + self.simulations)
        cp = coarse_problem(dp, self.factor)
        sim = simulate(cp, want_sq=False, options=self.options)
        total = source_total(dp.activity)
        self.last = expand_projection(sim.tally, cp.tally_shape, self.factor,
                                      total * self.problem.n_views / self.histories)[:, 1]
        self.simulations += 1
        return self.last


def fd_tally_sq_float(t) -> np.ndarray:
    """Forced-detection sum of squared scores (Q11.52) -> float64."""
    return t.cpu().numpy().astype(np.float64) / Q52


ADJOINT_FRAC_BITS = (40, 28, 16)


def adjoint(problem: DeviceProblem, dL_dtally, sim: Optional[Simulator] = None,
            frac_bits: Optional[int] = None, raw: bool = False, events: Optional[np.ndarray] = None):
    """dL/dmu (float64 tensor [nz, ny, nx]) for G = dL_dtally (tally layout).

    sim: the forward Simulator of the same problem; its event list (if it has
    one) restricts the replay to the tallied histories.  Without it every
    history of the range is replayed.  events: an explicit list of tallied
    histories (EVENT_DTYPE records, e.g. a subset of sim.events_numpy()) to
    replay instead of sim's list.  frac_bits: fractional bits of the
    fixed-point sums; None tries 40, 28 and 16 in turn, rerunning the call
    with fewer bits when a term overflowed (MC_STATUS_GRAD_OVERFLOW); an
    explicit value raises on overflow instead.  raw: the int64 sums (needs
    an explicit frac_bits)."""
    if frac_bits is None:
        if raw:
            raise McError("raw sums need an explicit frac_bits")
        for fb in ADJOINT_FRAC_BITS:
            try:
                return adjoint(problem, dL_dtally, sim, fb, False, events)
            except GradientOverflow:
                if fb == ADJOINT_FRAC_BITS[-1]:
                    raise
        raise AssertionError("unreachable")
    torch = _torch()
    dev = problem.mu.device
    if events is not None:
        ev = np.ascontiguousarray(events, dtype=EVENT_DTYPE)
        ev_t = torch.from_numpy(ev.view(np.int64).reshape(-1, 3).copy()).to(dev) if len(ev) else \
            torch.zeros((1, 3), dtype=torch.int64, device=dev)
        ev_n = torch.tensor([len(ev)], dtype=torch.int64, device=dev)
    G = dL_dtally.to(device=dev, dtype=torch.float64).contiguous()
    if G.numel() != int(np.prod(problem.tally_shape)):
        raise McError("dL_dtally has the wrong size")
    grad = torch.empty(problem.mu.shape, dtype=torch.int64, device=dev)
    status = torch.zeros(4, dtype=torch.int64, device=dev)
    arr = problem.c_struct()
    nb = _lib.mc_workspace_bytes(C.byref(arr), 1, None)
    if nb == 0:
        raise McError("mc_workspace_bytes: invalid problem description")
    if sim is not None and sim.options is not None and (sim.options.forced_detection or
                                                         sim.options.variance_reduction):
        raise McError("the adjoint takes the event list of an analog forward run")
    # the forward Simulator of this one problem already staged its tables
    opt = None
    if sim is not None and len(sim.problems) == 1 and sim.problems[0] is problem:
        ws, nb = sim.workspace, sim.workspace.numel()
        opt = McOptions(reuse_staging=1)
        if sim.options is not None:
            opt.brick_log2, opt.threshold_bytes = sim.options.brick_log2, sim.options.threshold_bytes
    else:
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    if events is not None:
        use_events, ev_ptr, n_ptr, cap = True, ev_t.data_ptr(), ev_n.data_ptr(), max(len(ev), 1)
    else:
        use_events = sim is not None and sim.events is not None
        ev_ptr = sim.events.data_ptr() if use_events else None
        n_ptr = sim.n_events.data_ptr() if use_events else None
        cap = sim.event_capacity if use_events else 0
    rc = _lib.mc_adjoint_mu(C.byref(arr), C.byref(opt) if opt is not None else None, G.data_ptr(),
                            ev_ptr, n_ptr, cap, grad.data_ptr(), int(frac_bits), status.data_ptr(),
                            ws.data_ptr(), nb, _stream_ptr())
    _check(rc, "mc_adjoint_mu")
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    if st[0] & (STATUS_BAD_MU | STATUS_NO_ACTIVITY | STATUS_BAD_ANGLE):
        raise McError(f"invalid device input (status bits {int(st[0])})")
    if st[0] & STATUS_GRAD_OVERFLOW:
        raise GradientOverflow(f"gradient overflow at frac_bits={frac_bits}; use fewer fractional bits")
    if st[0] & STATUS_BAD_EVENT:
        raise McError("an event did not replay to its bin (event list from another problem?)")
    if events is None and use_events and int(sim.n_events.item()) > sim.event_capacity:
        raise McError("the forward event list overflowed; raise event_capacity")
    if raw:
        return grad
    return grad.to(torch.float64) * (2.0 ** -frac_bits)


class MCProject:
    """torch.autograd.Function: mu -> projection tallies (float64 counts, tally
    layout), with the replaying adjoint as backward.  Activity and geometry
    are constants."""

    @staticmethod
    def apply(mu, problem: DeviceProblem, event_capacity: int = 1 << 20, frac_bits: Optional[int] = None):
        return _mc_project_fn().apply(mu, problem, event_capacity, frac_bits)


_FN = None


def _mc_project_fn():
    global _FN
    if _FN is not None:
        return _FN
    torch = _torch()

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mu, problem, event_capacity, frac_bits):
            dp = problem.with_(mu=mu.detach().to(torch.float32).contiguous())
            sim = simulate(dp, event_capacity=event_capacity, want_sq=False)
            if int(sim.n_events.item()) > event_capacity:
                raise McError("event list overflow in forward; raise event_capacity")
            ctx.dp, ctx.sim, ctx.frac_bits = dp, sim, frac_bits
            return sim.tally.view(dp.tally_shape).to(torch.float64) * (2.0 ** -32)

        @staticmethod
        def backward(ctx, grad_out):
            g = adjoint(ctx.dp, grad_out, ctx.sim, ctx.frac_bits)
            return g.to(torch.float32), None, None, None

    _FN = _Fn
    return _FN


# ---------------------------------------------------------------------------
# Graph capture and autotuning of the batched launch
# ---------------------------------------------------------------------------

class Graph:
    """A fixed sequence of library calls captured as one HIP graph by the
    library (mc_graph_begin / mc_graph_end) and replayed with
    mc_graph_launch.  fn() is run `warmup` times eagerly, then once under
    capture on a stream of its own; the graph keeps the buffers, sizes and
    options those calls were given.  fn must not allocate (workspaces are
    made beforehand) and must not synchronise."""

    def __init__(self, fn, warmup: int = 1):
        torch = _torch()
        self.stream = torch.cuda.Stream()       # capture needs a stream of its own
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                fn()
        torch.cuda.synchronize()
        s = self.stream.cuda_stream
        _check(_lib.mc_graph_begin(s), "mc_graph_begin")
        g = C.c_void_p()
        with torch.cuda.stream(self.stream):
            try:
                fn()
            finally:
                rc = _lib.mc_graph_end(s, C.byref(g))
        _check(rc, "mc_graph_end")
        self.graph = g

    def replay(self):
        _check(_lib.mc_graph_launch(self.graph, _stream_ptr()), "mc_graph_launch")

    def __del__(self):
        try:
            if getattr(self, "graph", None):
                _lib.mc_graph_destroy(self.graph)
                self.graph = None
        except Exception:
            pass


class GraphRunner(Graph):
    """One mc_simulate_projections call on a Simulator as a graph (staging,
    transport and finalize as graph nodes); replay() relaunches it on the
    current stream."""

    def __init__(self, sim: Simulator, warmup: int = 1):
        self.sim = sim
        super().__init__(sim.run, warmup)


def _size_class(problems: Sequence[DeviceProblem]) -> str:
    vox = sum(p.nx * p.ny * p.nz for p in problems)
    hist = sum((p.history_count or p.n_histories - p.history_offset) for p in problems)
    views = sum(p.n_views for p in problems)
    b = lambda x: int(np.floor(np.log2(max(x, 1))))
    return f"n{len(problems)}_vox2^{b(vox)}_hist2^{b(hist)}_views2^{b(views)}"


_TUNE_CACHE = {}


def autotune(problems: Union[DeviceProblem, Sequence[DeviceProblem]], *,
             bricks=(0, 2, 3), hist_per_lane=(4, 16, 64), block_sizes=(256,), reps: int = 2,
             cache_path: Optional[str] = None, verbose: bool = False) -> dict:
    """Pick launch options (threshold brick size, histories per lane claim,
    block size) by timing the transport kernel on these problems.  Every
    candidate gives bit-identical results (layout and scheduling only); the
    choice is cached per (GPU arch, size class)."""
    import json
    torch = _torch()
    if isinstance(problems, DeviceProblem):
        problems = [problems]
    arch = torch.cuda.get_device_properties(problems[0].mu.device).gcnArchName
    key = f"{arch}|{_size_class(problems)}"
    if cache_path and os.path.exists(cache_path) and not _TUNE_CACHE:
        try:
            _TUNE_CACHE.update(json.load(open(cache_path)))
        except (OSError, ValueError):
            pass
    if key in _TUNE_CACHE:
        return dict(_TUNE_CACHE[key])
    cands = [{"brick_log2": br, "hist_per_lane": h, "block_size": bs}
             for br in bricks for h in hist_per_lane for bs in block_sizes]
    arr = (McOptions * len(cands))(*[_opts(o) for o in cands])
    sim = Simulator(problems, want_sq=False)
    best_i = C.c_int32(-1)
    times = (C.c_float * len(cands))()
    _check(_lib.mc_autotune(sim._arr, len(problems), arr, len(cands), int(reps), sim.tally.data_ptr(),
                            sim.fates.data_ptr(), sim.status.data_ptr(), sim.workspace.data_ptr(),
                            sim.workspace.numel(), _stream_ptr(), C.byref(best_i), times), "mc_autotune")
    log = [(o, float(t)) for o, t in zip(cands, times)]
    best = cands[best_i.value]
    if verbose:
        for o, t in log:
            print(f"autotune {o}: {t:.3f} ms")
    _TUNE_CACHE[key] = dict(best)
    if cache_path:
        try:
            with open(cache_path, "w") as f:
                json.dump(_TUNE_CACHE, f, indent=1)
        except OSError:
            pass
    return dict(best)


# ---------------------------------------------------------------------------
# Response matrix and MLEM (Sec. 5.1)
# ---------------------------------------------------------------------------

@dataclass
class SystemMatrix:
    """Monte Carlo response matrix in CSR, both orientations (device tensors).
    Rows of T are projection bins (view, iv, iu); rows of Tt are image voxels."""
    n_bins: int
    n_img: int
    T_rowptr: "object"
    T_col: "object"
    T_val: "object"
    Tt_rowptr: "object"
    Tt_col: "object"
    Tt_val: "object"
    proj: "object"

    @property
    def nnz(self) -> int:
        return int(self.T_rowptr[-1].item())

    def to_scipy(self, transpose: bool = False):
        import scipy.sparse as sp
        n = self.nnz
        if transpose:
            return sp.csr_matrix((self.Tt_val[:n].cpu().numpy(), self.Tt_col[:n].cpu().numpy(),
                                  self.Tt_rowptr.cpu().numpy()), shape=(self.n_img, self.n_bins))
        return sp.csr_matrix((self.T_val[:n].cpu().numpy(), self.T_col[:n].cpu().numpy(),
                              self.T_rowptr.cpu().numpy()), shape=(self.n_bins, self.n_img))


def system_matrix(problem: DeviceProblem, sim: Simulator, classes: str = "all") -> SystemMatrix:
    """Response matrix from the event list of a forward Simulator run.
    classes: "all", "primary" (backprojector of the dual-matrix and
    additive-scatter forms) or "scatter" (its proj is the scatter projection)."""
    mask = {"all": 3, "primary": 1, "scatter": 2}[classes]
    torch = _torch()
    if sim.events is None:
        raise McError("the forward run kept no event list")
    n_ev = int(sim.n_events.reshape(-1)[0].item())
    if n_ev > sim.event_capacity:
        raise McError(f"the event list lost events ({n_ev} tallied, capacity {sim.event_capacity}): "
                      "rerun the forward call with a larger event_capacity")
    if problem.image_factor < 1:
        raise McError("problem.image_factor must be >= 1")
    dev = problem.mu.device
    f = problem.image_factor
    n_bins = problem.n_views * problem.nv * problem.nu
    n_img = (problem.nx // f) * (problem.ny // f) * (problem.nz // f)
    cap = sim.event_capacity
    arr = problem.c_struct()
    nb = _lib.mc_system_matrix_workspace_bytes(C.byref(arr), cap)
    if nb == 0:
        raise McError("mc_system_matrix_workspace_bytes: invalid arguments")
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    m = SystemMatrix(n_bins, n_img,
                     torch.empty(n_bins + 1, dtype=torch.int64, device=dev),
                     torch.empty(cap, dtype=torch.int32, device=dev),
                     torch.empty(cap, dtype=torch.float32, device=dev),
                     torch.empty(n_img + 1, dtype=torch.int64, device=dev),
                     torch.empty(cap, dtype=torch.int32, device=dev),
                     torch.empty(cap, dtype=torch.float32, device=dev),
                     torch.empty(n_bins, dtype=torch.float32, device=dev))
    rc = _lib.mc_system_matrix(C.byref(arr), sim.events.data_ptr(), sim.n_events.data_ptr(), cap,
                               mask, m.T_rowptr.data_ptr(), m.T_col.data_ptr(), m.T_val.data_ptr(),
                               m.Tt_rowptr.data_ptr(), m.Tt_col.data_ptr(), m.Tt_val.data_ptr(),
                               m.proj.data_ptr(), ws.data_ptr(), nb, _stream_ptr())
    _check(rc, "mc_system_matrix")
    return m


class Mlem:
    """MLEM on fixed CSR buffers: the workspace is allocated and the matrix's
    set-up (mlem_prepare) done once; each run is mlem_iterate_prepared.  The
    matrix must not change while this object is used (build a new one)."""

    def __init__(self, m: SystemMatrix):
        torch = _torch()
        self.m = m
        nb = _lib.mlem_workspace_bytes(m.n_bins, m.n_img)
        if nb == 0:
            raise McError("mlem_workspace_bytes: invalid sizes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=m.T_val.device)
        self.nnz = m.nnz                          # read once: it picks the schedule
        rc = _lib.mlem_prepare(m.n_bins, m.n_img, self.nnz, *self._csr(), self.ws.data_ptr(), self.ws.numel(),
                               _stream_ptr())
        _check(rc, "mlem_prepare")

    def _csr(self):
        m = self.m
        return (m.T_rowptr.data_ptr(), m.T_col.data_ptr(), m.T_val.data_ptr(), m.Tt_rowptr.data_ptr(),
                m.Tt_col.data_ptr(), m.Tt_val.data_ptr())

    def run(self, image, n_iter: int, proj=None):
        """image: float32 device tensor [n_img], S^0 in, S^n_iter out (in place)."""
        m = self.m
        P = m.proj if proj is None else proj
        rc = _lib.mlem_iterate_prepared(m.n_bins, m.n_img, self.nnz, *self._csr(), P.data_ptr(),
                                        image.data_ptr(), int(n_iter), self.ws.data_ptr(), self.ws.numel(),
                                        _stream_ptr())
        _check(rc, "mlem_iterate_prepared")
        return image

    def run_unprepared(self, image, n_iter: int, proj=None):
        """The same update through mlem_iterate (set-up repeated in the call)."""
        m = self.m
        P = m.proj if proj is None else proj
        rc = _lib.mlem_iterate(m.n_bins, m.n_img, self.nnz, *self._csr(), P.data_ptr(), image.data_ptr(),
                               int(n_iter), self.ws.data_ptr(), self.ws.numel(), _stream_ptr())
        _check(rc, "mlem_iterate")
        return image


def csr_from_scipy(T, device="cuda") -> SystemMatrix:
    """Device CSR pair from a host scipy matrix (rows = bins) and proj = 0."""
    torch = _torch()
    T = T.tocsr()
    T.sort_indices()
    Tt = T.T.tocsr()
    Tt.sort_indices()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a).astype(dt), device=device)
    return SystemMatrix(T.shape[0], T.shape[1], t(T.indptr, np.int64), t(T.indices, np.int32),
                        t(T.data, np.float32), t(Tt.indptr, np.int64), t(Tt.indices, np.int32),
                        t(Tt.data, np.float32), torch.zeros(T.shape[0], dtype=torch.float32, device=device))


def osem(c: SystemMatrix, image, n_iter: int, n_subsets: int, bins_per_view: int,
         b: Optional[SystemMatrix] = None, proj=None, scatter=None):
    """Ordered-subsets reconstruction (OSEM; dual matrix with backprojector b;
    additive scatter projection).  image: float32 device [n_img], in place."""
    torch = _torch()
    b = c if b is None else b
    P = c.proj if proj is None else proj
    nb = _lib.osem_workspace_bytes(c.n_bins, c.n_img, int(n_subsets), int(b.nnz))
    if nb == 0:
        raise McError("osem_workspace_bytes: invalid sizes (or more than 64 subsets)")
    ws = torch.empty(nb, dtype=torch.uint8, device=c.T_val.device)
    rc = _lib.osem_iterate(c.n_bins, c.n_img, int(bins_per_view), int(n_subsets),
                           c.T_rowptr.data_ptr(), c.T_col.data_ptr(), c.T_val.data_ptr(),
                           b.Tt_rowptr.data_ptr(), b.Tt_col.data_ptr(), b.Tt_val.data_ptr(), int(b.nnz),
                           P.data_ptr(), scatter.data_ptr() if scatter is not None else None,
                           image.data_ptr(), int(n_iter), ws.data_ptr(), nb, _stream_ptr())
    _check(rc, "osem_iterate")
    return image
