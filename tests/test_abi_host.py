"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every declared entry point, its structures match the header, and argument
validation rejects bad inputs before touching the device."""
import ctypes as C
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcspect.h")


def _mc():
    import paper_2105_13324_amd as mc
    return mc


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b((?:mc|mlem|osem)_\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    mc = _mc()
    lib = C.CDLL(mc.LIB_PATH)
    decl = declared_functions()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(mc.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", mc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in decl:
        assert re.search(r"\bT %s\b" % name, out), name


def test_region_profile_only_in_the_measurement_build():
    """mc_region_profile (the transport loop's region markers) exists only in
    libmcspect_prof.so; the product library carries no marker code."""
    mc = _mc()
    prof = os.path.join(os.path.dirname(mc.LIB_PATH), "libmcspect_prof.so")
    out = subprocess.run(["nm", "-D", "--defined-only", mc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "mc_region_profile" not in out
    if not os.path.exists(prof):
        pytest.skip("measurement build not built (python paper_2105_13324_amd/build.py --profile)")
    out = subprocess.run(["nm", "-D", "--defined-only", prof], capture_output=True,
                         text=True, check=True).stdout
    assert re.search(r"\bT mc_region_profile\b", out)
    for name in declared_functions():
        assert re.search(r"\bT %s\b" % name, out), name


def _layout_src(mc):
    fields = " ".join("F(mc_problem, %s)" % n for n, _ in mc.McProblem._fields_)
    return r"""
#include <stddef.h>
#include <stdio.h>
#include "mcspect.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("mc_problem size %zu\n", sizeof(mc_problem));
  """ + fields + r"""
  printf("mc_options size %zu\n", sizeof(mc_options));
  printf("mc_event size %zu\n", sizeof(mc_event));
  printf("mc_record size %zu\n", sizeof(mc_record));
  F(mc_record, e_final)
  return 0;
}
"""


def test_struct_layout_matches_header():
    mc = _mc()
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(_layout_src(mc))
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        t, f, v = line.split()
        got[(t, f)] = int(v)
    assert got[("mc_problem", "size")] == C.sizeof(mc.McProblem)
    for name, _ in mc.McProblem._fields_:
        assert got[("mc_problem", name)] == getattr(mc.McProblem, name).offset, name
    assert got[("mc_options", "size")] == C.sizeof(mc.McOptions)
    assert got[("mc_event", "size")] == mc.EVENT_DTYPE.itemsize
    assert got[("mc_record", "size")] == mc.RECORD_DTYPE.itemsize
    assert got[("mc_record", "e_final")] == mc.RECORD_DTYPE.fields["e_final"][1]


def _good():
    mc = _mc()
    p = mc.McProblem(nx=8, ny=8, nz=8, source_mode=0, voxel_cm=0.5, mu140=16, activity=16,
                     n_views=4, nu=8, nv=8, angle_rad=16, pixel_cm=0.5, radius_cm=10.0,
                     accept_half_angle_rad=0.05, e_lo_kev=126, e_hi_kev=154, e_cut_kev=10,
                     pe_fraction=1e-3, n_histories=1000, history_offset=0, history_count=0,
                     seed=0, problem_id=0, image_factor=0, max_steps=0)
    return p


def test_workspace_bytes_and_validation():
    mc = _mc()
    lib = mc._lib
    p = _good()
    n = lib.mc_workspace_bytes(C.byref(p), 1, None)
    assert n > 8 ** 3 * 12
    # grows with the grid
    p2 = _good(); p2.nx = 16
    assert lib.mc_workspace_bytes(C.byref(p2), 1, None) > n
    bad = [
        dict(nx=0), dict(voxel_cm=0.0), dict(voxel_cm=float("nan")), dict(mu140=None),
        dict(activity=None), dict(angle_rad=None), dict(n_views=0), dict(nu=0), dict(pixel_cm=-1.0),
        dict(radius_cm=2.0), dict(accept_half_angle_rad=0.0), dict(accept_half_angle_rad=2.0),
        dict(e_lo_kev=160.0), dict(e_cut_kev=0.0), dict(pe_fraction=1.5), dict(n_histories=0),
        dict(history_offset=2000), dict(history_offset=500, history_count=600),
        dict(image_factor=3), dict(source_mode=7), dict(nx=1025), dict(e_cut_kev=0.5),
        dict(e0_kev=600.0), dict(e0_kev=71.1), dict(e0_kev=5.0), dict(e0_kev=80.0, e_cut_kev=90.0),
    ]
    for b in bad:
        q = _good()
        for k, v in b.items():
            setattr(q, k, v)
        assert lib.mc_workspace_bytes(C.byref(q), 1, None) == 0, b
        rc = lib.mc_simulate_projections(C.byref(q), 1, None, 8, None, 8, None, None, None, 0,
                                         None, 8, 8, 1 << 30, None)
        assert rc == mc.MC_EINVAL, b


def test_simulate_rejects_bad_buffers_before_launch():
    mc = _mc()
    lib = mc._lib
    p = _good()
    need = lib.mc_workspace_bytes(C.byref(p), 1, None)
    sim = lib.mc_simulate_projections
    # missing outputs
    assert sim(C.byref(p), 1, None, None, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    assert sim(C.byref(p), 1, None, 8, None, None, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    assert sim(C.byref(p), 1, None, 8, None, 8, None, None, None, 0, None, None, 8, need, None) == mc.MC_EINVAL
    # events without a counter
    assert sim(C.byref(p), 1, None, 8, None, 8, None, None, 8, 10, None, 8, 8, need, None) == mc.MC_EINVAL
    # workspace too small
    assert sim(C.byref(p), 1, None, 8, None, 8, None, None, None, 0, None, 8, 8, need - 1, None) == mc.MC_ENOMEM
    # bad options
    o = mc.McOptions(hist_per_lane=0, block_size=96, blocks_per_cu=0, brick_log2=0)
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=1)
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, threshold_bytes=2)
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, forced_detection=3)
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    # convolution-based forced detection: the depth layers need more workspace,
    # an event list is refused, and so is a response wider than 24 pixels
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, forced_detection=2)
    need_cfd = lib.mc_workspace_bytes(C.byref(p), 1, C.byref(o))
    L = math.ceil(2 * p.radius_cm / p.pixel_cm)
    assert need_cfd >= need + 8 * L * 2 * p.n_views * p.nv * p.nu
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_ENOMEM
    assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, 8, 10, 8, 8, 8, need_cfd,
               None) == mc.MC_EINVAL
    wide = _good()
    wide.accept_half_angle_rad = 1.4
    assert lib.mc_workspace_bytes(C.byref(wide), 1, None) > 0
    assert lib.mc_workspace_bytes(C.byref(wide), 1, C.byref(o)) == 0
    assert sim(C.byref(wide), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need_cfd,
               None) == mc.MC_EINVAL
    # the adjoint is of analog tallies only
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, forced_detection=1)
    assert mc._lib.mc_adjoint_mu(C.byref(p), C.byref(o), 8, None, None, 0, 8, 40, 8, 8, need,
                                 None) == mc.MC_EINVAL
    # difference sources (reuse of photon tracks) are forward-only
    q = _good()
    q.activity_prev = 16
    assert lib.mc_workspace_bytes(C.byref(q), 1, None) == need
    assert mc._lib.mc_adjoint_mu(C.byref(q), None, 8, None, None, 0, 8, 40, 8, 8, need,
                                 None) == mc.MC_EINVAL
    q.image_factor = 2
    assert mc._lib.mc_system_matrix(C.byref(q), 8, 8, 16, 3, 8, 8, 8, 8, 8, 8, None, 8,
                                    1 << 30, None) == mc.MC_EINVAL
    # the response matrix normalises by the whole acquisition: a forward call
    # over part of the work range is refused
    for off, cnt in ((5, 0), (0, 600), (500, 500)):
        r = _good()
        r.image_factor, r.history_offset, r.history_count = 2, off, cnt
        assert mc._lib.mc_system_matrix(C.byref(r), 8, 8, 16, 3, 8, 8, 8, 8, 8, 8, None, 8,
                                        1 << 30, None) == mc.MC_EINVAL, (off, cnt)
    # weighted analog transport: flags 0..3, a forced-direction cone, not
    # with forced detection, not for the adjoint
    for kw in (dict(variance_reduction=4), dict(variance_reduction=-1),
               dict(variance_reduction=1, forced_direction_half_angle_rad=0.0),
               dict(variance_reduction=1, forced_direction_half_angle_rad=4.0),
               dict(variance_reduction=2, forced_detection=1)):
        o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, **kw)
        assert sim(C.byref(p), 1, C.byref(o), 8, None, 8, None, None, None, 0, None, 8, 8, need,
                   None) == mc.MC_EINVAL, kw
        assert mc._lib.mc_replay_histories(C.byref(p), C.byref(o), 8, 8, 5, 8, 8, 8, need,
                                           None) == mc.MC_EINVAL, kw
    o = mc.McOptions(hist_per_lane=0, block_size=0, blocks_per_cu=0, brick_log2=0, variance_reduction=2)
    assert mc._lib.mc_adjoint_mu(C.byref(p), C.byref(o), 8, None, None, 0, 8, 40, 8, 8, need,
                                 None) == mc.MC_EINVAL
    # coarse-grid scatter helpers: sizes are checked before any launch
    ba, ex = mc._lib.mc_block_activity, mc._lib.mc_expand_projection
    assert ba(8, 8, 8, 8, 3, 16, 8, None) == mc.MC_EINVAL       # 8 not a multiple of 3
    assert ba(8, 8, 8, 8, 2, 8, 8, None) == mc.MC_EINVAL        # in place
    assert ba(8, 8, 8, 8, 0, 16, 8, None) == mc.MC_EINVAL
    assert ba(None, 8, 8, 8, 2, 16, 8, None) == mc.MC_EINVAL
    assert ex(8, 0, 4, 4, 2, 1.0, 16, None) == mc.MC_EINVAL
    assert ex(8, 2, 4, 4, 0, 1.0, 16, None) == mc.MC_EINVAL
    assert ex(None, 2, 4, 4, 2, 1.0, 16, None) == mc.MC_EINVAL
    assert ex(8, 2, 4, 4, 2, float("nan"), 16, None) == mc.MC_EINVAL
    # projection arithmetic and graph helpers: arguments checked before any launch
    assert mc._lib.mc_source_total(None, None, 10, 8, None) == mc.MC_EINVAL
    assert mc._lib.mc_source_total(8, None, 0, 8, None) == mc.MC_EINVAL
    assert mc._lib.mc_scale_tally(8, 10, float("inf"), 8, 0, None) == mc.MC_EINVAL
    assert mc._lib.mc_scale_tally(8, 10, 1.0, 8, 2, None) == mc.MC_EINVAL
    assert mc._lib.mc_scale_tally(8, 0, 1.0, 8, 0, None) == mc.MC_EINVAL
    assert mc._lib.mc_graph_begin(None) == mc.MC_EINVAL       # the legacy default stream
    assert mc._lib.mc_graph_end(None, None) == mc.MC_EINVAL
    assert mc._lib.mc_graph_launch(None, None) == mc.MC_EINVAL
    assert mc._lib.mc_graph_destroy(None) == mc.MC_OK
    assert mc._lib.mc_check_status(None, None) == mc.MC_EINVAL
    # MLEM: sizes, entry count and workspace checked before any launch
    ml = mc._lib.mlem_iterate
    wsb = mc._lib.mlem_workspace_bytes(100, 50)
    assert wsb > 0 and mc._lib.mlem_workspace_bytes(0, 50) == 0
    args = lambda nb, nv, nnz, ws: (nb, nv, nnz, 8, 8, 8, 8, 8, 8, 8, 8, 3, 8, ws, None)
    assert ml(*args(100, 50, -1, wsb)) == mc.MC_EINVAL
    assert ml(*args(0, 50, 10, wsb)) == mc.MC_EINVAL
    assert ml(*args(100, 1 << 31, 10, wsb)) == mc.MC_EINVAL
    assert ml(*args(100, 50, 10, wsb - 1)) == mc.MC_ENOMEM
    best = C.c_int32(7)
    assert mc._lib.mc_autotune(C.byref(p), 1, None, 1, 1, 8, 8, 8, 8, need, None, C.byref(best),
                               None) == mc.MC_EINVAL
    assert mc._lib.mc_autotune(C.byref(p), 1, C.byref(o), 0, 1, 8, 8, 8, 8, need, None, C.byref(best),
                               None) == mc.MC_EINVAL
    assert sim(None, 1, None, 8, None, 8, None, None, None, 0, None, 8, 8, need, None) == mc.MC_EINVAL
    assert mc._lib.mc_error_string(mc.MC_EINVAL) == b"invalid argument"
    assert mc._lib.mc_replay_histories(C.byref(p), None, None, None, 5, None, 8, 8, need, None) == mc.MC_EINVAL
